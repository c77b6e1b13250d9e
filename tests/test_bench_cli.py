"""The benchmark's command-line contract, on the CPU: more than one GPU is
refused with a message, the options are listed, and the measured HBM traffic
of a kernel class is reported only for the kernel source it was measured on."""
import hashlib
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_options_are_listed():
    r = subprocess.run([sys.executable, BENCH, "--help"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--precision", "--no-cpu-baseline", "--no-extras",
                "--no-inclusions", "--inclusion-iterations"):
        assert opt in r.stdout, opt


def test_measured_traffic_follows_the_kernel_source():
    import bench   # the repository root is on sys.path (conftest)
    key = ("patch_solve", 9, "mixed")
    entry = bench.MEASURED_TRAFFIC[key]
    path = os.path.join(ROOT, "paper_1503_03467_amd", "csrc", entry["source"])
    digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    saved = dict(entry)
    try:
        entry["sha256"] = digest
        assert bench.measured_traffic(*key) == entry["bytes_per_launch"]
        entry["sha256"] = "0" * 64
        assert bench.measured_traffic(*key) is None
        assert bench.measured_traffic("no_such_class", 9, "mixed") is None
    finally:
        entry.clear()
        entry.update(saved)
