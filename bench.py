#!/usr/bin/env python3
"""Throughput of the gamblet hierarchy build + solve on one MI355X.

One step = one pass of the whole hot path on the 512 x 512-cell rough
problem (q = 9, 261,121 interior DOF, lognormal product coefficient with
sigma = 2, N(0,1) cell source, patch radius 3): build the localized
hierarchy from the coefficient (assembly, subband operators, patch solves,
restrictions, Galerkin coarsening) and solve to a relative error of 1e-8
(flexible CG on the FP64 fine residual, subband solves in FP32).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

The timed line is the rough 512 x 512-cell workload: a step of the
2048 x 2048-cell inclusion workload (16 right-hand sides, discs of a = 1e6)
takes minutes (its outer iteration needs over a thousand iterations at patch
radius 4), so it is measured once, as the extra "inclusion_workload_q11"
(build, the 16 right-hand sides as one block, the adjoint gradient), next to
the other workloads.

Besides the timed steps the line carries: the roofline figure of the
dominant build kernel (HIP events in the timed region, HBM traffic from
counters taken on the same kernel source), the CPU oracle's direct solve as
the baseline (and as the error reference), and unless --no-extras: the FP64
path, the adjoint gradient, patch radii 1-4 and a smaller radius below the
finest transition, the hierarchy on the level-q gamblets of the localized
mass inverse and its level-q operator, the 1024 x 1024-cell adjoint workload,
a 32-problem sample of the batch workload, and the gamblet transform with
compression.

    python bench.py [--steps K] [--warmup W] [--precision mixed|fp64] [--no-cpu-baseline] [--no-extras]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VALU_FMA_PEAK_TFLOPS = 78.6    # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP64 or unpacked FP32 FMA); FP64 matrix cores too
MFMA_F32_PEAK_TFLOPS = 157.3   # dense FP32 matrix-core peak
# single-kernel build classes (one launch per level, a definite algorithmic
# amount of work); the solve-phase classes are mixtures of small launches, and
# bracketing them with events would also replace the replayed iteration graph
# by kernel-by-kernel launches inside the timed steps
ROOFLINE_CLASSES = ("patch_solve", "patch_band", "galerkin", "subband_operator")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--inner", choices=["chebyshev", "cg"], default="chebyshev",
                    help="iteration on the subband systems (library default: chebyshev)")
    ap.add_argument("--inner-iters", type=int, default=None, help="finest-level budget (default: library's)")
    ap.add_argument("--inner-iters-coarse", type=int, default=None, help="coarser-level budget (default: library's)")
    ap.add_argument("--kappa", type=float, default=None, help="Chebyshev interval ratio, finest level")
    ap.add_argument("--kappa-coarse", type=float, default=None, help="Chebyshev interval ratio, coarser levels")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FP64-path and adjoint measurements")
    ap.add_argument("--no-inclusions", action="store_true", help="skip the 2048 x 2048-cell inclusion workload")
    ap.add_argument("--inclusion-iterations", type=int, default=0,
                    help="only run K outer iterations of the inclusion workload's 16-right-hand-side block "
                         "(for kernel profiles) and print their time")
    return ap.parse_args()


def level_geometry(H):
    return {k: H.level(k) for k in range(1, H.q + 1)}


# HBM traffic per launch of a kernel class, from rocprofv3 counter runs of this benchmark
# (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, averaged over the class's launches of one step,
# scaled by the factors measured on a plain 1 GiB copy).  Valid only for the kernel source it was
# measured on: the entry records the SHA-256 of that source file, and a mismatch reports None.
MEASURED_TRAFFIC = {
    # matrix-core patch solves, levels 8..2 of the 512x512-cell benchmark (parent-major copy of B^(k),
    # then the patch kernel): 104,893 KiB fetched and 96,059 KiB written per build over 7 launches
    # (FETCH x 2.0 + WRITE x 1.0); profiles/q9_kernels_hbm_fraction_and_mfma.md
    ("patch_solve", 9, "mixed"): {
        "bytes_per_launch": 44740763,
        "source": "kernels_build.hip",
        "sha256": "b28678d5f313c0d07e67c2b30ba4ab038afaa0e9159bff33c6c5f73654f1027c",
    },
    # band patch solves of the finest transition (one launch per build): 16,069 KiB fetched, 80,491 KiB
    # written (R of the 65,536 coarse cells with its write amplification); same profile
    ("patch_band", 9, "mixed"): {
        "bytes_per_launch": 115331744,
        "source": "kernels_build.hip",
        "sha256": "b28678d5f313c0d07e67c2b30ba4ab038afaa0e9159bff33c6c5f73654f1027c",
    },
}


def measured_traffic(name, q, precision):
    import hashlib
    e = MEASURED_TRAFFIC.get((name, q, precision))
    if not e:
        return None
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1503_03467_amd", "csrc", e["source"])
    try:
        digest = hashlib.sha256(open(path, "rb").read()).hexdigest()
    except OSError:
        return None
    return e["bytes_per_launch"] if digest == e["sha256"] else None


def kernel_work(name, geo, q, elem, inner="chebyshev"):
    """Algorithmic bytes (HBM-bound classes) or flops (arithmetic-bound) summed over one
    build (build kernels) or one launch (solve kernels).  Returns (kind, amount)."""
    if name in ("patch_solve", "patch_band"):
        # dense Cholesky plus two triangular solves, p^3 / 3 + 2 p^2 per patch (levels k < q); at the
        # finest transition the band Cholesky, p (bw^2 + 4 bw) with half-bandwidth bw = 3 (w_y + 1) + 2
        import numpy as np
        fl = 0.0
        levels = [q] if name == "patch_band" else range(2, q)
        for k in levels:
            g = geo[k]
            nc = g["nk"] // 2
            rho = g["rho"]
            w = np.minimum(np.arange(nc) + rho, nc - 1) - np.maximum(np.arange(nc) - rho, 0) + 1
            p = 3.0 * np.outer(w, w)
            if name == "patch_band":
                bw = 3.0 * (w[None, :] + 1) + 2
                fl += float((p * (bw ** 2 + 4 * bw)).sum())
            else:
                fl += float((p ** 3 / 3.0 + 2.0 * p ** 2).sum())
        return "flops", fl
    if name == "galerkin":
        fl = 0.0
        for k in range(2, q + 1):
            g, c = geo[k], geo[k - 1]
            nc = g["nk"] // 2
            Sk = 2 * g["s"] + 1
            Sc = 2 * c["s"] + 1
            fl += 2.0 * nc * nc * g["rw"] ** 2 * (Sk * Sk + Sc * Sc)
        return "flops", fl
    if name == "fine_cg":
        np2 = (geo[q]["nk"] // 2) ** 2
        if inner == "chebyshev":
            # per parent and launch (several fused steps): r, d, x, block-Jacobi 3x3 and 4 cell
            # coefficients read once; r, d, x written once
            return "bytes", elem * np2 * (9 + 9 + 4 + 9)
        # per parent: r, w, s, u, p, x, block-Jacobi 3x3 and 4 cell coefficients read;
        # u, p, x, r, s, w written (one fused iteration of the finest subband CG)
        return "bytes", elem * np2 * (9 + 9 + 9 + 4 + 18)
    if name in ("cg_spmv", "cg_update", "cg_init"):
        by = 0.0
        for k in range(2, q):
            g = geo[k]
            np2 = (g["nk"] // 2) ** 2
            T = 2 * g["t"] + 1
            if name == "cg_spmv" and inner == "chebyshev":
                # B blocks, d once, r read + written, block-Jacobi, d_new and x
                by += elem * np2 * (9 * T * T + 3 + 6 + 9 + 3 + 6)
            elif name == "cg_spmv":
                # B blocks, z once, q and p read + written
                by += elem * np2 * (9 * T * T + 3 + 12)
            elif name == "cg_update":
                # x rw, p, r rw, q, BJ, z written
                by += elem * np2 * (6 + 3 + 6 + 3 + 9 + 3)
            else:
                by += elem * np2 * (4 + 9 + 15)
        return "bytes", by
    if name in ("restrict", "prolong"):
        by = 0.0
        for k in range(2, q + 1):
            g = geo[k]
            nc2 = (g["nk"] // 2) ** 2
            nk2 = g["nk"] ** 2
            by += elem * (g["rw"] ** 2 * nc2 + nk2 + nc2 + (3 * nc2 if name == "prolong" else 0))
        return "bytes", by
    if name == "fine_apply":
        n2 = geo[q]["nk"] ** 2
        return "bytes", 8.0 * 3 * n2
    if name == "subband_operator":
        by = 0.0
        for k in range(2, q + 1):
            g = geo[k]
            S = 2 * g["s"] + 1
            T = 2 * g["t"] + 1
            by += elem * (S * S * g["nk"] ** 2 + (9 * T * T + 9) * (g["nk"] // 2) ** 2)
        return "bytes", by
    return "bytes", 0.0


def host_info():
    """CPU model, usable cores and BLAS threads of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = None
    try:
        from threadpoolctl import threadpool_info
        blas = max((d.get("num_threads", 0) for d in threadpool_info() if d.get("user_api") == "blas"), default=None)
    except Exception:
        pass
    return {"cpu_model": model, "cores_usable": len(os.sched_getaffinity(0)), "blas_threads": blas}


def superlu_leg(a, g):
    """The oracle's direct solve (Q1 assembly, SuperLU factor, solves with two
    FP64 refinement steps; single-threaded) of one problem and its right-hand
    sides ([nrhs][n][n]), timed on the host.  Returns the record and the solutions."""
    from oracle import fem
    t0 = time.perf_counter()
    fe = fem.assemble(a)
    b = fem.load_cellwise(g, fe.h)
    ds = fem.DirectSolver(fe.A)
    t1 = time.perf_counter()
    u = ds.solve(b)
    t2 = time.perf_counter()
    nrhs = g.shape[0] if g.ndim == 3 else 1
    dof = fe.A.shape[0]
    return {"dof": dof, "rhs": nrhs, "factor_s": t1 - t0, "solve_s": t2 - t1,
            "dof_per_s": dof * nrhs / (t2 - t0), "threads": 1, "kind": "oracle (SuperLU)"}, u


def oracle_localized_leg(S):
    """The oracle's localized hierarchy (Algorithm 2, patch radius 3) and its
    solve with refinement to 1e-10, numpy/scipy with BLAS on every core, on a
    bounded sample: the 128 x 128-cell problem of the rough recipe (sigma = 2)."""
    from oracle import fem
    from oracle import gamblets as G
    pr = S.rough_problem(7, 2.0, S.TAG_Q9_ROUGH)
    t0 = time.perf_counter()
    fe = fem.assemble(pr.a)
    h = G.localized_hierarchy(fe.A, G.Tree(7), 3)
    t1 = time.perf_counter()
    _, sweeps, _ = G.refine_solve(h, fe.A, fem.load_cellwise(pr.g[0], fe.h), tol=1e-10)
    t2 = time.perf_counter()
    return {"sample": "128x128-cell rough problem (sigma=2), radius 3", "dof": pr.dof, "build_s": t1 - t0,
            "solve_s": t2 - t1, "refinement_sweeps": sweeps, "dof_per_s": pr.dof / (t2 - t0),
            "kind": "oracle (numpy, localized build + refined solve)", **host_info()}


def exact_workloads(P, S, torch, dev):
    """The exact hierarchy (Algorithm 1, dense FP64) on its two 64 x 64-scale
    workloads: the 64 x 64-cell lognormal product field (sigma = 1) with g = 1,
    and Example 5.1 (65 x 65 cells, K = 6, nodal source).  Build and solve
    timed apart (minimum of three), error against the oracle's direct solve,
    and the energy error of the solution compressed in the normalized exact
    basis; the oracle's own dense exact hierarchy timed beside it."""
    import numpy as np
    from oracle import fem
    from oracle import gamblets as G
    print("# exact hierarchy workloads", file=sys.stderr, flush=True)
    out = {}
    pr = S.q6_exact_problem()
    cases = {"q6_lognormal_g1": (pr.a, pr.g[0], 0, "cell"),
             "example_5_1": (S.example51_coefficient(), S.example51_nodal_source(), 1, "nodal")}
    for name, (a_np, g_np, geometry, source) in cases.items():
        a = torch.as_tensor(a_np, device=dev)
        g = torch.as_tensor(g_np, device=dev)
        fe = fem.assemble(a_np)
        b = fem.load_nodal(g_np, fe.h) if source == "nodal" else fem.load_cellwise(g_np, fe.h)
        u_ref = fem.DirectSolver(fe.A).solve(b)
        best_b, best_s = float("inf"), float("inf")
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = P.Hierarchy(a, exact=True, geometry=geometry, source=source)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            u = H.solve(g)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            best_b, best_s = min(best_b, (t1 - t0) * 1e3), min(best_s, (t2 - t1) * 1e3)
            if _ < 2:
                H.close()
        err = float(np.linalg.norm(u.cpu().numpy().ravel()[fe.interior] - u_ref) / np.linalg.norm(u_ref))
        nrm = H.energy_norm(u)
        total = H.transform_size()
        comp = {}
        for frac in (0.01, 0.05, 0.25):
            c = H.transform(u)
            H.compress(c, int(round(frac * total)))
            comp[f"{frac:g}"] = H.energy_norm(u - H.inverse_transform(c)) / nrm
        H.close()
        tc = time.perf_counter()
        G.exact_hierarchy(fe.A, G.Tree(6, offset=geometry))
        cpu_s = time.perf_counter() - tc
        out[name] = {"dof": fe.A.shape[0], "build_ms": best_b, "solve_ms": best_s,
                     "rel_err_vs_direct": err, "energy_err_vs_kept_fraction": comp,
                     "oracle_exact_hierarchy_s": cpu_s, **host_info()}
    # the problem on the unit cube: 16^3 cells, lognormal coefficient (sigma = 1), N(0,1) cell source
    from oracle import fem3d
    n = 16
    a3 = np.exp(S.rng(S.TAG_Q6_EXACT, 0, 7).standard_normal((n, n, n)))
    g3 = S.rng(S.TAG_Q6_EXACT, 0, 8).standard_normal((n, n, n))
    fe3 = fem3d.assemble(a3)
    u3_ref = fem.DirectSolver(fe3.A).solve(fem3d.load_cellwise(g3, fe3.h))
    ad, gd = torch.as_tensor(a3, device=dev), torch.as_tensor(g3, device=dev)
    best_b, best_s = float("inf"), float("inf")
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        H = P.Hierarchy(ad, exact=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        u3 = H.solve(gd)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        H.close()
        best_b, best_s = min(best_b, (t1 - t0) * 1e3), min(best_s, (t2 - t1) * 1e3)
    err3 = float(np.linalg.norm(u3.cpu().numpy().ravel()[fe3.interior] - u3_ref) / np.linalg.norm(u3_ref))
    out["cube_16_lognormal"] = {"dof": fe3.A.shape[0], "build_ms": best_b, "solve_ms": best_s,
                                "rel_err_vs_direct": err3}
    return out


def cpu_baseline(pr, dof):
    """The oracle (Q1 assembly, SuperLU factor and solve, two FP64 refinement
    steps; single-threaded) on the full benchmark problem, repeated for about
    10 s of host time.  Returns the baseline record and the oracle's solution."""
    from oracle import fem
    print("# cpu baseline (oracle direct solve)", file=sys.stderr, flush=True)
    reps, spent, t_sum, u_ref = 0, 0.0, 0.0, None
    while spent < 10.0 and reps < 8:
        tt = time.perf_counter()
        fe = fem.assemble(pr.a)
        b = fem.load_cellwise(pr.g[0], fe.h)
        u_ref = fem.DirectSolver(fe.A).solve(b)
        d = time.perf_counter() - tt
        t_sum += d
        spent += d
        reps += 1
    hi = host_info()
    cpu = {"value": dof / (t_sum / reps), "unit": "DOF/s", "cores": 1, "kind": "oracle",
           "sample": f"full 512x512-cell problem, {reps} repetitions: Q1 assembly + SuperLU factor/solve + "
                     f"2 FP64 refinement steps (single-threaded); host has {hi['cores_usable']} cores",
           "cpu_model": hi["cpu_model"]}
    return cpu, u_ref


INCLUSION_SETTINGS = dict(precision="mixed-fp64-build", rtol=1e-8, max_outer=6000, inner="cheb-cg", inner_iters=8,
                          inner_iters_coarse=16, window_tol=1000.0)


def inclusion_iterations(P, S, torch, dev, k):
    """k outer iterations of the inclusion workload's 16-right-hand-side block
    (the build and the solve settings of the full workload; for profiles)."""
    pr = S.inclusion_problem(q=11, nrhs=16, a_incl=1e6)
    a = torch.as_tensor(pr.a, device=dev)
    g = torch.as_tensor(pr.g, device=dev)
    kw = dict(INCLUSION_SETTINGS, max_outer=k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = P.Hierarchy(a, rho=4, max_rhs=16, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    H.solve(g, check=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    its = H.last_info.outer_iters
    H.close()
    print(json.dumps({"workload": "inclusion block, 16 right-hand sides", "build_ms": (t1 - t0) * 1e3,
                      "outer_iters": its, "ms_per_outer_iter": (t2 - t1) * 1e3 / max(1, its)}), flush=True)


def inclusion_workload(P, S, torch, dev, cpu_leg=True):
    """The 2048 x 2048-cell inclusion workload (discs of a = 1e6 on 10% of the
    cells over the product field, 16 N(0,1) right-hand sides, patch radius 4),
    one pass: FP64-built hierarchy with window corrections, the 16 right-hand
    sides as one block (FP32 subband iterations: 8 Chebyshev steps on the
    finest level, 16 CG iterations below; FP64 outer iteration to 1e-8), and
    the adjoint gradient of J = |u_0|^2 / 2 (the first right-hand side's
    solution).  Also the outer iterations of one right-hand side with radius 5
    at the finest transition.  Error figures against the direct solve are in
    the GPU tests (the direct solve of this size takes minutes on the host)."""
    print("# inclusion workload, 2048 x 2048 cells", file=sys.stderr, flush=True)
    os.environ["GBL_PROGRESS"] = "1"   # the library reports its outer iterations on stderr every 15 s
    pr = S.inclusion_problem(q=11, nrhs=16, a_incl=1e6)
    a = torch.as_tensor(pr.a, device=dev)
    g = torch.as_tensor(pr.g, device=dev)
    kw = dict(INCLUSION_SETTINGS)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = P.Hierarchy(a, rho=4, max_rhs=16, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("# inclusion workload: built, solving 16 right-hand sides", file=sys.stderr, flush=True)
    u = H.solve(g, check=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = H.last_info
    print("# inclusion workload: solved, adjoint", file=sys.stderr, flush=True)
    u0 = u[:1].contiguous()
    H.adjoint(u0, u0, check=False)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ainfo = H.last_info
    wins = {str(k): H.level(k)["nwin"] for k in range(3, 11)}
    H.close()
    del u, u0
    dof = ((1 << 11) - 1) ** 2
    out = {"dof": dof, "rhs": 16, "rho": 4, "build_ms": (t1 - t0) * 1e3, "solve_16rhs_ms": (t2 - t1) * 1e3,
           "adjoint_grad_ms": (t3 - t2) * 1e3, "outer_iters": info.outer_iters, "status": info.status,
           "rel_update": info.rel_update, "adjoint_outer_iters": ainfo.outer_iters,
           "build_solve_dof_per_s": dof * 16 / (t2 - t0), "windows_per_level": wins,
           "settings": {k: v for k, v in kw.items()}}
    # radius 5 at the finest transition (the paper sizes radii like ln(1/H_k)), one right-hand side
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = P.Hierarchy(a, rho=5, rho_coarse=4, max_rhs=1, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    H.solve(g[0], check=False)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    out["finest_radius_5_one_rhs"] = {"build_ms": (t1 - t0) * 1e3, "solve_ms": (t2 - t1) * 1e3,
                                      "outer_iters": H.last_info.outer_iters}
    H.close()
    os.environ.pop("GBL_PROGRESS", None)
    if cpu_leg:
        print("# inclusion workload: oracle direct solve of the 16 right-hand sides on the host", file=sys.stderr,
              flush=True)
        out["cpu_superlu"], _ = superlu_leg(pr.a, pr.g)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1503_03467_amd as P
    import synthetic as S

    dev = torch.device("cuda:0")
    if args.inclusion_iterations > 0:
        inclusion_iterations(P, S, torch, dev, args.inclusion_iterations)
        return
    pr = S.q9_rough_problem()
    q, dof = pr.q, pr.dof
    a = torch.as_tensor(pr.a, device=dev)
    g = torch.as_tensor(pr.g[0], device=dev)
    torch.cuda.synchronize()

    def step(prec):
        H = P.Hierarchy(a, rho=pr.rho, precision=prec, rtol=args.rtol, inner_iters=args.inner_iters,
                        inner_iters_coarse=args.inner_iters_coarse, inner=args.inner, kappa=args.kappa,
                        kappa_coarse=args.kappa_coarse)
        u = H.solve(g, check=False)
        info = H.last_info
        return H, u, info

    print(f"# warmup {args.warmup} steps", file=sys.stderr, flush=True)
    # first warm-up steps with every kernel class timed, to find the dominant one
    # (timing the iteration classes launches the iterations kernel by kernel);
    # several steps, since the two patch classes take about the same time
    n_prof = max(1, min(3, args.warmup - 1))
    P.profile_reset()
    P.profile_enable("all")
    for _ in range(n_prof):
        H, u, info = step(args.precision)
        geo = level_geometry(H)
        H.close()
    torch.cuda.synchronize()
    prof_all = {k: (v[0] / n_prof, v[1] / n_prof) for k, v in P.profile_read().items()}
    P.profile_enable(None)
    P.profile_reset()
    # the other warm-up steps as timed, so that the replayed iteration graph is
    # set up before the timed region
    for _ in range(max(1, args.warmup - n_prof)):
        H, u, info = step(args.precision)
        H.close()
    torch.cuda.synchronize()
    dominant = max((k for k in prof_all if k in ROOFLINE_CLASSES), key=lambda k: prof_all[k][0])

    # timed region: only the dominant class is bracketed by events
    P.profile_enable([dominant])
    print(f"# timed {args.steps} steps (events on {dominant})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    marks = [t0]
    for _ in range(args.steps):
        H, u, info = step(args.precision)
        infos.append(info)
        H.close()
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print("# step wall times (ms, host clock; a solve ends with a host read of its status): "
          + " ".join("%.3f" % ((b - a) * 1e3) for a, b in zip(marks, marks[1:])), file=sys.stderr, flush=True)
    P.profile_enable(None)
    bad = [(i, inf.status) for i, inf in enumerate(infos) if inf.status != 0]
    if bad:
        print(f"timed steps did not converge (step, status): {bad}", file=sys.stderr, flush=True)
        sys.exit(1)
    dom_ms, dom_launches = P.profile_read()[dominant]
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = dof / (ms_per_step * 1e-3)

    elem = 4 if args.precision == "mixed" else 8
    kind, work = kernel_work(dominant, geo, q, elem, args.inner)
    inner_iters = H.opts.inner_iters
    inner_iters_coarse = H.opts.inner_iters_coarse
    # work is per build (build kernels: one launch per level) or per launch (solve kernels)
    build_kernel = dominant in ("patch_solve", "patch_band", "galerkin", "subband_operator", "assemble")
    launches_per_step = dom_launches / args.steps
    per_launch_work = work / launches_per_step if build_kernel else work
    avg_launch_ms = dom_ms / max(dom_launches, 1)
    if kind == "flops":
        achieved = per_launch_work / (avg_launch_ms * 1e-3) / 1e12
        # the patch solves below the finest level run on the matrix cores (FP32 in the mixed
        # path, FP64 in the FP64 path, whose dense peak equals the FP64 vector peak)
        mfma = dominant == "patch_solve" and os.environ.get("GBL_PATCH_MFMA", "1") != "0"
        peak = MFMA_F32_PEAK_TFLOPS if (mfma and args.precision == "mixed") else VALU_FMA_PEAK_TFLOPS
        roof = {"bound": "mfma" if mfma else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": None}
    else:
        achieved = per_launch_work / (avg_launch_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None}
    roof.update({"kernel": dominant, "avg_launch_ms": avg_launch_ms, "launches_per_step": launches_per_step,
                 "algorithmic_per_launch": per_launch_work})
    roof["traffic"] = measured_traffic(dominant, q, args.precision)

    # CPU baseline leg: the oracle's direct solve of the same problem, timed on
    # the host; its solution is also the reference for the error figures
    extras = {}
    cpu, u_ref = (None, None) if args.no_cpu_baseline else cpu_baseline(pr, dof)

    def rel_err(u_gpu):
        if u_ref is None:
            return None
        return float(np.linalg.norm(u_gpu.cpu().numpy()[1:-1, 1:-1].ravel() - u_ref) / np.linalg.norm(u_ref))

    extras["rel_err_vs_oracle"] = rel_err(u)
    extras["outer_iters"] = max(i.outer_iters for i in infos)
    extras["profile_warmup_ms_per_step"] = {k: v[0] for k, v in prof_all.items() if v[1]}   # mean of the profiled steps

    if not args.no_extras:
        # plain FP64 GPU path at the same accuracy
        print("# fp64 path", file=sys.stderr, flush=True)
        H, u64, _ = step("fp64")
        H.close()
        torch.cuda.synchronize()
        tt = time.perf_counter()
        n64 = 2
        for _ in range(n64):
            H, u64, info64 = step("fp64")
            H.close()
        torch.cuda.synchronize()
        extras["fp64_ms_per_step"] = (time.perf_counter() - tt) * 1e3 / n64
        extras["fp64_rel_err_vs_oracle"] = rel_err(u64)
        extras["mixed_speedup_vs_fp64"] = extras["fp64_ms_per_step"] / ms_per_step
        # adjoint gradient of J = 1/2 |u - u_obs|^2 through the same hierarchy
        print("# adjoint", file=sys.stderr, flush=True)
        a_obs = torch.as_tensor(S.product_field(pr.n) * S.lognormal_factor(pr.n, 1.0, S.rng(pr.tag, 0, S.KIND_OBS)),
                                device=dev)
        Hobs = P.Hierarchy(a_obs, rho=pr.rho, precision="mixed", rtol=args.rtol)
        u_obs = Hobs.solve(g)
        Hobs.close()
        H, u, _ = step(args.precision)
        dJdu = (u - u_obs).contiguous()
        H.adjoint(u, dJdu, check=False)
        torch.cuda.synchronize()
        tt = time.perf_counter()
        nadj = 3
        for _ in range(nadj):
            H.adjoint(u, dJdu, check=False)
        torch.cuda.synchronize()
        extras["adjoint_grad_ms"] = (time.perf_counter() - tt) * 1e3 / nadj
        H.close()
        # patch radius against outer iterations: gamblets with a smaller radius
        # as the preconditioner of the FP64 flexible CG (build and solve timed
        # apart, the minimum of three runs each)
        print("# patch radius trade-off", file=sys.stderr, flush=True)
        trade = {}
        for prec in ("mixed", "fp64"):
            for rho in (1, 2, 3, 4):
                best_b, best_s = float("inf"), float("inf")
                for _ in range(3):
                    torch.cuda.synchronize()
                    tb = time.perf_counter()
                    Hr = P.Hierarchy(a, rho=rho, precision=prec, rtol=args.rtol if prec == "mixed" else 1e-10,
                                     max_outer=2000)
                    torch.cuda.synchronize()
                    ts = time.perf_counter()
                    ur = Hr.solve(g, check=False)
                    torch.cuda.synchronize()
                    te = time.perf_counter()
                    info_r = Hr.last_info
                    Hr.close()
                    best_b, best_s = min(best_b, (ts - tb) * 1e3), min(best_s, (te - ts) * 1e3)
                err_r = rel_err(ur)
                trade[f"{prec}_rho{rho}"] = {"build_ms": best_b, "solve_ms": best_s, "total_ms": best_b + best_s,
                                             "outer_iters": info_r.outer_iters, "rel_err_vs_oracle": err_r}
        # a radius per level: 3 at the finest transition, smaller below it
        for rho_c in (2, 1):
            best_b, best_s = float("inf"), float("inf")
            for _ in range(3):
                torch.cuda.synchronize()
                tb = time.perf_counter()
                Hr = P.Hierarchy(a, rho=3, precision=args.precision, rtol=args.rtol, max_outer=2000, rho_coarse=rho_c)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                ur = Hr.solve(g, check=False)
                torch.cuda.synchronize()
                te = time.perf_counter()
                info_r = Hr.last_info
                Hr.close()
                best_b, best_s = min(best_b, (ts - tb) * 1e3), min(best_s, (te - ts) * 1e3)
            trade[f"{args.precision}_rho3_coarse{rho_c}"] = {"build_ms": best_b, "solve_ms": best_s,
                                                             "total_ms": best_b + best_s,
                                                             "outer_iters": info_r.outer_iters,
                                                             "rel_err_vs_oracle": rel_err(ur)}
        extras["patch_radius_tradeoff"] = trade
        # the hierarchy started from the level-q gamblets of the localized mass
        # inverse (patch radius rho_q node steps) instead of the nodal basis
        print("# hierarchy from the mass-inverse level-q gamblets", file=sys.stderr, flush=True)
        mass = {}
        for rho_q in (1, 3):
            best_b, best_s = float("inf"), float("inf")
            for _ in range(3):
                torch.cuda.synchronize()
                tb = time.perf_counter()
                Hm = P.Hierarchy(a, rho=pr.rho, precision=args.precision, rtol=args.rtol, max_outer=400,
                                 level_q_mass=rho_q)
                torch.cuda.synchronize()
                ts = time.perf_counter()
                um = Hm.solve(g, check=False)
                torch.cuda.synchronize()
                te = time.perf_counter()
                info_m = Hm.last_info
                Hm.close()
                best_b, best_s = min(best_b, (ts - tb) * 1e3), min(best_s, (te - ts) * 1e3)
            mass[f"rho_q{rho_q}"] = {"build_ms": best_b, "solve_ms": best_s, "total_ms": best_b + best_s,
                                     "outer_iters": info_m.outer_iters, "rel_err_vs_oracle": rel_err(um)}
        extras["level_q_mass_hierarchy"] = mass
        # level-q gamblets from the localized mass inverse (radius 3): the
        # table of 1-D factors, the level-q operator and load
        print("# level-q gamblets (localized mass inverse)", file=sys.stderr, flush=True)
        lq = P.LevelQ(q, 3)
        # any interior vector times the load map: the cell source, cut to the interior nodes
        bq = torch.as_tensor(pr.g[0][1:, 1:].ravel().copy(), device=dev)
        w1, w2 = lq.operator(a), lq.operator(a)   # two output blocks cached by the allocator
        del w1, w2
        torch.cuda.synchronize()

        def event_ms(fn, reps=5):
            # the library launches on torch's current stream, where the events are recorded
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                out = fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / reps, out

        t_table, _ = event_ms(lambda: P.LevelQ(q, 3))
        t_op, aq = event_ms(lambda: lq.operator(a))
        t_load, _ = event_ms(lambda: lq.load(bq))
        op_bytes = aq.numel() * 8 + pr.n * pr.n * 8
        extras["level_q_mass_inverse"] = {"rho_q": 3, "table_ms": t_table, "operator_ms": t_op, "load_ms": t_load,
                                          "operator_bytes": op_bytes,
                                          "operator_GBps": op_bytes / (t_op * 1e-3) / 1e9,
                                          "operator_hbm_frac": op_bytes / (t_op * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del aq
        # the adjoint workload (1024 x 1024 cells, sigma = 1, J = |u - u_obs|^2 / 2):
        # build, solve and adjoint gradient timed apart (minimum of two runs)
        print("# adjoint workload, 1024 x 1024 cells", file=sys.stderr, flush=True)
        pa = S.adjoint_problem(q=10)
        a10 = torch.as_tensor(pa.a, device=dev)
        g10 = torch.as_tensor(pa.g[0], device=dev)
        Ho = P.Hierarchy(torch.as_tensor(pa.extra["a_obs"], device=dev), rho=3, precision=args.precision,
                         rtol=args.rtol)
        uo10 = Ho.solve(g10)
        Ho.close()
        best = [float("inf")] * 3
        for _ in range(3):   # the first run sets up the iteration graph
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H10 = P.Hierarchy(a10, rho=3, precision=args.precision, rtol=args.rtol)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            u10 = H10.solve(g10, check=False)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            H10.adjoint(u10, (u10 - uo10).contiguous(), check=False)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            it10 = H10.last_info.outer_iters
            H10.close()
            best = [min(b, v) for b, v in zip(best, ((t1 - t0) * 1e3, (t2 - t1) * 1e3, (t3 - t2) * 1e3))]
        dof10 = ((1 << 10) - 1) ** 2
        extras["adjoint_workload_q10"] = {"dof": dof10, "build_ms": best[0], "solve_ms": best[1],
                                          "adjoint_grad_ms": best[2], "adjoint_outer_iters": it10,
                                          "build_solve_dof_per_s": dof10 / ((best[0] + best[1]) * 1e-3)}
        if not args.no_cpu_baseline:
            print("# adjoint workload: oracle direct solve on the host", file=sys.stderr, flush=True)
            leg, u10_ref = superlu_leg(pa.a, pa.g[:1])
            u10_np = u10.cpu().numpy()[1:-1, 1:-1].ravel()
            extras["adjoint_workload_q10"]["cpu_superlu"] = leg
            extras["adjoint_workload_q10"]["rel_err_vs_direct"] = float(
                np.linalg.norm(u10_np - u10_ref) / np.linalg.norm(u10_ref))
        del a10, g10, uo10, u10
        # batch workload: 256 independent problems of 64 x 64 to 256 x 256
        # cells with 64 right-hand sides each, built and solved concurrently
        # (each problem's 64 right-hand sides as one block)
        print("# batch workload", file=sys.stderr, flush=True)
        probs = S.batch_problems(count=256, nrhs=64)
        coeffs = [torch.as_tensor(pb.a, device=dev) for pb in probs]
        srcs = [torch.as_tensor(pb.g, device=dev) for pb in probs]
        hs = P.build_batched(coeffs[:16], rho=3, precision=args.precision, rtol=args.rtol, max_rhs=64)
        P.solve_batched(hs, srcs[:16], check=False)   # warm-up: streams, graphs
        for h in hs:
            h.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hs = P.build_batched(coeffs, rho=3, precision=args.precision, rtol=args.rtol, max_rhs=64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        P.solve_batched(hs, srcs, check=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        its = [h.last_info.outer_iters for h in hs]
        for h in hs:
            h.close()
        dofs = sum(((1 << pb.q) - 1) ** 2 * 64 for pb in probs)
        extras["batch_workload"] = {"problems": len(probs), "rhs_per_problem": 64, "rhs_block": 64,
                                    "q_counts": {str(qq): sum(1 for pb in probs if pb.q == qq) for qq in (6, 7, 8)},
                                    "build_ms": (t1 - t0) * 1e3, "solve_ms": (t2 - t1) * 1e3,
                                    "build_solve_ms": (t2 - t0) * 1e3, "dof_per_s": dofs / (t2 - t0),
                                    "outer_iters_max": max(its)}
        del coeffs, srcs, hs
        # gamblet transform of a solution, compression by thresholding and the
        # reconstruction (discussion of Example 5.1, Figures 10-11): the smooth
        # source of the example on this grid, and the benchmark's white-noise source
        print("# gamblet transform", file=sys.stderr, flush=True)
        H, u, _ = step(args.precision)
        us = H.solve(torch.as_tensor(S.smooth_cell_source(q), device=dev))
        total = H.transform_size()

        def timed(fn, reps=5):
            # HIP events on torch's current stream (the library's stream); a
            # compression includes its host read of the threshold
            fn()
            torch.cuda.synchronize()
            return event_ms(fn, reps)

        tr = {"coefficients": total}
        tr["transform_ms"], c = timed(lambda: H.transform(us))
        tr["inverse_ms"], _ = timed(lambda: H.inverse_transform(c))
        tr["compress_1pct_ms"], _ = timed(lambda: H.compress(c.clone(), total // 100))
        errs = {}
        for name, uu in (("smooth_source", us), ("white_noise_source", u)):
            nrm = H.energy_norm(uu)
            e = {}
            for frac in (0.01, 0.05, 0.25):
                cc = H.transform(uu)
                H.compress(cc, int(round(frac * total)))
                e[f"{frac:g}"] = H.energy_norm(uu - H.inverse_transform(cc)) / nrm
            errs[name] = e
        tr["energy_err_vs_kept_fraction"] = errs
        extras["gamblet_transform"] = tr
        H.close()

        # the build kernels picked per level by timing (autotune), mixed and FP64:
        # one build fills the table, then build + solve steps as above
        print("# autotuned build kernels", file=sys.stderr, flush=True)
        tuned = {}
        for prec in ("mixed", "fp64"):
            rt = args.rtol if prec == "mixed" else 1e-10
            Ht = P.Hierarchy(a, rho=pr.rho, precision=prec, rtol=rt, autotune=True)
            choices = {str(k): [Ht.level(k)["patch_kernel"], Ht.level(k)["galerkin_kernel"]] for k in range(2, q + 1)}
            Ht.close()
            torch.cuda.synchronize()
            tt = time.perf_counter()
            nt = 5
            for _ in range(nt):
                Ht = P.Hierarchy(a, rho=pr.rho, precision=prec, rtol=rt, autotune=True)
                ut = Ht.solve(g, check=False)
                st_t = Ht.last_info.status
                Ht.close()
            torch.cuda.synchronize()
            tuned[prec] = {"ms_per_step": (time.perf_counter() - tt) * 1e3 / nt, "status": st_t,
                           "rel_err_vs_oracle": rel_err(ut),
                           "choices_per_level_patch_galerkin": choices}
        tuned["default_ms_per_step"] = {"mixed": ms_per_step, "fp64": extras.get("fp64_ms_per_step")}
        extras["autotuned_build"] = tuned
        extras["exact_workloads"] = exact_workloads(P, S, torch, dev)
        if not args.no_cpu_baseline:
            print("# oracle localized build + solve on the host", file=sys.stderr, flush=True)
            extras["cpu_oracle_localized"] = oracle_localized_leg(S)

    if not args.no_inclusions:
        extras["inclusion_workload_q11"] = inclusion_workload(P, S, torch, dev, not args.no_cpu_baseline)

    out = {
        "metric": "DOF/s gamblet build+solve at 1e-8 rel err; adjoint grad time; % HBM roof",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "q9 rough lognormal (sigma=2) product coefficient, 512x512 cells, 261121 DOF, "
                               "N(0,1) cell source, patch radius 3, build+solve to 1e-8",
                   "q": q, "dof": dof, "rho": pr.rho, "sigma": 2.0, "precision": args.precision,
                   "rtol": args.rtol, "inner": args.inner, "inner_iters": inner_iters,
                   "inner_iters_coarse": inner_iters_coarse, "kappa": H.opts.kappa,
                   "kappa_coarse": H.opts.kappa_coarse},
        "roofline": roof,
        "cpu_baseline": cpu,
        **extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
