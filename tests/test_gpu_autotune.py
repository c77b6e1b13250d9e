"""The build-kernel autotuner (``autotune`` / ``autotune_path`` of gbl_opts):
every level records a choice, a second build with the same table reuses it
and gives the same bits, a table read from a file is obeyed, and autotuned
hierarchies keep the parity bounds (FP64 levels against the oracle at 1e-10,
mixed solves against the direct solve at 1e-8)."""
import numpy as np
import pytest

import synthetic as S
from oracle import fem
from oracle import gamblets as G
from tests.gpu_layout import restriction_to_matrix, stencil_to_matrix

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    import paper_1503_03467_amd as P
    return P


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_autotune_records_reuses_and_obeys_a_table(tmp_path):
    P = _P()
    q = 8
    print("CASE test=autotune q=8 mixed", flush=True)
    pr = S.rough_problem(q, 2.0, 41)
    a, g = _dev(pr.a), _dev(pr.g[0])
    path = str(tmp_path / "tune.txt")
    H1 = P.Hierarchy(a, rho=3, precision="mixed", autotune=True, autotune_path=path)
    lines = open(path).read().split("\n")
    lines = [x for x in lines if x]
    assert len(lines) == 2 * (q - 1), lines            # one patch and one Galerkin choice per transition
    assert all(x.split()[0].startswith("gfx") and ":f32:" in x for x in lines)
    choices = {k: (H1.level(k)["patch_kernel"], H1.level(k)["galerkin_kernel"]) for k in range(2, q + 1)}
    assert all(v in (0, 1) for c in choices.values() for v in c), choices
    print("choices per level", choices, flush=True)
    u1 = H1.solve(g)
    ref = fem.solve(pr.a, pr.g[0])
    assert _rel(u1.cpu().numpy()[1:-1, 1:-1], ref[1:-1, 1:-1]) < 1e-8
    # same table: same choices, same bits
    H2 = P.Hierarchy(a, rho=3, precision="mixed", autotune=True, autotune_path=path)
    assert len([x for x in open(path).read().split("\n") if x]) == len(lines)
    for k in range(2, q + 1):
        l1, l2 = H1.level(k), H2.level(k)
        assert (l2["patch_kernel"], l2["galerkin_kernel"]) == choices[k]
        assert torch.equal(l1["R"], l2["R"]) and torch.equal(l1["A"], l2["A"])
    assert torch.equal(H2.solve(g), u1)
    # a table with every applicable choice flipped, read from a file
    flipped = tmp_path / "flipped.txt"
    with open(flipped, "w") as f:
        for x in lines:
            key, ch, t0, t1 = x.split()
            other = 1 - int(ch)
            if float((t0, t1)[other]) >= 0:   # the other candidate applies here
                f.write(f"{key} {other} {t0} {t1}\n")
            else:
                f.write(x + "\n")
    H3 = P.Hierarchy(a, rho=3, precision="mixed", autotune=True, autotune_path=str(flipped))
    want = {}
    for x in open(flipped).read().split("\n"):
        if x:
            key, ch = x.split()[:2]
            want[key] = int(ch)
    for k in range(2, q + 1):
        lv = H3.level(k)
        assert lv["patch_kernel"] in (0, 1) and lv["galerkin_kernel"] in (0, 1)
    n_flipped = sum(1 for k in range(2, q + 1) for i in range(2) if
                    (H3.level(k)["patch_kernel"], H3.level(k)["galerkin_kernel"])[i] != choices[k][i])
    assert n_flipped >= 1
    assert _rel(H3.solve(g).cpu().numpy()[1:-1, 1:-1], ref[1:-1, 1:-1]) < 1e-8
    for H in (H1, H2, H3):
        H.close()


def test_autotuned_fp64_levels_match_oracle():
    P = _P()
    q, rho = 6, 3
    print("CASE test=autotune_fp64 q=6", flush=True)
    pr = S.rough_problem(q, 1.0, 42)
    fe = fem.assemble(pr.a)
    tree = G.Tree(q)
    h = G.localized_hierarchy(fe.A, tree, rho)
    H = P.Hierarchy(_dev(pr.a), rho=rho, precision="fp64", autotune=True)
    for k in range(q, 0, -1):
        lv = H.level(k)
        A = stencil_to_matrix(lv["A"].cpu().numpy(), q, k, tree.size(k))
        Ar = h.levels[k].A
        assert abs(A - Ar).max() <= 1e-10 * abs(Ar).max(), k
        if k >= 2:
            assert lv["patch_kernel"] in (0, 1) and lv["galerkin_kernel"] in (0, 1)
            R = restriction_to_matrix(lv["R"].cpu().numpy(), lv["rho"], q, k, tree.size(k))
            assert abs(R - h.levels[k].R).max() <= 1e-10 * abs(h.levels[k].R).max(), k
    u = H.solve(_dev(pr.g[0])).cpu().numpy()
    ref = fem.solve(pr.a, pr.g[0])
    assert _rel(u[1:-1, 1:-1], ref[1:-1, 1:-1]) < 1e-10
    H.close()
