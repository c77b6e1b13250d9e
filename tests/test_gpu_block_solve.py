"""Several right-hand sides solved together (blocks of up to 64 sharing one
launch per step, each right-hand side in its own copy of the per-solve
workspace region) against the same right-hand sides solved one at a time.

With a fixed number of outer iterations (a target no iteration reaches) the
block solve must reproduce every single solve bit for bit; with the normal
stopping rule every right-hand side must reach the direct solve's accuracy.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import fem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    import paper_1503_03467_amd as P
    return P


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


@pytest.mark.parametrize("precision,inner,q", [("mixed", "chebyshev", 7), ("fp64", "cg", 6),
                                               ("mixed-fp64-build", "cheb-cg", 6)])
def test_block_equals_single_bit_for_bit(precision, inner, q):
    print("CASE test=block_bits", precision, inner, q, flush=True)
    P = _P()
    pr = S.rough_problem(q, 1.0, 31, nrhs=6)
    a = _dev(pr.a)
    g = _dev(pr.g)
    kw = dict(rho=3, precision=precision, rtol=1e-15, max_outer=9, inner=inner)
    if inner != "chebyshev":
        kw.update(inner_iters=8, inner_iters_coarse=4)
    Hb = P.Hierarchy(a, max_rhs=4, **kw)          # blocks of 4 and 2
    ub = Hb.solve(g, check=False)
    assert Hb.last_info.outer_iters == 9
    Hb.close()
    Hs = P.Hierarchy(a, max_rhs=1, **kw)
    for r in range(6):
        us = Hs.solve(g[r], check=False)
        assert torch.equal(us, ub[r]), (r, float((us - ub[r]).abs().max()))
    Hs.close()


@pytest.mark.parametrize("q,nrhs,max_rhs,inner", [(6, 70, 64, "chebyshev"), (6, 70, 64, "cheb-cg"),
                                                  (9, 10, 10, "chebyshev"), (10, 3, 3, "chebyshev"),
                                                  (8, 10, 10, "cheb-cg"), (9, 9, 9, "cheb-cg")])
def test_wide_blocks_equal_single_bit_for_bit(q, nrhs, max_rhs, inner):
    """Blocks of 64 plus a remainder (the CG scalar steps and window-free
    operators over 8 chunks), and blocks on levels of 512 x 512 points and more,
    where the prolongations read R once per chunk of 8 right-hand sides (q = 9:
    the finest level, chunks of 8 and 2; q = 10: also level 9, one chunk of 3),
    and the block CG operator stages the coarse vectors of levels with 64 or
    more parents per side in LDS (q = 8 and 9 with CG below the finest level)."""
    print("CASE test=wide_block_bits", q, nrhs, max_rhs, inner, flush=True)
    P = _P()
    pr = S.rough_problem(q, 1.0, 33, nrhs=nrhs)
    a = _dev(pr.a)
    g = _dev(pr.g)
    kw = dict(rho=3, precision="mixed", rtol=1e-15, max_outer=9, inner=inner)
    if inner != "chebyshev":
        kw.update(inner_iters=8, inner_iters_coarse=4)
    Hb = P.Hierarchy(a, max_rhs=max_rhs, **kw)
    ub = Hb.solve(g, check=False)
    assert Hb.last_info.outer_iters == 9
    Hb.close()
    Hs = P.Hierarchy(a, max_rhs=1, **kw)
    for r in range(nrhs):
        us = Hs.solve(g[r], check=False)
        assert torch.equal(us, ub[r]), (r, float((us - ub[r]).abs().max()))
    Hs.close()


def test_block_adjoint_equals_single():
    print("CASE test=block_adjoint", flush=True)
    P = _P()
    pr = S.rough_problem(6, 1.0, 32, nrhs=3)
    a = _dev(pr.a)
    g = _dev(pr.g)
    kw = dict(rho=3, precision="mixed", rtol=1e-15, max_outer=7)
    Hb = P.Hierarchy(a, max_rhs=3, **kw)
    u = Hb.solve(g, check=False)
    dJdu = (u * 0.5).contiguous()
    gb, _, lb = Hb.adjoint(u, dJdu, check=False)
    Hb.close()
    Hs = P.Hierarchy(a, max_rhs=1, **kw)
    for r in range(3):
        gs, _, ls = Hs.adjoint(u[r].contiguous(), dJdu[r].contiguous(), check=False)
        assert torch.equal(ls, lb[r]), r
        assert torch.equal(gs, gb[r]), r
    Hs.close()


@pytest.mark.parametrize("nrhs,max_rhs", [(16, 16), (20, 8)])
def test_block_solve_matches_direct(nrhs, max_rhs):
    print("CASE test=block_direct", nrhs, max_rhs, flush=True)
    pr = S.rough_problem(7, 1.0, 33, nrhs=nrhs)
    u_ref = fem.solve(pr.a, pr.g)
    P = _P()
    H = P.Hierarchy(_dev(pr.a), rho=3, precision="mixed", rtol=1e-9, max_rhs=max_rhs)
    u = H.solve(_dev(pr.g)).cpu().numpy()
    print("info", H.last_info, flush=True)
    H.close()
    for r in range(nrhs):
        err = np.linalg.norm(u[r] - u_ref[r]) / np.linalg.norm(u_ref[r])
        assert err < 1e-8, (r, err)
