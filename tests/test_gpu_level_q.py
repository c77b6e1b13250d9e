"""GPU level-q gamblets from the localized mass inverse (Algorithm 2, the
lines before the level loop; Definition 5.2) against the FP64 CPU oracle,
through the C ABI.

The GPU forms each patch inverse as the outer product of two tridiagonal
solves (the mass matrix and a box patch are Kronecker products); the oracle
solves the two-dimensional patch systems.  Both are FP64: 1e-13 relative on
the gamblet weights, loads and nodal values, 1e-12 on the operator (sums of
up to 49 x 9 products of entries of mixed sign)."""
import numpy as np
import pytest

import synthetic as S
from oracle import fem
from oracle import mass_inverse as MI

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    import paper_1503_03467_amd as P
    return P


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("q,rho", [(2, 1), (2, 4), (4, 1), (4, 3), (5, 2), (5, 4)])
def test_gamblets_match_oracle(q, rho):
    _case(test="level_q_gamblets", q=q, rho=rho)
    n = 1 << q
    m = n - 1
    lq = _P().LevelQ(q, rho)
    W = lq.gamblets().cpu().numpy()
    Minv = MI.localized_mass_inverse(MI.mass_matrix(n), n, rho).toarray()
    w = 2 * rho + 1
    ref = np.zeros_like(W)
    for i in range(m * m):
        ix, iy = divmod(i, m)
        for dx in range(-rho, rho + 1):
            for dy in range(-rho, rho + 1):
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < m and 0 <= jy < m:
                    ref[i, (dx + rho) * w + dy + rho] = Minv[jx * m + jy, i]
    err = _rel(W, ref)
    print("weights rel err", err)
    assert err < 1e-13


@pytest.mark.parametrize("q,rho,sigma", [(3, 1, 1.0), (4, 2, 2.0), (5, 3, 2.0), (5, 4, 1.0)])
def test_operator_load_and_nodal_match_oracle(q, rho, sigma):
    _case(test="level_q_operator", q=q, rho=rho, sigma=sigma)
    pr = S.rough_problem(q, sigma, 51)
    fe = fem.assemble(pr.a)
    lq_ref = MI.level_q_gamblets(fe, rho)
    m = fe.n - 1
    lq = _P().LevelQ(q, rho)
    st = lq.operator(_dev(pr.a)).cpu().numpy()
    ref = MI.stencil_rows(lq_ref, np.arange(m * m))
    err = _rel(st, ref)
    print("operator rel err", err)
    assert err < 1e-12
    b = fem.load_cellwise(pr.g[0], fe.h)
    g = lq.load(_dev(b)).cpu().numpy()
    assert _rel(g, MI.level_q_load(lq_ref, b)) < 1e-13
    U = np.random.default_rng(3).standard_normal(m * m)
    v = lq.to_nodal(_dev(U)).cpu().numpy()
    assert _rel(v, MI.level_q_to_nodal(lq_ref, U)) < 1e-13


def test_gpu_pieces_give_the_fe_solution():
    """Galerkin solve in the psi^(q) basis with the GPU operator, load and
    nodal map (a dense solve of the assembled stencil on the host) equals the
    finite-element solution."""
    q, rho = 5, 3
    _case(test="level_q_solution", q=q, rho=rho)
    pr = S.rough_problem(q, 2.0, 52)
    fe = fem.assemble(pr.a)
    m = fe.n - 1
    lq = _P().LevelQ(q, rho)
    st = lq.operator(_dev(pr.a)).cpu().numpy()
    Sw = 2 * rho + 1
    W = 2 * Sw + 1
    Aq = np.zeros((m * m, m * m))
    for i in range(m * m):
        ix, iy = divmod(i, m)
        for e in np.flatnonzero(st[i]):
            dx, dy = e // W - Sw, e % W - Sw
            Aq[i, (ix + dx) * m + iy + dy] = st[i, e]
    assert np.abs(Aq - Aq.T).max() <= 1e-13 * np.abs(Aq).max()
    b = fem.load_cellwise(pr.g[0], fe.h)
    U = np.linalg.solve(Aq, lq.load(_dev(b)).cpu().numpy())
    u = lq.to_nodal(_dev(U)).cpu().numpy()
    u_ref = fem.DirectSolver(fe.A).solve(b)
    err = float(np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref))
    print("solution rel err", err)
    assert err < 1e-10


def test_full_size_rows_match_oracle():
    """512 x 512 cells, patch radius 3 (the benchmark problem's coefficient):
    sampled operator rows, including the corners and edges, against the
    oracle's entry-by-entry products y^(i)T A y^(j); the whole operator is
    symmetric."""
    _case(test="level_q_full_size")
    pr = S.q9_rough_problem()
    q, rho = pr.q, 3
    fe = fem.assemble(pr.a)
    M = MI.mass_matrix(fe.n)
    m = fe.n - 1
    lq = _P().LevelQ(q, rho)
    st = lq.operator(_dev(pr.a))
    torch.cuda.synchronize()
    rng = np.random.default_rng(9)
    rows = [0, m - 1, m * m - 1, m * (m - 1), 2 * m + 1] + [int(x) for x in rng.integers(0, m * m, 6)]
    got = st[rows].cpu().numpy()
    for r, i in enumerate(rows):
        ref = MI.operator_row(fe, M, rho, i)
        err = _rel(got[r], ref)
        assert err < 1e-12, (i, err)
    # symmetry: entry (i, d) equals entry (i + d, -d)
    Sw = 2 * rho + 1
    W = 2 * Sw + 1
    stc = st.cpu().numpy().reshape(m, m, W, W)
    asym = 0.0
    for dx in range(-Sw, Sw + 1):
        for dy in range(-Sw, Sw + 1):
            x0, x1 = max(0, -dx), min(m, m - dx)
            y0, y1 = max(0, -dy), min(m, m - dy)
            a1 = stc[x0:x1, y0:y1, dx + Sw, dy + Sw]
            a2 = stc[x0 + dx:x1 + dx, y0 + dy:y1 + dy, Sw - dx, Sw - dy]
            asym = max(asym, float(np.abs(a1 - a2).max()))
    print("asymmetry", asym / np.abs(stc).max())
    assert asym <= 1e-13 * np.abs(stc).max()
