"""The exact (unlocalized) hierarchy of Algorithm 1 on the GPU against the FP64
CPU oracle, through the C ABI: level matrices A^(k), B^(k), R^(k-1,k), the
subband solve of Theorem 4.15 against a sparse direct solve, and the
representation of the solution in the normalized exact basis (discussion of
Example 5.1, Figures 10-11) with its compression at 1, 5 and 25 % of the
coefficients.

Geometries: 0 is the 2^q x 2^q cell mesh of the other tests (cells on the two
low edges of level q-1 have one or two children); 1 is the mesh of Example
5.1 itself, (2^q + 1)^2 cells and 2^q x 2^q interior nodes, a uniform
quad-tree (``oracle.gamblets.Tree(q, offset=1)``).

Tolerances: everything here is FP64 on both sides.  The level matrices differ
only by the rounding order of the dense products and Cholesky solves; relative
to the largest entry of each matrix, 1e-10 (the FP64-path bound).  Solves are
compared with the relative Euclidean error 1e-10 after the two refinement
steps the library takes (a single subband solve already sits near 1e-13 at
these sizes).
"""
import numpy as np
import pytest

import synthetic as S
from oracle import fem
from oracle import gamblets as G
from tests.gpu_layout import subband_map

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _P():
    import paper_1503_03467_amd as P
    return P


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def _case(**kw):
    print("CASE", " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _nodal(fe, u_int):
    full = np.zeros((fe.n + 1) ** 2)
    full[fe.interior] = u_int
    return full.reshape(fe.n + 1, fe.n + 1)


def _coefficient(q, geometry, tag):
    n = (1 << q) + geometry
    return S.product_field(n, K=5) * np.exp(S.rng(tag).standard_normal((n, n)))


def _gpu_to_oracle(c, tree, q):
    """GPU coefficient vector -> (c1, {k: ck}) in oracle order and the padding entries."""
    c1 = c[:4].copy()
    ck, pads = {}, []
    for k in range(2, q + 1):
        npar = 1 << (2 * (k - 1))
        blk = c[npar: 4 * npar]
        m = subband_map(tree, k)
        out = np.zeros(int(m.max()) + 1)
        out[m[m >= 0]] = blk[m >= 0]
        ck[k] = out
        pads.append(blk[m < 0])
    return c1, ck, np.concatenate(pads)


@pytest.mark.parametrize("q,geometry", [(3, 0), (4, 0), (5, 0), (3, 1), (4, 1), (5, 1)])
def test_exact_level_matrices_match_oracle(q, geometry):
    _case(test="exact_levels", q=q, geometry=geometry)
    a = _coefficient(q, geometry, 501 + q)
    fe = fem.assemble(a)
    tree = G.Tree(q, offset=geometry)
    h = G.exact_hierarchy(fe.A, tree)
    H = _P().Hierarchy(_dev(a), exact=True, geometry=geometry)
    torch.cuda.synchronize()
    for k in range(q, 0, -1):
        lv = H.level(k)
        assert lv["n"] == tree.size(k)
        assert _maxrel(lv["A"].cpu().numpy(), h.levels[k].A) < 1e-10, k
        if k == 1:
            continue
        ref = h.levels[k]
        assert _maxrel(lv["R"].cpu().numpy(), ref.R) < 1e-10, k
        B = lv["B"].cpu().numpy()
        m = subband_map(tree, k)
        real = np.flatnonzero(m >= 0)
        pad = np.flatnonzero(m < 0)
        Bo = np.zeros_like(ref.B)
        Bo[np.ix_(m[real], m[real])] = B[np.ix_(real, real)]
        assert _maxrel(Bo, ref.B) < 1e-10, k
        # padding rows: identity, decoupled from the real subband rows
        if pad.size:
            assert np.array_equal(B[np.ix_(pad, pad)], np.eye(pad.size))
            assert not np.any(B[np.ix_(pad, real)]) and not np.any(B[np.ix_(real, pad)])
    H.close()


@pytest.mark.parametrize("geometry", [0, 1])
def test_exact_construction_4_11(geometry):
    """W from the differences of Construction 4.11: B^(k) and the transform
    coefficients follow the oracle built with that construction (1e-10), while
    A^(k), R and the solve equal those of Construction 4.13 (they do not
    depend on the choice of W)."""
    q = 4
    _case(test="exact_construction_4_11", q=q, geometry=geometry)
    a = _coefficient(q, geometry, 801)
    fe = fem.assemble(a)
    tree = G.Tree(q, offset=geometry)
    h1 = G.exact_hierarchy(fe.A, tree, construction=1)
    H1 = _P().Hierarchy(_dev(a), exact=True, geometry=geometry, w_kind=1)
    H2 = _P().Hierarchy(_dev(a), exact=True, geometry=geometry)
    for k in range(q, 1, -1):
        l1, l2 = H1.level(k), H2.level(k)
        assert _maxrel(l1["A"].cpu().numpy(), h1.levels[k].A) < 1e-10
        assert _maxrel(l1["R"].cpu().numpy(), l2["R"].cpu().numpy()) < 1e-10
        B = l1["B"].cpu().numpy()
        m = subband_map(tree, k)
        real = np.flatnonzero(m >= 0)
        Bo = np.zeros_like(h1.levels[k].B)
        Bo[np.ix_(m[real], m[real])] = B[np.ix_(real, real)]
        assert _maxrel(Bo, h1.levels[k].B) < 1e-10, k
    n = (1 << q) + geometry
    g = S.rng(802).standard_normal((n, n))
    u1, u2 = H1.solve(_dev(g)), H2.solve(_dev(g))
    assert _rel(u1.cpu().numpy(), u2.cpu().numpy()) < 1e-12
    uref = fem.DirectSolver(fe.A).solve(fem.load_cellwise(g, fe.h))
    c1_ref, ck_ref = G.normalized_coefficients(h1, uref)
    c = H1.transform(_dev(_nodal(fe, uref)))
    c1, ck, pads = _gpu_to_oracle(c.cpu().numpy(), tree, q)
    assert not np.any(pads)
    allg = np.concatenate([c1] + [ck[k] for k in sorted(ck)])
    allr = np.concatenate([c1_ref] + [ck_ref[k] for k in sorted(ck_ref)])
    assert _rel(allg, allr) < 1e-10
    back = H1.inverse_transform(c).cpu().numpy().ravel()[fe.interior]
    assert _rel(back, uref) < 1e-12
    H1.close()
    H2.close()


@pytest.mark.parametrize("q,geometry,source", [(4, 0, "cell"), (6, 0, "cell"), (5, 1, "cell"), (6, 1, "nodal"),
                                                 (7, 0, "cell")])
def test_exact_solve_matches_direct(q, geometry, source):
    """Theorem 4.15: the subband sum equals the direct solve.  (q=6, geometry 0,
    g = 1) is the 64 x 64 exact workload; (q=6, geometry 1, nodal) is Example 5.1."""
    _case(test="exact_solve", q=q, geometry=geometry, source=source)
    if (q, geometry, source) == (6, 1, "nodal"):
        a, gsrc = S.example51_coefficient(), S.example51_nodal_source()
    elif (q, geometry) == (6, 0):
        pr = S.q6_exact_problem()
        a, gsrc = pr.a, pr.g[0]
    else:
        a = _coefficient(q, geometry, 601 + q)
        n = (1 << q) + geometry
        gsrc = S.rng(611 + q).standard_normal((n, n))
    fe = fem.assemble(a)
    b = fem.load_nodal(gsrc, fe.h) if source == "nodal" else fem.load_cellwise(gsrc, fe.h)
    ref = fem.DirectSolver(fe.A).solve(b)
    H = _P().Hierarchy(_dev(a), exact=True, geometry=geometry, source=source, max_rhs=2)
    u = H.solve(_dev(gsrc)).cpu().numpy()
    assert np.all(u[0, :] == 0) and np.all(u[:, 0] == 0) and np.all(u[-1, :] == 0) and np.all(u[:, -1] == 0)
    err = _rel(u.ravel()[fe.interior], ref)
    print("exact solve rel err", err, flush=True)
    assert err < 1e-10
    # two right-hand sides in one call give the same solutions
    g2 = np.stack([gsrc, -2.0 * gsrc])
    u2 = H.solve(_dev(g2)).cpu().numpy()
    assert _rel(u2[0].ravel()[fe.interior], ref) < 1e-10
    assert _rel(u2[1].ravel()[fe.interior], -2.0 * ref) < 1e-10
    H.close()


@pytest.mark.parametrize("geometry", [0, 1])
def test_exact_solve_lifts_dirichlet_data(geometry):
    """Non-zero boundary values are moved to the load (b - A_IB u_B) and kept in u."""
    q = 4
    _case(test="exact_dirichlet", q=q, geometry=geometry)
    a = _coefficient(q, geometry, 701)
    n = (1 << q) + geometry
    g = S.rng(702).standard_normal((n, n))
    ub = S.rng(703).standard_normal((n + 1, n + 1))
    ref = fem.solve(a, g, ub)
    H = _P().Hierarchy(_dev(a), exact=True, geometry=geometry)
    u = H.solve(_dev(g), u_boundary=_dev(ub)).cpu().numpy()
    assert _rel(u, ref) < 1e-10
    H.close()


@pytest.mark.parametrize("geometry", [0, 1])
def test_exact_transform_and_compression_match_oracle(geometry):
    """Coefficients on psi^(1)/||psi^(1)||_a and chi^(k)/||chi^(k)||_a, the round
    trip, the energy norm, and compression to 1, 5 and 25 % (energy errors and
    kept sets equal to the oracle's).  Geometry 1 is Example 5.1."""
    q = 6
    _case(test="exact_compression", q=q, geometry=geometry)
    if geometry == 1:
        a, gsrc, source = S.example51_coefficient(), S.example51_nodal_source(), "nodal"
    else:
        pr = S.rough_problem(q, 2.0, 34)
        a, gsrc, source = pr.a, S.smooth_cell_source(q), "cell"
    fe = fem.assemble(a)
    tree = G.Tree(q, offset=geometry)
    h = G.exact_hierarchy(fe.A, tree)
    b = fem.load_nodal(gsrc, fe.h) if source == "nodal" else fem.load_cellwise(gsrc, fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    c1_ref, ck_ref = G.normalized_coefficients(h, u)
    H = _P().Hierarchy(_dev(a), exact=True, geometry=geometry, source=source)
    u_dev = _dev(_nodal(fe, u))
    c = H.transform(u_dev)
    c1, ck, pads = _gpu_to_oracle(c.cpu().numpy(), tree, q)
    assert not np.any(pads)
    allg = np.concatenate([c1] + [ck[k] for k in sorted(ck)])
    allr = np.concatenate([c1_ref] + [ck_ref[k] for k in sorted(ck_ref)])
    assert _rel(allg, allr) < 1e-10
    # round trip and energy norm
    back = H.inverse_transform(c).cpu().numpy().ravel()[fe.interior]
    assert _rel(back, u) < 1e-12
    eref = float(np.sqrt(u @ (fe.A @ u)))
    assert abs(H.energy_norm(u_dev) - eref) <= 1e-12 * eref
    # compression
    total = allr.size
    errs = []
    for frac in (0.01, 0.05, 0.25):
        keep = int(round(frac * total))
        a1, ak = G.compress(c1_ref, ck_ref, keep)
        v_ref = G.reconstruct_normalized(h, a1, ak)
        e_ref = float(np.sqrt((u - v_ref) @ (fe.A @ (u - v_ref)))) / eref
        cc = c.clone()
        thr = H.compress(cc, keep)
        g1, gk, _ = _gpu_to_oracle(cc.cpu().numpy(), tree, q)
        kept_g = np.concatenate([g1] + [gk[k] for k in sorted(gk)]) != 0
        kept_r = np.concatenate([a1] + [ak[k] for k in sorted(ak)]) != 0
        assert np.array_equal(kept_g, kept_r), frac
        assert thr == pytest.approx(np.min(np.abs(allr[kept_r])), rel=1e-10)
        v = H.inverse_transform(cc)
        e = H.energy_norm(v - u_dev) / eref
        print(f"exact compression geometry={geometry} keep={frac:.2f} energy error gpu={e:.4e} oracle={e_ref:.4e}",
              flush=True)
        assert abs(e - e_ref) <= 1e-8 * max(e_ref, 1e-3)
        errs.append(e)
    assert errs[0] > errs[1] > errs[2]
    H.close()


def test_exact_source_constant_on_level_one_cells_lives_in_psi1():
    """g = 1 on the 64 x 64 exact workload: the load b = h^2 (1, ..., 1) is a sum
    of level-1 measurement functions, so the solution is the level-1 gamblet
    part alone (Theorem 4.6 / the conditional-expectation reading of Section
    3: u^(1) = u when b lies in the range of the level-1 aggregation): every
    subband coefficient of levels 2..q vanishes to rounding."""
    _case(test="exact_level1_source")
    pr = S.q6_exact_problem()
    H = _P().Hierarchy(_dev(pr.a), exact=True)
    u = H.solve(_dev(pr.g[0]))
    c = H.transform(u).cpu().numpy()
    assert np.linalg.norm(c[4:]) <= 1e-12 * np.linalg.norm(c[:4])
    H.close()


def test_exact_mode_rejections():
    """Options the exact hierarchy does not take are refused with EINVAL."""
    P = _P()
    a = _dev(np.ones((8, 8)))
    with pytest.raises(P.GambletError):
        P.Hierarchy(_dev(np.ones((1 << 8, 1 << 8))), exact=True)   # q = 8 exceeds the dense limit
    H = P.Hierarchy(a, exact=True)
    m = 9
    with pytest.raises(P.GambletError):
        H.adjoint(_dev(np.zeros((m, m))), _dev(np.zeros((m, m))))
    H.close()
