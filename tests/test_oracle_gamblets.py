"""Pins of the gamblet oracle against the paper's identities and brute force.

Each test fixes a part of ``oracle.gamblets`` through something the paper
proves or a different computation of the same object:

* Lemma 4.12: Helmert rows orthonormal, last row constant.
* Theorem 4.15 / eq. (orthogonal decomposition of u): the exact transform
  reproduces the direct FE solve, and its subbands are A-orthogonal
  (Theorem 4.6).
* Theorem 4.8: R pi^T = I, A^(k) = R A^(k+1) R^T, R = A^(k) pi Theta^(k+1),
  Theta^(k) = pi Theta^(k+1) pi^T, checked against the closed form
  A^(k) = (Pi A^-1 Pi^T)^-1 built from A^-1 alone.
* Remark 4.10: R A W^T = 0.
* Eq. defining psi^(k) as constrained minimisers: brute-force KKT solves.
* Theorem 4.3: u^(k) is the A-Galerkin projection onto V^(k).
* Constructions 4.11 and 4.13 give the same R and subbands.
* Localized transform (Definition 5.3): equals the exact one when the patch
  covers the level, equals the patchwise energy minimisation of Remark 5.4,
  and its error decreases geometrically in rho (Theorem 5.5).
"""
import numpy as np
import pytest
import scipy.sparse as sp

import synthetic as S
from oracle import fem
from oracle import gamblets as G


def _setup(q, sigma=1.0, tag=5):
    pr = S.rough_problem(q, sigma, tag)
    fe = fem.assemble(pr.a)
    b = fem.load_cellwise(pr.g[0], fe.h)
    return pr, fe, b


def _Pi(tree, k):
    """pi^(k,q) as a product of one-level aggregations."""
    P = sp.identity(tree.size(tree.q), format="csr")
    for j in range(tree.q, k, -1):
        P = tree.pi(j) @ P
    return P.toarray()


@pytest.mark.parametrize("m", [1, 2, 3, 4, 7])
def test_helmert(m):
    U = G.helmert(m)
    np.testing.assert_allclose(U @ U.T, np.eye(m), atol=1e-15)
    np.testing.assert_allclose(U[-1], np.full(m, 1.0 / np.sqrt(m)), atol=1e-15)


@pytest.mark.parametrize("q,sigma", [(4, 1.0), (5, 2.0), (6, 1.0)])
def test_exact_transform_reproduces_direct_solve(q, sigma):
    _, fe, b = _setup(q, sigma)
    u = fem.DirectSolver(fe.A).solve(b)
    H = G.exact_hierarchy(fe.A, G.Tree(q))
    assert np.linalg.norm(G.solve(H, b) - u) / np.linalg.norm(u) < 1e-12
    sb = G.subbands(H, b)
    assert np.linalg.norm(sum(sb) - u) / np.linalg.norm(u) < 1e-12
    A = fe.A
    en = [np.sqrt(s @ (A @ s)) for s in sb]
    for i in range(len(sb)):
        for j in range(i + 1, len(sb)):
            assert abs(sb[i] @ (A @ sb[j])) <= 1e-11 * en[i] * en[j]


@pytest.mark.parametrize("q", [4, 5])
def test_theorem_4_8_identities_and_closed_form(q):
    _, fe, _ = _setup(q, 2.0, tag=9)
    tree = G.Tree(q)
    H = G.exact_hierarchy(fe.A, tree)
    Ainv = np.linalg.inv(fe.A.toarray())
    for k in range(q, 1, -1):
        lv = H.levels[k]
        P = tree.pi(k).toarray()
        R = lv.R
        np.testing.assert_allclose(R @ P.T, np.eye(P.shape[0]), atol=1e-12)
        Wd = lv.W.toarray()
        assert np.abs(R @ lv.A @ Wd.T).max() <= 1e-12 * np.abs(lv.A).max()
        Pk = _Pi(tree, k)
        Pkm1 = _Pi(tree, k - 1)
        Theta_k = Pk @ Ainv @ Pk.T
        Theta_km1 = Pkm1 @ Ainv @ Pkm1.T
        np.testing.assert_allclose(Theta_km1, P @ Theta_k @ P.T, rtol=1e-12, atol=1e-15)
        Akm1 = np.linalg.inv(Theta_km1)
        Anext = H.levels[k - 1].A
        assert np.linalg.norm(Anext - Akm1) / np.linalg.norm(Akm1) < 1e-10
        np.testing.assert_allclose(R, Anext @ P @ Theta_k, atol=1e-9 * np.abs(R).max())


@pytest.mark.parametrize("q", [3, 4])
def test_gamblets_are_constrained_energy_minimisers(q):
    """psi^(k)_i minimises c^T A c s.t. pi^(k,q) c = e_i (brute-force KKT)."""
    _, fe, _ = _setup(q, 1.0, tag=12)
    tree = G.Tree(q)
    H = G.exact_hierarchy(fe.A, tree)
    A = fe.A.toarray()
    N = A.shape[0]
    for k in range(1, q):
        Pi = _Pi(tree, k)
        m = Pi.shape[0]
        KKT = np.block([[A, Pi.T], [Pi, np.zeros((m, m))]])
        rhs = np.zeros((N + m, m))
        rhs[N:, :] = np.eye(m)
        Psi_kkt = np.linalg.solve(KKT, rhs)[:N].T
        Psi = np.eye(m)
        for j in range(k + 1, q + 1):
            Psi = Psi @ H.levels[j].R
        np.testing.assert_allclose(Psi, Psi_kkt, atol=1e-10)


def test_partial_sums_are_galerkin_projections():
    q = 5
    _, fe, b = _setup(q, 1.0, tag=13)
    tree = G.Tree(q)
    H = G.exact_hierarchy(fe.A, tree)
    A = fe.A.toarray()
    u = np.linalg.solve(A, b)
    sb = G.subbands(H, b)
    Ainv = np.linalg.inv(A)
    acc = np.zeros_like(u)
    for k in range(1, q):
        acc = acc + sb[k - 1]
        Pi = _Pi(tree, k)
        Y = Ainv @ Pi.T
        proj = Y @ np.linalg.solve(Pi @ Y, Pi @ u)
        assert np.linalg.norm(acc - proj) / np.linalg.norm(u) < 1e-10


def test_constructions_agree():
    q = 5
    _, fe, b = _setup(q, 2.0, tag=14)
    tree = G.Tree(q)
    H1 = G.exact_hierarchy(fe.A, tree, construction=1)
    H2 = G.exact_hierarchy(fe.A, tree, construction=2)
    for k in range(q, 1, -1):
        np.testing.assert_allclose(H1.levels[k].R, H2.levels[k].R, atol=1e-11)
    s1, s2 = G.subbands(H1, b), G.subbands(H2, b)
    for x, y in zip(s1, s2):
        assert np.linalg.norm(x - y) <= 1e-11 * np.linalg.norm(sum(s2))
    L1 = G.localized_hierarchy(fe.A, tree, 2, construction=1)
    L2 = G.localized_hierarchy(fe.A, tree, 2, construction=2)
    for k in range(q, 1, -1):
        assert abs(L1.levels[k].R - L2.levels[k].R).max() < 1e-11


def test_localized_equals_exact_when_patch_covers_level():
    q = 5
    _, fe, b = _setup(q, 1.0, tag=15)
    tree = G.Tree(q)
    H = G.exact_hierarchy(fe.A, tree)
    L = G.localized_hierarchy(fe.A, tree, rho=1 << q)
    for k in range(q, 1, -1):
        np.testing.assert_allclose(L.levels[k].R.toarray(), H.levels[k].R, atol=1e-11)
        np.testing.assert_allclose(L.levels[k - 1].A.toarray(), H.levels[k - 1].A,
                                   atol=1e-10 * np.abs(H.levels[k - 1].A).max())


@pytest.mark.parametrize("rho", [1, 2])
def test_localized_R_equals_patch_energy_minimisation(rho):
    q = 5
    _, fe, _ = _setup(q, 2.0, tag=16)
    tree = G.Tree(q)
    L = G.localized_hierarchy(fe.A, tree, rho)
    for k in range(q, 1, -1):
        R_kkt = G.localized_R_by_energy_minimization(L.levels[k].A, tree, k, rho)
        assert abs(R_kkt - L.levels[k].R).max() < 1e-10


def test_localization_error_decays_in_rho():
    q = 6
    _, fe, b = _setup(q, 1.0, tag=17)
    tree = G.Tree(q)
    u = fem.DirectSolver(fe.A).solve(b)
    A = fe.A
    errs = []
    for rho in (1, 2, 3):
        L = G.localized_hierarchy(fe.A, tree, rho)
        e = G.solve(L, b) - u
        errs.append(np.sqrt(e @ (A @ e) / (u @ (A @ u))))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.5 * errs[1] and errs[1] < 0.5 * errs[0]


def test_refinement_reaches_direct_solution():
    q = 5
    _, fe, b = _setup(q, 2.0, tag=18)
    tree = G.Tree(q)
    L = G.localized_hierarchy(fe.A, tree, 2)
    u = fem.DirectSolver(fe.A).solve(b)
    ur, sweeps, _ = G.refine_solve(L, fe.A, b, tol=1e-12)
    assert np.linalg.norm(ur - u) / np.linalg.norm(u) < 1e-10


def test_paper_geometry_tree_is_uniform():
    """Example 5.1 geometry: 2^q interior nodes per dimension, 4 children everywhere."""
    tree = G.Tree(3, offset=1)
    assert tree.size(3) == 64
    assert all(len(ch) == 4 for ch in tree.children[3])
    tree0 = G.Tree(3)
    counts = sorted(len(ch) for ch in tree0.children[3])
    assert counts.count(1) == 1 and counts.count(2) == 6 and counts.count(4) == 9


@pytest.mark.parametrize("rho", [1, 2, 3])
def test_tree_box_sizes(rho):
    """Definition 5.3's patch as read here (the box of coarse cells within rho
    in each coordinate, clipped to the domain): an interior box holds
    (2 rho + 1)^2 cells, a corner box (rho + 1)^2, an edge box
    (rho + 1)(2 rho + 1); level-q boxes are clipped to the interior nodes."""
    tree = G.Tree(6)
    k = 5
    side = 1 << k
    idx = lambda x, y: x * side + y
    assert tree.box(k, idx(10, 12), rho).size == (2 * rho + 1) ** 2
    assert tree.box(k, idx(0, 0), rho).size == (rho + 1) ** 2
    assert tree.box(k, idx(side - 1, side - 1), rho).size == (rho + 1) ** 2
    assert tree.box(k, idx(0, 12), rho).size == (rho + 1) * (2 * rho + 1)
    # the members are exactly the cells within rho in both coordinates
    members = {tuple(c) for c in tree.coords[k][tree.box(k, idx(10, 12), rho)]}
    assert members == {(x, y) for x in range(10 - rho, 11 + rho) for y in range(12 - rho, 13 + rho)}
    # level q: node (1, 1) is the first interior node; its box stops at the boundary
    m = (1 << 6) - 1
    assert tree.box(6, 0, rho).size == (rho + 1) ** 2
    assert tree.box(6, (m // 2) * m + m // 2, rho).size == (2 * rho + 1) ** 2


def test_example51_exact_transform():
    """Example 5.1 end to end: exact transform on the paper's own mesh reproduces the FE solve."""
    a = S.example51_coefficient()
    fe = fem.assemble(a, h=1.0 / 65.0)
    b = fem.load_nodal(S.example51_nodal_source(), fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    tree = G.Tree(6, offset=1)
    H = G.exact_hierarchy(fe.A, tree)
    assert np.linalg.norm(G.solve(H, b) - u) / np.linalg.norm(u) < 1e-12


def test_per_level_radii():
    """Algorithm 2 with one patch radius per transition: equal radii given per
    level reproduce the single-radius hierarchy, and radii that cover every
    level reproduce the exact hierarchy (Algorithm 1)."""
    q = 4
    pr = S.rough_problem(q, 1.5, 24)
    fe = fem.assemble(pr.a)
    tree = G.Tree(q)
    one = G.localized_hierarchy(fe.A, tree, 2)
    per = G.localized_hierarchy(fe.A, tree, {k: 2 for k in range(2, q + 1)})
    for k in range(1, q + 1):
        assert abs(one.levels[k].A - per.levels[k].A).max() == 0.0
    cover = G.localized_hierarchy(fe.A, tree, {k: 1 << (k - 1) for k in range(2, q + 1)})
    ex = G.exact_hierarchy(fe.A, tree)
    for k in range(1, q + 1):
        d = abs(cover.levels[k].A - ex.levels[k].A).max() / abs(ex.levels[k].A).max()
        assert d < 1e-10, (k, d)
    mixed = G.localized_hierarchy(fe.A, tree, {q: 2, 3: 1, 2: 1})
    assert abs(mixed.levels[2].A - one.levels[2].A).max() > 0.0
