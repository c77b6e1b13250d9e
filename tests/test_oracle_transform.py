"""Pins of the oracle's gamblet transform (representation of a vector in the
basis psi^(1)/||psi^(1)||_a, chi^(k)/||chi^(k)||_a; discussion of Example 5.1)
and of its compression.

* the reconstruction of Theorem 4.15 inverts the transform (a basis has one
  representation), for the exact and the localized hierarchy;
* for the exact hierarchy the transform of u = A^-1 b equals the subband
  coefficients w^(k) = B^(k)-1 W^(k) g^(k), U^(1) = A^(1)-1 g^(1) of
  Algorithm 1 (an independent route: subband solves, not measurements);
* the exact gamblet subspaces are A-orthogonal across levels, so the energy
  of u splits over the levels (Pythagoras);
* ||chi^(k)_j||_a^2 = B^(k)_jj and ||psi^(1)_i||_a^2 = A^(1)_ii, checked on the
  gamblets formed explicitly on the fine mesh;
* compression keeps exactly the largest coefficients; keeping all of them
  changes nothing, and the energy error shrinks as more are kept.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import fem
from oracle import gamblets as G


def _setup(q, rho, seed=3, sigma=1.5):
    pr = S.rough_problem(q, sigma, seed)
    fe = fem.assemble(pr.a)
    tree = G.Tree(q)
    h = G.exact_hierarchy(fe.A, tree) if rho is None else G.localized_hierarchy(fe.A, tree, rho)
    return pr, fe, tree, h


def _energy(A, v):
    return float(np.sqrt(v @ (A @ v)))


@pytest.mark.parametrize("q,rho", [(4, None), (5, 2), (5, 3)])
def test_reconstruction_inverts_transform(q, rho):
    pr, fe, tree, h = _setup(q, rho)
    u = np.random.default_rng(7).standard_normal(tree.size(q))
    U1, w = G.gamblet_transform(h, u)
    v = G.inverse_transform(h, U1, w)
    assert np.linalg.norm(v - u) / np.linalg.norm(u) < 1e-12
    c1, ck = G.normalized_coefficients(h, u)
    v2 = G.reconstruct_normalized(h, c1, ck)
    assert np.linalg.norm(v2 - u) / np.linalg.norm(u) < 1e-12


@pytest.mark.parametrize("q", [3, 4])
def test_transform_of_solution_equals_subband_solves(q):
    pr, fe, tree, h = _setup(q, None, seed=11)
    b = fem.load_cellwise(pr.g[0], fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    U1, w = G.gamblet_transform(h, u)
    U1s, ws, _ = G.subband_coefficients(h, b)
    assert np.linalg.norm(U1 - U1s) / np.linalg.norm(U1s) < 1e-10
    for k in ws:
        assert np.linalg.norm(w[k] - ws[k]) / max(np.linalg.norm(ws[k]), 1e-300) < 1e-9, k


def test_exact_levels_are_energy_orthogonal():
    q = 4
    pr, fe, tree, h = _setup(q, None, seed=5)
    u = np.random.default_rng(2).standard_normal(tree.size(q))
    U1, w = G.gamblet_transform(h, u)
    parts = U1 @ (h.levels[1].A @ U1) + sum(w[k] @ (h.levels[k].B @ w[k]) for k in w)
    total = u @ (fe.A @ u)
    assert abs(parts - total) / total < 1e-11
    # the normalized coefficients carry the per-level energies only within a
    # level's Gram matrix, not as a plain sum of squares (chi^(k) are not
    # A-orthogonal inside a level)
    c1, ck = G.normalized_coefficients(h, u)
    assert abs(np.sum(c1 ** 2) + sum(np.sum(ck[k] ** 2) for k in ck) - total) / total > 1e-6


@pytest.mark.parametrize("rho", [None, 2])
def test_energy_scales_match_explicit_gamblets(rho):
    q = 4
    pr, fe, tree, h = _setup(q, rho, seed=9)
    s1, sk = G.energy_scales(h)
    rng = np.random.default_rng(4)
    for i in rng.choice(tree.size(1), 2, replace=False):
        e = np.zeros(tree.size(1)); e[i] = 1.0
        psi = G.prolong(h, 1, e)
        assert abs(_energy(fe.A, psi) - s1[i]) / s1[i] < 1e-10
    for k in (2, 3, q):
        nj = h.levels[k].W.shape[0]
        for j in rng.choice(nj, 3, replace=False):
            e = np.zeros(nj); e[j] = 1.0
            chi = G.prolong(h, k, h.levels[k].W.T @ e)
            assert abs(_energy(fe.A, chi) - sk[k][j]) / sk[k][j] < 1e-10, (k, j)


def test_compression_keeps_the_largest_and_converges():
    q = 5
    pr, fe, tree, h = _setup(q, 3, seed=13)
    b = fem.load_cellwise(pr.g[0], fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    c1, ck = G.normalized_coefficients(h, u)
    allc = np.concatenate([c1] + [ck[k] for k in sorted(ck)])
    n = allc.size
    # keeping everything changes nothing; keeping nothing gives zero
    f1, fk = G.compress(c1, ck, n)
    assert np.array_equal(np.concatenate([f1] + [fk[k] for k in sorted(fk)]), allc)
    z1, zk = G.compress(c1, ck, 0)
    assert not np.any(np.concatenate([z1] + [zk[k] for k in sorted(zk)]))
    # the kept set is the largest magnitudes
    keep = n // 20
    k1, kk = G.compress(c1, ck, keep)
    kept = np.concatenate([k1] + [kk[k] for k in sorted(kk)])
    nz = np.flatnonzero(kept)
    assert nz.size == keep
    assert np.min(np.abs(allc[nz])) >= np.max(np.abs(np.delete(allc, nz)))
    # energy error of the compressed reconstruction decreases as more is kept
    errs = []
    for frac in (0.01, 0.05, 0.2, 1.0):
        a1, ak = G.compress(c1, ck, int(round(frac * n)))
        v = G.reconstruct_normalized(h, a1, ak)
        errs.append(_energy(fe.A, u - v) / _energy(fe.A, u))
    assert errs[-1] < 1e-12
    assert all(x >= y - 1e-12 for x, y in zip(errs, errs[1:])), errs


def test_exact_basis_compresses_a_smooth_solution():
    """With the exact gamblets (the setting of Example 5.1 and Figures 10-11),
    the solution for a smooth source keeps most of its energy in the coarse
    levels, so 1% of the normalized coefficients leave an energy error of a few
    percent (white noise in the source, by contrast, spreads the energy over all
    levels)."""
    q = 6
    pr = S.rough_problem(q, 2.0, 34)
    fe = fem.assemble(pr.a)
    tree = G.Tree(q)
    h = G.exact_hierarchy(fe.A, tree)
    errs = {}
    for label, g in (("smooth", S.smooth_cell_source(q)), ("noise", pr.g[0])):
        u = fem.DirectSolver(fe.A).solve(fem.load_cellwise(g, fe.h))
        c1, ck = G.normalized_coefficients(h, u)
        n = c1.size + sum(v.size for v in ck.values())
        a1, ak = G.compress(c1, ck, int(round(0.01 * n)))
        v = G.reconstruct_normalized(h, a1, ak)
        errs[label] = _energy(fe.A, u - v) / _energy(fe.A, u)
    assert errs["smooth"] < 0.1
    assert errs["noise"] > 5 * errs["smooth"]
