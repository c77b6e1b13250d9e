"""Pins of the oracle's level-q gamblets from the localized mass inverse
(Algorithm 2, first lines; Definition 5.2; Algorithm 1's exact level-q
gamblets as the limit of a patch covering the grid).

* the assembled mass matrix is h^2 T (x) T, T = tridiag(1, 4, 1)/6 the 1-D
  linear-element mass matrix over h (textbook closed form);
* on a box patch the patch mass matrix is a Kronecker product too, so every
  localized column is the outer product of two 1-D banded solves (an
  independent route: scipy's banded solver on the 1-D patches);
* a patch covering the grid gives M^-1 exactly; the truncation error decays
  geometrically with rho (M has condition number <= 9);
* the defining property: int psi_i phi_j = delta_ij for j in the patch;
* whatever rho, psi^(q),loc span the nodal space, so the Galerkin solution in
  that basis, Minv A^(q),loc^-1 g^(q),loc, is the finite-element solution
  A^-1 b: this fails if A^(q),loc or g^(q),loc has a transposed or missing
  factor;
* the gamblet hierarchy started from these level-q gamblets (exact for
  small q, localized with patch radius 3) returns the finite-element
  solution.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import synthetic as S
from oracle import fem
from oracle import gamblets as G
from oracle import mass_inverse as MI


def _1d_mass(m, h):
    return h * (np.diag(np.full(m, 4.0)) + np.diag(np.ones(m - 1), 1) + np.diag(np.ones(m - 1), -1)) / 6.0


@pytest.mark.parametrize("n", [4, 7, 16])
def test_mass_matrix_is_kronecker_product(n):
    h = 1.0 / n
    M = MI.mass_matrix(n).toarray()
    T = _1d_mass(n - 1, h)
    assert np.abs(M - np.kron(T, T)).max() < 1e-15
    # an interior hat function integrates to h^2: the row sums away from the
    # boundary
    ix = np.arange(1, n - 2)
    rows = (ix[:, None] * (n - 1) + ix[None, :]).ravel()
    assert np.abs(M[rows].sum(axis=1) - h * h).max() < 1e-15


@pytest.mark.parametrize("n,rho", [(8, 1), (8, 2), (16, 3)])
def test_localized_columns_are_outer_products_of_1d_solves(n, rho):
    h = 1.0 / n
    m = n - 1
    Minv = MI.localized_mass_inverse(MI.mass_matrix(n), n, rho).toarray()
    T = _1d_mass(m, h)
    rng = np.random.default_rng(1)
    for i in list(rng.choice(m * m, 12, replace=False)) + [0, m - 1, m * m - 1]:
        ix, iy = divmod(int(i), m)
        cols = []
        for c in (ix, iy):
            lo, hi = max(0, c - rho), min(m, c + rho + 1)
            sz = hi - lo
            ab = np.zeros((3, sz))
            ab[0, 1:] = np.diag(T, 1)[lo:hi - 1]
            ab[1, :] = np.diag(T)[lo:hi]
            ab[2, :-1] = np.diag(T, -1)[lo:hi - 1]
            e = np.zeros(sz)
            e[c - lo] = 1.0
            y = np.zeros(m)
            y[lo:hi] = sla.solve_banded((1, 1), ab, e)
            cols.append(y)
        ref = np.outer(cols[0], cols[1]).ravel()
        assert np.abs(Minv[:, i] - ref).max() <= 1e-12 * np.abs(ref).max(), i


def test_full_patch_is_the_inverse_and_truncation_decays():
    n = 12
    M = MI.mass_matrix(n)
    Mi = np.linalg.inv(M.toarray())
    full = MI.localized_mass_inverse(M, n, n).toarray()
    assert np.abs(full - Mi).max() / np.abs(Mi).max() < 1e-12
    errs = [np.abs(MI.localized_mass_inverse(M, n, r).toarray() - Mi).max() / np.abs(Mi).max()
            for r in (1, 2, 3, 4)]
    # exponential decay of M^-1 away from the diagonal (1-D factor
    # (sqrt 3 - 2)^d, about 0.27 per node step)
    for a, b in zip(errs, errs[1:]):
        assert b < 0.45 * a, errs


@pytest.mark.parametrize("rho", [1, 3])
def test_gamblets_are_dual_to_the_nodal_basis_on_their_patch(rho):
    n = 10
    M = MI.mass_matrix(n)
    Minv = MI.localized_mass_inverse(M, n, rho)
    D = (M @ Minv).toarray()   # D[j, i] = int phi_j psi_i
    m = n - 1
    for i in range(m * m):
        p = MI.patch_nodes(n, i, rho)
        e = (p == i).astype(float)
        assert np.abs(D[p, i] - e).max() < 1e-13, i


@pytest.mark.parametrize("rho", [1, 2, 3])
def test_solution_in_the_level_q_basis_is_the_fe_solution(rho):
    q = 4
    pr = S.rough_problem(q, 2.0, 41)
    fe = fem.assemble(pr.a)
    b = fem.load_cellwise(pr.g[0], fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    lq = MI.level_q_gamblets(fe, rho)
    U = np.linalg.solve(lq.A.toarray(), MI.level_q_load(lq, b))
    v = MI.level_q_to_nodal(lq, U)
    assert np.linalg.norm(v - u) / np.linalg.norm(u) < 1e-10
    # A^(q),loc is symmetric positive definite with the stencil width the
    # patches imply (2 rho + 1 node steps)
    Aq = lq.A.toarray()
    assert np.abs(Aq - Aq.T).max() <= 1e-14 * np.abs(Aq).max()
    assert np.linalg.eigvalsh(Aq).min() > 0
    st = MI.stencil_rows(lq, np.arange(Aq.shape[0]))
    assert np.count_nonzero(np.abs(st).sum(axis=0)) == (4 * rho + 3) ** 2


def test_hierarchy_from_mass_inverse_gamblets_returns_the_fe_solution():
    """Algorithm 1 with its own level-q gamblets (exact mass inverse) and
    Algorithm 2 with the localized ones (patch radius 3 at every level): the
    exact hierarchy reproduces A^-1 b directly; the localized one, used as the
    preconditioner of a refinement loop on the nodal residual, converges to
    it."""
    q = 4
    pr = S.rough_problem(q, 1.5, 42)
    fe = fem.assemble(pr.a)
    b = fem.load_cellwise(pr.g[0], fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    tree = G.Tree(q)
    exact = MI.level_q_gamblets(fe, fe.n)
    h = G.exact_hierarchy(exact.A, tree)
    v = MI.level_q_to_nodal(exact, G.solve(h, MI.level_q_load(exact, b)))
    assert np.linalg.norm(v - u) / np.linalg.norm(u) < 1e-10
    loc = MI.level_q_gamblets(fe, 3)
    hl = G.localized_hierarchy(loc.A, tree, 3)
    v = np.zeros_like(b)
    for _ in range(30):
        r = b - fe.A @ v
        v = v + MI.level_q_to_nodal(loc, G.solve(hl, MI.level_q_load(loc, r)))
    assert np.linalg.norm(v - u) / np.linalg.norm(u) < 1e-10
