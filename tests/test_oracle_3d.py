"""Pins of the three-dimensional oracle (the problem of Section 1 with d = 3;
Table 1 and the constructions of Section 4 are written for any d): trilinear
element matrices against Gauss quadrature, the constant-coefficient solution
against the three-dimensional sine transform, the reproduction of linear
functions with Dirichlet data, the eight-child tree, and the exact hierarchy
of Algorithm 1 on it (subband sum = direct solve, the closed form of
Theorem 4.8, A-orthogonal subbands, independence of the W construction)."""
import numpy as np
import pytest
import scipy.fft as sfft
import scipy.sparse as sp

from oracle import fem
from oracle import fem3d
from oracle import gamblets as G


def _hat(d, s):
    return 1.0 - s if d == 0 else s


def _dhat(d, s):
    return -1.0 if d == 0 else 1.0


def test_element_matrices_match_quadrature():
    """Trilinear basis written out term by term, integrated with two Gauss
    points per direction (exact for these degree-2 integrands)."""
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    w = np.array([0.5, 0.5])
    loc = [(dx, dy, dz) for dx in (0, 1) for dy in (0, 1) for dz in (0, 1)]
    K = np.zeros((8, 8))
    M = np.zeros((8, 8))
    for ix, x in enumerate(g):
        for iy, y in enumerate(g):
            for iz, z in enumerate(g):
                wt = w[ix] * w[iy] * w[iz]
                phi = [_hat(a, x) * _hat(b, y) * _hat(c, z) for a, b, c in loc]
                grad = [np.array([_dhat(a, x) * _hat(b, y) * _hat(c, z), _hat(a, x) * _dhat(b, y) * _hat(c, z),
                                  _hat(a, x) * _hat(b, y) * _dhat(c, z)]) for a, b, c in loc]
                for i in range(8):
                    for j in range(8):
                        K[i, j] += wt * grad[i] @ grad[j]
                        M[i, j] += wt * phi[i] * phi[j]
    assert np.allclose(K, fem3d.K_UNIT3, atol=1e-14)
    assert np.allclose(M, fem3d.M_UNIT3, atol=1e-15)
    assert abs(K.sum()) < 1e-13   # constants have no energy


@pytest.mark.parametrize("n", [4, 8])
def test_constant_coefficient_matches_sine_transform(n):
    """a = 1: the interior stiffness is K x M x M + M x K x M + M x M x K with the
    1-D matrices K = tridiag(-1, 2, -1) / h, M = h tridiag(1, 4, 1) / 6, which the
    orthonormal DST-I diagonalises: u = S diag(1 / lambda) S b."""
    h = 1.0 / n
    fe = fem3d.assemble(np.ones((n, n, n)))
    b = fem3d.load_cellwise(np.random.default_rng(n).standard_normal((n, n, n)), h)
    u = fem.DirectSolver(fe.A).solve(b)
    th = np.arange(1, n) * np.pi / n
    kap = (2.0 - 2.0 * np.cos(th)) / h
    mu = h * (4.0 + 2.0 * np.cos(th)) / 6.0
    lam = (kap[:, None, None] * mu[None, :, None] * mu[None, None, :] + mu[:, None, None] * kap[None, :, None]
           * mu[None, None, :] + mu[:, None, None] * mu[None, :, None] * kap[None, None, :])
    B = b.reshape(n - 1, n - 1, n - 1)
    U = sfft.idstn(sfft.dstn(B, type=1, norm="ortho") / lam, type=1, norm="ortho")
    assert np.linalg.norm(U.ravel() - u) <= 1e-12 * np.linalg.norm(u)


def test_linear_functions_are_reproduced_with_dirichlet_data():
    """Q1 elements contain the linear functions: with g = 0, a constant
    coefficient and boundary values of u = 1 + x + 2y - 3z, the discrete
    solution is u (each interior row of A sums a gradient against the
    integral of the basis gradient, zero for a linear u)."""
    n = 6
    a = np.full((n, n, n), 2.5)
    fe = fem3d.assemble(a)
    x = np.arange(n + 1) / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    lin = 1.0 + X + 2.0 * Y - 3.0 * Z
    b = fem3d.lift(fe, np.zeros(fe.A.shape[0]), lin)
    u = fem.DirectSolver(fe.A).solve(b)
    assert np.abs(fem3d.full_nodal(fe, u, lin) - lin).max() < 1e-12


def test_nodal_load_is_the_tensor_mass_matrix():
    n = 5
    h = 1.0 / n
    gn = np.random.default_rng(4).standard_normal((n - 1,) * 3)
    Mh = sp.diags([np.full(n - 2, 1.0), np.full(n - 1, 4.0), np.full(n - 2, 1.0)], [-1, 0, 1]) * (h / 6.0)
    M3 = sp.kron(sp.kron(Mh, Mh), Mh)
    assert np.allclose(fem3d.load_nodal(gn, h), M3 @ gn.ravel(), atol=1e-16)


def test_cell_load_integrates_the_hats():
    """int phi_i over a cell is h^3 / 8, so a cell source gives (h^3/8) sum of its eight cells."""
    n = 4
    h = 1.0 / n
    g = np.zeros((n, n, n))
    g[1, 2, 0] = 1.0
    b = fem3d.load_cellwise(g, h).reshape((n - 1,) * 3)
    expect = np.zeros((n + 1,) * 3)
    expect[1:3, 2:4, 0:2] = h ** 3 / 8.0
    assert np.allclose(b, expect[1:-1, 1:-1, 1:-1], atol=1e-18)


def test_tree3_child_counts():
    tree = G.Tree3(2)
    assert tree.size(2) == 27 and tree.size(1) == 8
    counts = sorted(len(c) for c in tree.children[2])
    assert counts == [1, 2, 2, 2, 4, 4, 4, 8]
    tree1 = G.Tree3(3, offset=1)
    assert tree1.size(3) == 512 and all(len(c) == 8 for c in tree1.children[3])
    assert G.Tree3(3).box(2, 0, 1).size == 8 and G.Tree3(3).box(2, 21, 1).size == 27


@pytest.mark.parametrize("offset", [0, 1])
def test_exact_hierarchy_3d(offset):
    q = 3
    n = (1 << q) + offset
    rng = np.random.default_rng(10 + offset)
    a = np.exp(rng.standard_normal((n, n, n)))
    fe = fem3d.assemble(a)
    tree = G.Tree3(q, offset=offset)
    h = G.exact_hierarchy(fe.A, tree)
    b = fem3d.load_cellwise(rng.standard_normal((n, n, n)), fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    # Theorem 4.15: the subband sum is the solution
    assert np.linalg.norm(G.solve(h, b) - u) <= 1e-12 * np.linalg.norm(u)
    # closed form of Theorem 4.8: A^(k) = (pi A^-1 pi^T)^-1 with pi the aggregation from level q
    Ainv = np.linalg.inv(fe.A.toarray())
    P = sp.identity(tree.size(q), format="csr")
    for k in range(q, 1, -1):
        P = tree.pi(k) @ P
        Ak = np.linalg.inv(P.toarray() @ Ainv @ P.toarray().T)
        assert np.allclose(h.levels[k - 1].A, Ak, rtol=1e-9, atol=1e-9 * np.abs(Ak).max())
    # the subband parts are A-orthogonal
    parts = G.subbands(h, b)
    A = fe.A.toarray()
    for i in range(len(parts)):
        for j in range(i):
            num = parts[i] @ A @ parts[j]
            assert abs(num) <= 1e-10 * np.sqrt((parts[i] @ A @ parts[i]) * (parts[j] @ A @ parts[j]))
    # Constructions 4.11 and 4.13 give the same R and A^(k)
    h1 = G.exact_hierarchy(fe.A, tree, construction=1)
    for k in range(q, 1, -1):
        assert np.allclose(h1.levels[k].R, h.levels[k].R, atol=1e-12)
