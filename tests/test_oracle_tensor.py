"""Pins of the oracle's tensor-coefficient assembly (the symmetric matrix
a(x) of Section 1 in two dimensions): the element matrices against Gauss
quadrature of the bilinear basis, the isotropic case against the scalar
assembly, a constant diagonal anisotropic tensor against the sine transform,
linear functions reproduced for a constant full tensor (which pins the
off-diagonal part), and the exact hierarchy of Algorithm 1 reproducing the
direct solve."""
import numpy as np
import scipy.fft as sfft

from oracle import fem
from oracle import gamblets as G


def _spd_field(n, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0, np.pi, (n, n))
    l1, l2 = np.exp(rng.standard_normal((n, n))), np.exp(rng.standard_normal((n, n)))
    c, s = np.cos(t), np.sin(t)
    return np.stack([l1 * c * c + l2 * s * s, (l1 - l2) * c * s, l1 * s * s + l2 * c * c], axis=-1)


def test_tensor_element_matches_quadrature():
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    loc = [(0, 0), (1, 0), (0, 1), (1, 1)]
    hat = lambda d, s: 1.0 - s if d == 0 else s
    dhat = lambda d: -1.0 if d == 0 else 1.0
    a11, a12, a22 = 2.0, 0.7, 1.3
    A = np.array([[a11, a12], [a12, a22]])
    K = np.zeros((4, 4))
    for x in g:
        for y in g:
            grads = [np.array([dhat(dx) * hat(dy, y), hat(dx, x) * dhat(dy)]) for dx, dy in loc]
            for i in range(4):
                for j in range(4):
                    K[i, j] += 0.25 * grads[i] @ A @ grads[j]
    Kxx, Kyy, Ks = fem.tensor_element_parts()
    assert np.allclose(K, a11 * Kxx + a22 * Kyy + a12 * Ks, atol=1e-14)
    assert np.allclose(Kxx + Kyy, fem.K_UNIT, atol=1e-15)


def test_isotropic_tensor_equals_scalar_assembly():
    n = 8
    a = np.exp(np.random.default_rng(1).standard_normal((n, n)))
    a3 = np.stack([a, np.zeros_like(a), a], axis=-1)
    assert abs(fem.assemble_tensor(a3).A - fem.assemble(a).A).max() < 1e-14


def test_diagonal_anisotropic_tensor_matches_sine_transform():
    """a = diag(a11, a22) constant: A = a11 K x M + a22 M x K (1-D interior
    stiffness K = tridiag(-1, 2, -1) / h, mass M = h tridiag(1, 4, 1) / 6),
    diagonalised by the orthonormal DST-I."""
    n, a11, a22 = 16, 3.0, 0.25
    h = 1.0 / n
    a3 = np.zeros((n, n, 3))
    a3[..., 0], a3[..., 2] = a11, a22
    fe = fem.assemble_tensor(a3)
    b = fem.load_cellwise(np.random.default_rng(2).standard_normal((n, n)), h)
    u = fem.DirectSolver(fe.A).solve(b)
    th = np.arange(1, n) * np.pi / n
    kap = (2.0 - 2.0 * np.cos(th)) / h
    mu = h * (4.0 + 2.0 * np.cos(th)) / 6.0
    lam = a11 * kap[:, None] * mu[None, :] + a22 * mu[:, None] * kap[None, :]
    U = sfft.idstn(sfft.dstn(b.reshape(n - 1, n - 1), type=1, norm="ortho") / lam, type=1, norm="ortho")
    assert np.linalg.norm(U.ravel() - u) <= 1e-12 * np.linalg.norm(u)


def test_constant_full_tensor_reproduces_linear_functions():
    n = 10
    a3 = np.zeros((n, n, 3))
    a3[..., 0], a3[..., 1], a3[..., 2] = 2.0, -0.8, 1.1
    fe = fem.assemble_tensor(a3)
    x = np.arange(n + 1) / n
    X, Y = np.meshgrid(x, x, indexing="ij")
    lin = 0.5 - 2.0 * X + 3.0 * Y
    u = fem.DirectSolver(fe.A).solve(fem.lift(fe, np.zeros(fe.A.shape[0]), lin))
    assert np.abs(fem.full_nodal(fe, u, lin) - lin).max() < 1e-12


def test_exact_hierarchy_with_tensor_coefficient():
    q = 4
    n = 1 << q
    fe = fem.assemble_tensor(_spd_field(n, 3))
    h = G.exact_hierarchy(fe.A, G.Tree(q))
    b = fem.load_cellwise(np.random.default_rng(4).standard_normal((n, n)), fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    assert np.linalg.norm(G.solve(h, b) - u) <= 1e-12 * np.linalg.norm(u)
