"""Pins of the finite-element oracle against facts that do not come from it.

* Example 5.1's printed contrast (golden fixture).
* Element matrices re-derived by Gauss quadrature of the bilinear basis.
* Constant-coefficient solutions in closed form (orthonormal sine transform).
* Reproduction of constants and of linear functions (consistency of Q1).
* The adjoint gradient against a cancellation-free finite difference and the
  plain two-sided difference of J.
"""
import os

import numpy as np
import pytest
import scipy.fft as sfft

import synthetic as S
from oracle import fem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden_number(name):
    with open(os.path.join(GOLDEN, name)) as f:
        vals = [ln for ln in f.read().splitlines() if ln.strip() and not ln.startswith("#")]
    return float(vals[0])


def test_example51_contrast_matches_paper():
    a = S.example51_coefficient()
    assert a.shape == (65, 65)
    assert round(a.max() / a.min()) == _golden_number("example51_contrast.txt")


def _bilinear_grad(xi, eta):
    # local nodes (0,0),(1,0),(0,1),(1,1) on the unit square
    phi = np.array([(1 - xi) * (1 - eta), xi * (1 - eta), (1 - xi) * eta, xi * eta])
    dx = np.array([-(1 - eta), (1 - eta), -eta, eta])
    dy = np.array([-(1 - xi), -xi, (1 - xi), xi])
    return phi, dx, dy


def test_element_matrices_by_quadrature():
    gp, gw = np.polynomial.legendre.leggauss(3)
    gp = 0.5 * (gp + 1.0)
    gw = 0.5 * gw
    K = np.zeros((4, 4))
    M = np.zeros((4, 4))
    for x, wx in zip(gp, gw):
        for y, wy in zip(gp, gw):
            phi, dx, dy = _bilinear_grad(x, y)
            K += wx * wy * (np.outer(dx, dx) + np.outer(dy, dy))
            M += wx * wy * np.outer(phi, phi)
    np.testing.assert_allclose(fem.K_UNIT, K, atol=1e-15)
    np.testing.assert_allclose(fem.M_UNIT, M, atol=1e-15)


@pytest.mark.parametrize("q", [4, 6])
def test_constant_coefficient_closed_form(q):
    """For a = 1 the interior stiffness is 3 I - (I + T)(I + T)/3 with T the 1-D
    neighbour-sum operator, diagonalised by the orthonormal DST-I."""
    n = 1 << q
    rng = np.random.default_rng(q)
    b = rng.standard_normal((n - 1, n - 1))
    th = np.arange(1, n) * np.pi / n
    c = 2.0 * np.cos(th)
    lam = 3.0 - (1.0 + c[:, None]) * (1.0 + c[None, :]) / 3.0
    u_ref = sfft.dstn(sfft.dstn(b, type=1, norm="ortho") / lam, type=1, norm="ortho")
    fe = fem.assemble(np.ones((n, n)))
    u = fem.DirectSolver(fe.A).solve(b.ravel())
    assert np.linalg.norm(u - u_ref.ravel()) / np.linalg.norm(u_ref) < 1e-13


def test_mass_closed_form():
    """Q1 mass matrix on a uniform grid: symbol (h^2/9)(2 + cos t1)(2 + cos t2)."""
    n = 16
    h = 1.0 / n
    rng = np.random.default_rng(3)
    g = rng.standard_normal((n - 1, n - 1))
    th = np.arange(1, n) * np.pi / n
    sym = (h * h / 9.0) * (2.0 + np.cos(th))[:, None] * (2.0 + np.cos(th))[None, :]
    ref = sfft.dstn(sym * sfft.dstn(g, type=1, norm="ortho"), type=1, norm="ortho")
    np.testing.assert_allclose(fem.load_nodal(g, h), ref.ravel(), rtol=0, atol=1e-15)


def test_cell_load_integrates_constant():
    """sum_i b_i = int g * (fraction of each cell's basis mass on interior nodes)."""
    n = 8
    h = 1.0 / n
    b = fem.load_cellwise(np.ones((n, n)), h)
    # every interior node collects 4 quarter-cells
    np.testing.assert_allclose(b, np.full((n - 1) ** 2, h * h), rtol=1e-15)


def test_constants_and_linear_functions_reproduced():
    n = 16
    rng = np.random.default_rng(0)
    a = np.exp(rng.standard_normal((n, n)))
    xs = np.arange(n + 1) / n
    X, Y = np.meshgrid(xs, xs, indexing="ij")
    ub = np.full((n + 1, n + 1), 2.5)
    u = fem.solve(a, np.zeros((n, n)), ub)
    np.testing.assert_allclose(u, 2.5, atol=1e-12)
    lin = 0.3 + X - 2.0 * Y
    u = fem.solve(np.full((n, n), 7.0), np.zeros((n, n)), lin)
    np.testing.assert_allclose(u, lin, atol=1e-12)


def test_direct_solver_residual():
    pr = S.rough_problem(6, 2.0, 11)
    fe = fem.assemble(pr.a)
    b = fem.load_cellwise(pr.g[0], fe.h)
    u = fem.DirectSolver(fe.A).solve(b)
    assert np.linalg.norm(fe.A @ u - b) / np.linalg.norm(b) < 1e-13


def test_adjoint_against_woodbury_fd():
    pr = S.adjoint_problem(q=5, tag=77)
    u_obs = fem.solve(pr.extra["a_obs"], pr.g[0])[1:-1, 1:-1].ravel()
    _, J, ga, gg = fem.adjoint(pr.a, pr.g[0], u_obs)
    cells = pr.extra["fd_cells"]
    fd = fem.fd_log_a(pr.a, pr.g[0], u_obs, cells, step=1e-6)
    ref = ga.ravel()[cells]
    assert np.linalg.norm(fd - ref) / np.linalg.norm(ref) < 1e-7


def test_woodbury_fd_against_plain_difference():
    """The Woodbury update must agree with re-solving at a_e e^{+-s} (large step)."""
    pr = S.adjoint_problem(q=4, tag=78)
    u_obs = np.zeros(15 * 15)
    cells = pr.extra["fd_cells"][:6]
    s = 1e-3
    fd = fem.fd_log_a(pr.a, pr.g[0], u_obs, cells, step=s)
    plain = []
    for c in cells:
        Js = []
        for sgn in (1, -1):
            a2 = pr.a.copy().ravel()
            a2[c] *= np.exp(sgn * s)
            u = fem.solve(a2.reshape(pr.a.shape), pr.g[0])[1:-1, 1:-1].ravel()
            Js.append(0.5 * u @ u)
        plain.append((Js[0] - Js[1]) / (2 * s))
    np.testing.assert_allclose(fd, plain, rtol=1e-7)


def test_source_gradient_is_exact_difference():
    """J is quadratic in g: the central difference with any step is exact."""
    pr = S.adjoint_problem(q=4, tag=79)
    u_obs = np.zeros(15 * 15)
    _, _, _, gg = fem.adjoint(pr.a, pr.g[0], u_obs)
    for c in (0, 37, 200):
        Js = []
        for sgn in (1, -1):
            g2 = pr.g[0].copy().ravel()
            g2[c] += sgn * 0.5
            u = fem.solve(pr.a, g2.reshape(pr.a.shape))[1:-1, 1:-1].ravel()
            Js.append(0.5 * u @ u)
        assert abs((Js[0] - Js[1]) / 1.0 - gg.ravel()[c]) < 1e-12 * max(1.0, abs(gg.ravel()[c]))
