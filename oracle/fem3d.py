"""Q1 (trilinear) finite elements for -div(a grad u) = g on the unit cube (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The problem of Section 1 is stated for any dimension d; this is its d = 3
discretisation in the manner of Section 5.1: ``a`` constant on every cubic
cell, the nodal basis spanned on each cell by the products of the 1-D hat
functions (the three-dimensional analogue of Example 5.1's {1, x1, x2, x1 x2}),
zero Dirichlet data lifted onto the load when given.

Mesh: ``n`` cells per dimension, ``h = 1/n``; node ``(i, j, l)`` at
``(i h, j h, l h)``, interior nodes ``1 <= i, j, l <= n-1`` numbered
``((i-1)(n-1) + (j-1))(n-1) + (l-1)``.  Cell ``(ex, ey, ez)`` has the corner
nodes ``(ex+dx, ey+dy, ez+dz)``, local index ``4 dx + 2 dy + dz``.

Element matrices come from the 1-D element matrices of a unit interval,
stiffness [[1, -1], [-1, 1]] and mass [[2, 1], [1, 2]] / 6: the gradient of a
product of hats splits into three products, so on a cube of side h the
stiffness is h (K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1) and the mass
h^3 (M1 x M1 x M1) (Kronecker products in the local order above).

Pins (tests/test_oracle_3d.py): the element matrices against Gauss quadrature
of the trilinear basis written out term by term, the constant-coefficient
solution against the three-dimensional sine transform, and the load against
quadrature.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

K1 = np.array([[1.0, -1.0], [-1.0, 1.0]])
M1 = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
K_UNIT3 = (np.kron(np.kron(K1, M1), M1) + np.kron(np.kron(M1, K1), M1) + np.kron(np.kron(M1, M1), K1))
M_UNIT3 = np.kron(np.kron(M1, M1), M1)


def cell_nodes(n: int) -> np.ndarray:
    """[n^3, 8] global node ids (node (i,j,l) -> (i (n+1) + j)(n+1) + l), cell id (ex n + ey) n + ez."""
    e = np.arange(n)
    ex, ey, ez = np.meshgrid(e, e, e, indexing="ij")
    s = n + 1
    cols = []
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                cols.append(((ex + dx) * s + (ey + dy)) * s + (ez + dz))
    return np.stack([c.ravel() for c in cols], axis=1)


def interior_ids(n: int) -> np.ndarray:
    i = np.arange(1, n)
    I, J, L = np.meshgrid(i, i, i, indexing="ij")
    return ((I * (n + 1) + J) * (n + 1) + L).ravel()


def boundary_mask(n: int) -> np.ndarray:
    m = np.zeros((n + 1,) * 3, dtype=bool)
    m[0], m[-1] = True, True
    m[:, 0], m[:, -1] = True, True
    m[:, :, 0], m[:, :, -1] = True, True
    return m.ravel()


@dataclass
class FEProblem3:
    n: int
    h: float
    A: sp.csc_matrix          # interior x interior
    A_IB: sp.csr_matrix       # interior x boundary
    interior: np.ndarray
    boundary: np.ndarray


def _global(n: int, elem: np.ndarray, weights: np.ndarray) -> sp.csr_matrix:
    cn = cell_nodes(n)
    rows = np.repeat(cn, 8, axis=1).ravel()
    cols = np.tile(cn, (1, 8)).ravel()
    vals = (weights[:, None, None] * elem[None, :, :]).ravel()
    nn = (n + 1) ** 3
    return sp.coo_matrix((vals, (rows, cols)), shape=(nn, nn)).tocsr()


def assemble(a: np.ndarray) -> FEProblem3:
    """A = h sum_e a_e K_unit3 over the cells (first step of Algorithms 1 and 2, d = 3)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    assert a.shape == (n, n, n)
    h = 1.0 / n
    full = _global(n, h * K_UNIT3, a.ravel())
    inner = interior_ids(n)
    bnd = np.flatnonzero(boundary_mask(n))
    return FEProblem3(n=n, h=h, A=full[inner][:, inner].tocsc(), A_IB=full[inner][:, bnd].tocsr(),
                      interior=inner, boundary=bnd)


def load_cellwise(g: np.ndarray, h: float) -> np.ndarray:
    """b_i = int phi_i g = (h^3 / 8) sum over the eight cells around node i of g_e (g [n]^3 or [nrhs][n]^3)."""
    g = np.asarray(g, dtype=np.float64)
    single = g.ndim == 3
    if single:
        g = g[None]
    nrhs, n = g.shape[0], g.shape[1]
    out = np.zeros((nrhs, n + 1, n + 1, n + 1))
    q = h ** 3 / 8.0 * g
    for dx in (0, 1):
        for dy in (0, 1):
            for dz in (0, 1):
                out[:, dx:dx + n, dy:dy + n, dz:dz + n] += q
    b = out[:, 1:-1, 1:-1, 1:-1].reshape(nrhs, -1)
    return b[0] if single else b


def load_nodal(gn: np.ndarray, h: float) -> np.ndarray:
    """b = M g for a nodal source given at the interior nodes ([n-1]^3, zero on the boundary)."""
    m = gn.shape[0]
    n = m + 1
    full = np.zeros((n + 1,) * 3)
    full[1:-1, 1:-1, 1:-1] = gn
    M = _global(n, h ** 3 * M_UNIT3, np.ones(n ** 3))
    return (M @ full.ravel())[interior_ids(n)]


def lift(fe: FEProblem3, b: np.ndarray, u_boundary: np.ndarray | None) -> np.ndarray:
    """b - A_IB u_B for Dirichlet values u_B (any array of (n+1)^3 nodal values per right-hand side)."""
    if u_boundary is None:
        return b
    ub = np.asarray(u_boundary, dtype=np.float64).reshape(-1, (fe.n + 1) ** 3)[:, fe.boundary]
    out = np.atleast_2d(b) - (fe.A_IB @ ub.T).T
    return out[0] if np.ndim(b) == 1 else out


def full_nodal(fe: FEProblem3, u_int: np.ndarray, u_boundary: np.ndarray | None = None) -> np.ndarray:
    full = np.zeros((fe.n + 1) ** 3)
    if u_boundary is not None:
        full[fe.boundary] = np.asarray(u_boundary, dtype=np.float64).ravel()[fe.boundary]
    full[fe.interior] = u_int
    return full.reshape((fe.n + 1,) * 3)
