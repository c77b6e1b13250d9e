"""Q1 finite elements for -div(a grad u) = g on the unit square (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The discrete problem is the one of Section 5.1: find u in the span of the
nodal basis with <phi_j, u>_a = int phi_j g for every interior node j
(discrete weak form of the problem of Section 1), with ``a`` constant on
every square cell (Section 5.1) and the nodal basis spanned by
{1, x1, x2, x1 x2} on each cell (Example 5.1).  Boundary values are Dirichlet
data, zero in the paper; non-zero data are lifted onto the load.

Mesh: ``n`` cells per dimension, ``h = 1/n``; node ``(i, j)`` sits at
``(i h, j h)``, ``0 <= i, j <= n``; interior nodes ``1 <= i, j <= n-1`` are
numbered ``(i-1)(n-1) + (j-1)``.  Cell ``(ex, ey)`` has corner nodes
``(ex, ey), (ex+1, ey), (ex, ey+1), (ex+1, ey+1)`` in that local order.

Pins (tests): constant-coefficient closed form via the sine transform,
brute-force element integration by quadrature, the Example 5.1 load, and
the gradient against a cancellation-free finite difference.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# Element matrices of the bilinear element on a square, local node order
# (0,0), (1,0), (0,1), (1,1).  Stiffness is independent of the side length in
# two dimensions; the mass matrix scales with h^2.
K_UNIT = np.array([[4.0, -1.0, -1.0, -2.0],
                   [-1.0, 4.0, -2.0, -1.0],
                   [-1.0, -2.0, 4.0, -1.0],
                   [-2.0, -1.0, -1.0, 4.0]]) / 6.0
M_UNIT = np.array([[4.0, 2.0, 2.0, 1.0],
                   [2.0, 4.0, 1.0, 2.0],
                   [2.0, 1.0, 4.0, 2.0],
                   [1.0, 2.0, 2.0, 4.0]]) / 36.0


def cell_nodes(n: int) -> np.ndarray:
    """[n*n, 4] global node ids (node (i,j) -> i*(n+1)+j) of every cell, cell id ex*n+ey."""
    ex, ey = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ex = ex.ravel()
    ey = ey.ravel()
    s = n + 1
    return np.stack([ex * s + ey, (ex + 1) * s + ey, ex * s + ey + 1, (ex + 1) * s + ey + 1], axis=1)


def interior_ids(n: int) -> np.ndarray:
    """Global ids of interior nodes in interior order (i-1)(n-1)+(j-1)."""
    i, j = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="ij")
    return (i * (n + 1) + j).ravel()


def boundary_mask(n: int) -> np.ndarray:
    m = np.zeros((n + 1, n + 1), dtype=bool)
    m[0, :] = m[-1, :] = m[:, 0] = m[:, -1] = True
    return m.ravel()


@dataclass
class FEProblem:
    n: int
    h: float
    A_full: sp.csr_matrix      # all (n+1)^2 nodes
    A: sp.csc_matrix           # interior x interior
    A_IB: sp.csr_matrix        # interior x boundary
    interior: np.ndarray
    boundary: np.ndarray


def assemble(a: np.ndarray, h: float | None = None) -> FEProblem:
    """Stiffness matrix A = sum_e a_e K_unit over cells (Algorithm 1, step 2)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    assert a.shape == (n, n)
    if h is None:
        h = 1.0 / n
    cn = cell_nodes(n)
    rows = np.repeat(cn, 4, axis=1).ravel()
    cols = np.tile(cn, (1, 4)).ravel()
    vals = (a.ravel()[:, None, None] * K_UNIT[None, :, :]).ravel()
    nn = (n + 1) ** 2
    A_full = sp.coo_matrix((vals, (rows, cols)), shape=(nn, nn)).tocsr()
    inner = interior_ids(n)
    bnd = np.flatnonzero(boundary_mask(n))
    A = A_full[inner][:, inner].tocsc()
    A_IB = A_full[inner][:, bnd].tocsr()
    return FEProblem(n=n, h=h, A_full=A_full, A=A, A_IB=A_IB, interior=inner, boundary=bnd)


# Tensor-valued coefficients (the symmetric matrix a(x) of Section 1): per
# cell a constant SPD matrix [[a11, a12], [a12, a22]].  On a cell the local
# basis is hat_dx(x) hat_dy(y) (local index dx + 2 dy), so
#   int dx phi_i dx phi_j = k1[dx_i][dx_j] m1[dy_i][dy_j],
#   int dy phi_i dy phi_j = m1[dx_i][dx_j] k1[dy_i][dy_j],
#   int dx phi_i dy phi_j = c1[dx_i][dx_j] c1[dy_j][dy_i],
# with the unit-interval matrices k1 (stiffness), m1 (mass) and
# c1[a][b] = int hat_a' hat_b = (+1/2 for a = 1, -1/2 for a = 0); the cell
# side cancels in two dimensions.
K1_1D = np.array([[1.0, -1.0], [-1.0, 1.0]])
M1_1D = np.array([[2.0, 1.0], [1.0, 2.0]]) / 6.0
C1_1D = np.array([[-0.5, -0.5], [0.5, 0.5]])


def tensor_element_parts():
    """(Kxx, Kyy, Kxy + Kyx) over the local nodes (0,0), (1,0), (0,1), (1,1)."""
    loc = [(0, 0), (1, 0), (0, 1), (1, 1)]
    Kxx = np.array([[K1_1D[a[0], b[0]] * M1_1D[a[1], b[1]] for b in loc] for a in loc])
    Kyy = np.array([[M1_1D[a[0], b[0]] * K1_1D[a[1], b[1]] for b in loc] for a in loc])
    Kxy = np.array([[C1_1D[a[0], b[0]] * C1_1D[b[1], a[1]] for b in loc] for a in loc])
    return Kxx, Kyy, Kxy + Kxy.T


def assemble_tensor(a3: np.ndarray) -> FEProblem:
    """Stiffness of -div(a grad u) with a per-cell symmetric tensor a3[ex][ey] = (a11, a12, a22)."""
    a3 = np.asarray(a3, dtype=np.float64)
    n = a3.shape[0]
    assert a3.shape == (n, n, 3)
    Kxx, Kyy, Ks = tensor_element_parts()
    cn = cell_nodes(n)
    rows = np.repeat(cn, 4, axis=1).ravel()
    cols = np.tile(cn, (1, 4)).ravel()
    a11, a12, a22 = (a3[..., i].ravel()[:, None, None] for i in range(3))
    vals = (a11 * Kxx[None] + a22 * Kyy[None] + a12 * Ks[None]).ravel()
    nn = (n + 1) ** 2
    A_full = sp.coo_matrix((vals, (rows, cols)), shape=(nn, nn)).tocsr()
    inner = interior_ids(n)
    bnd = np.flatnonzero(boundary_mask(n))
    return FEProblem(n=n, h=1.0 / n, A_full=A_full, A=A_full[inner][:, inner].tocsc(),
                     A_IB=A_full[inner][:, bnd].tocsr(), interior=inner, boundary=bnd)


def load_cellwise(g: np.ndarray, h: float) -> np.ndarray:
    """Load of a source constant on every cell: b_i = int phi_i g = (h^2/4) sum_{e ni i} g_e.

    ``g`` is ``[n][n]`` or ``[nrhs][n][n]``; returns ``[N]`` or ``[nrhs][N]``.
    """
    g = np.asarray(g, dtype=np.float64)
    single = g.ndim == 2
    if single:
        g = g[None]
    nrhs, n, _ = g.shape
    out = np.zeros((nrhs, n + 1, n + 1))
    q = 0.25 * h * h * g
    out[:, :-1, :-1] += q
    out[:, 1:, :-1] += q
    out[:, :-1, 1:] += q
    out[:, 1:, 1:] += q
    b = out[:, 1:-1, 1:-1].reshape(nrhs, -1)
    return b[0] if single else b


def load_nodal(gn: np.ndarray, h: float) -> np.ndarray:
    """Load of a nodal source g = sum_i g_i phi_i (Example 5.1): b = M g.

    ``gn`` holds the interior nodal values ``[n-1][n-1]``; boundary values are 0.
    """
    m = gn.shape[0]
    n = m + 1
    full = np.zeros((n + 1, n + 1))
    full[1:-1, 1:-1] = gn
    cn = cell_nodes(n)
    rows = np.repeat(cn, 4, axis=1).ravel()
    cols = np.tile(cn, (1, 4)).ravel()
    vals = np.tile((h * h * M_UNIT).ravel(), n * n)
    nn = (n + 1) ** 2
    M = sp.coo_matrix((vals, (rows, cols)), shape=(nn, nn)).tocsr()
    return (M @ full.ravel())[interior_ids(n)]


def lift(fe: FEProblem, b: np.ndarray, u_boundary: np.ndarray | None) -> np.ndarray:
    """Move known Dirichlet values to the right-hand side: b - A_IB u_B."""
    if u_boundary is None:
        return b
    ub = np.asarray(u_boundary, dtype=np.float64).reshape(-1, (fe.n + 1) ** 2)[:, fe.boundary]
    out = np.atleast_2d(b) - (fe.A_IB @ ub.T).T
    return out[0] if np.ndim(b) == 1 else out


class DirectSolver:
    """Sparse LU of the interior stiffness matrix plus FP64 iterative refinement."""

    def __init__(self, A: sp.spmatrix, refine: int = 2, ordering: str = "MMD_AT_PLUS_A"):
        self.A = sp.csc_matrix(A)
        self.lu = spla.splu(self.A, permc_spec=ordering)
        self.refine = refine

    def solve(self, b: np.ndarray) -> np.ndarray:
        b = np.asarray(b, dtype=np.float64)
        bt = b.T if b.ndim == 2 else b
        x = self.lu.solve(bt)
        for _ in range(self.refine):
            x = x + self.lu.solve(bt - self.A @ x)
        return x.T if b.ndim == 2 else x


def full_nodal(fe: FEProblem, u_int: np.ndarray, u_boundary: np.ndarray | None = None) -> np.ndarray:
    """Interior values (plus optional boundary values) -> [(n+1)][(n+1)] nodal array."""
    n = fe.n
    full = np.zeros((n + 1) ** 2)
    if u_boundary is not None:
        ub = np.asarray(u_boundary, dtype=np.float64).ravel()
        full[fe.boundary] = ub[fe.boundary]
    full[fe.interior] = u_int
    return full.reshape(n + 1, n + 1)


def solve(a: np.ndarray, g: np.ndarray, u_boundary: np.ndarray | None = None) -> np.ndarray:
    """FE solution u = A^{-1}(b - A_IB u_B) for a cell source, as a full nodal array."""
    fe = assemble(a)
    b = lift(fe, load_cellwise(g, fe.h), u_boundary)
    u = DirectSolver(fe.A).solve(b)
    if u.ndim == 1:
        return full_nodal(fe, u, u_boundary)
    return np.stack([full_nodal(fe, ui, u_boundary) for ui in u])


# ----------------------------------------------------------------------------
# Adjoint gradient of J = 1/2 |u - u_obs|^2 (Euclidean over interior nodes)
# with respect to log a_e and g_e.  Not in the paper: it differentiates the
# discrete problem of Section 5.1.
# ----------------------------------------------------------------------------

def cell_energy_gradient(a: np.ndarray, u_full: np.ndarray, lam_full: np.ndarray) -> np.ndarray:
    """dJ/d log a_e = -a_e lam_e^T K_unit u_e per cell (u with boundary values, lam zero there)."""
    n = a.shape[0]
    cn = cell_nodes(n)
    ue = u_full.ravel()[cn]
    le = lam_full.ravel()[cn]
    return (-a.ravel() * np.einsum("ci,ij,cj->c", le, K_UNIT, ue)).reshape(n, n)


def cell_source_gradient(lam_full: np.ndarray, h: float) -> np.ndarray:
    """dJ/d g_e = (h^2/4) sum of lam over the four corners of cell e."""
    n = lam_full.shape[0] - 1
    cn = cell_nodes(n)
    return (0.25 * h * h * lam_full.ravel()[cn].sum(axis=1)).reshape(n, n)


def adjoint(a: np.ndarray, g: np.ndarray, u_obs_int: np.ndarray,
            u_boundary: np.ndarray | None = None):
    """Return (u_full, J, dJ/dlog a, dJ/dg) by the adjoint method (A is symmetric)."""
    fe = assemble(a)
    solver = DirectSolver(fe.A)
    b = lift(fe, load_cellwise(g, fe.h), u_boundary)
    u = solver.solve(b)
    r = u - u_obs_int
    J = 0.5 * float(r @ r)
    lam = solver.solve(r)
    u_full = full_nodal(fe, u, u_boundary)
    lam_full = full_nodal(fe, lam)
    return u_full, J, cell_energy_gradient(a, u_full, lam_full), cell_source_gradient(lam_full, fe.h)


def fd_log_a(a: np.ndarray, g: np.ndarray, u_obs_int: np.ndarray, cells, step: float = 1e-6):
    """Central difference of J in log a_e without cancellation (zero Dirichlet data).

    Scaling a_e by e^s changes A by a low-rank term U C U^T on the cell's
    interior corners, C = (e^s - 1) a_e K_sub.  The solution change follows
    from the push-through (Woodbury) identity
    du = -A^{-1} U (I + C U^T A^{-1} U)^{-1} C U^T u, and
    dJ = (u - u_obs)^T du + |du|^2 / 2 is formed without subtracting two
    nearly equal values of J.
    """
    fe = assemble(a)
    n = fe.n
    solver = DirectSolver(fe.A)
    u = solver.solve(load_cellwise(g, fe.h))
    r = u - u_obs_int
    cn = cell_nodes(n)
    pos = -np.ones((n + 1) ** 2, dtype=np.int64)
    pos[fe.interior] = np.arange(fe.interior.size)
    out = []
    for c in np.asarray(cells).ravel():
        loc = np.flatnonzero(pos[cn[c]] >= 0)
        idx = pos[cn[c]][loc]
        Ksub = K_UNIT[np.ix_(loc, loc)]
        Umat = np.zeros((u.size, idx.size))
        Umat[idx, np.arange(idx.size)] = 1.0
        AinvU = solver.solve(Umat.T).T
        G = AinvU[idx, :]
        ae = a.ravel()[c]
        dJ = []
        for s in (step, -step):
            C = np.expm1(s) * ae * Ksub
            z = np.linalg.solve(np.eye(idx.size) + C @ G, C @ u[idx])
            du = -AinvU @ z
            dJ.append(float(r @ du) + 0.5 * float(du @ du))
        out.append((dJ[0] - dJ[1]) / (2.0 * step))
    return np.array(out)
