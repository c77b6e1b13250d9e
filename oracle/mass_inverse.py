"""Oracle (test infrastructure only; never used by the product path): level-q
gamblets from the localized inverse of the mass matrix (Algorithm 1, the mass
matrix inversion and the level-q gamblets; Algorithm 2, the localized mass
inverse, the level-q gamblets, their load and their stiffness matrix;
Definition 5.2).

Plain FP64 numpy/scipy, written from the paper's definitions:

* M_ij = int phi_i phi_j over the interior Q1 basis (Algorithm 2, first
  line);
* for every interior node i, the patch i^rho: interior nodes whose node cells
  lie within rho cells of node i's, read as the box |dx|, |dy| <= rho clipped
  to the interior; y^(i,rho) solves M^(i,rho) y = e_i on the patch, and column
  i of the localized inverse holds y on the patch, zero elsewhere
  (Definition 5.2);
* psi^(q),loc_i = sum_j Minv_loc[j, i] phi_j, so that in the phi basis
  A^(q),loc = Minv_loc^T A Minv_loc, g^(q),loc_i = int psi_i g =
  (Minv_loc^T b)_i, and a level-q coefficient vector U stands for the nodal
  vector Minv_loc U (Algorithm 2, the lines that form psi^(q), g^(q) and
  A^(q)).

With rho at least the grid size the patch is the whole interior and the
localized inverse is M^-1, the exact level-q gamblets of Algorithm 1.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from oracle import fem


def mass_matrix(n: int, h: float | None = None) -> sp.csc_matrix:
    """Interior Q1 mass matrix M_ij = int phi_i phi_j, assembled cell by cell."""
    if h is None:
        h = 1.0 / n
    cn = fem.cell_nodes(n)
    rows = np.repeat(cn, 4, axis=1).ravel()
    cols = np.tile(cn, (1, 4)).ravel()
    vals = np.tile((h * h * fem.M_UNIT).ravel(), n * n)
    nn = (n + 1) ** 2
    M = sp.coo_matrix((vals, (rows, cols)), shape=(nn, nn)).tocsr()
    inner = fem.interior_ids(n)
    return M[inner][:, inner].tocsc()


def patch_nodes(n: int, i: int, rho: int) -> np.ndarray:
    """Interior indices of the patch i^rho of interior node i (box of radius
    rho in node steps, clipped to the interior)."""
    m = n - 1
    ix, iy = divmod(i, m)
    xs = np.arange(max(0, ix - rho), min(m, ix + rho + 1))
    ys = np.arange(max(0, iy - rho), min(m, iy + rho + 1))
    return (xs[:, None] * m + ys[None, :]).ravel()


def localized_mass_inverse(M: sp.spmatrix, n: int, rho: int) -> sp.csc_matrix:
    """Columns y^(i,rho) of Definition 5.2, one dense patch solve per node."""
    M = sp.csr_matrix(M)
    N = (n - 1) ** 2
    rows, cols, vals = [], [], []
    for i in range(N):
        p = patch_nodes(n, i, rho)
        Mp = M[p][:, p].toarray()
        e = (p == i).astype(np.float64)
        y = np.linalg.solve(Mp, e)
        rows.append(p)
        cols.append(np.full(p.size, i))
        vals.append(y)
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsc()


@dataclass
class LevelQ:
    n: int
    rho: int
    Minv: sp.csc_matrix     # columns: psi^(q),loc in the phi basis
    A: sp.csc_matrix        # A^(q),loc = Minv^T A Minv


def level_q_gamblets(fe: fem.FEProblem, rho: int) -> LevelQ:
    """psi^(q),loc and their stiffness matrix A^(q),loc (Algorithm 2, lines
    that form the localized mass inverse, psi^(q) and A^(q))."""
    M = mass_matrix(fe.n, fe.h)
    Minv = localized_mass_inverse(M, fe.n, rho)
    Aq = (Minv.T @ fe.A @ Minv).tocsc()
    return LevelQ(n=fe.n, rho=rho, Minv=Minv, A=Aq)


def level_q_load(lq: LevelQ, b: np.ndarray) -> np.ndarray:
    """g^(q),loc_i = int psi^(q),loc_i g = sum_j Minv[j, i] b_j, b_j = int phi_j g."""
    return lq.Minv.T @ b


def level_q_to_nodal(lq: LevelQ, U: np.ndarray) -> np.ndarray:
    """Nodal values of sum_i U_i psi^(q),loc_i."""
    return lq.Minv @ U


def stencil_rows(lq: LevelQ, rows: np.ndarray) -> np.ndarray:
    """Rows of A^(q),loc as stencils [len(rows)][(2S+1)^2], S = 2 rho + 1:
    entry (dx + S)(2S+1) + (dy + S) couples node (ix, iy) with
    (ix + dx, iy + dy); zero where that node is not interior."""
    m = lq.n - 1
    S = 2 * lq.rho + 1
    W = 2 * S + 1
    A = sp.csr_matrix(lq.A)
    out = np.zeros((len(rows), W * W))
    for r, i in enumerate(rows):
        ix, iy = divmod(int(i), m)
        lo, hi = A.indptr[i], A.indptr[i + 1]
        for j, v in zip(A.indices[lo:hi], A.data[lo:hi]):
            jx, jy = divmod(int(j), m)
            dx, dy = jx - ix, jy - iy
            assert abs(dx) <= S and abs(dy) <= S
            out[r, (dx + S) * W + (dy + S)] = v
    return out


def local_column(M: sp.spmatrix, n: int, rho: int, i: int):
    """Column i of the localized inverse (Definition 5.2: one patch solve),
    as (patch node indices, values)."""
    p = patch_nodes(n, i, rho)
    Mp = sp.csr_matrix(M)[p][:, p].toarray()
    return p, np.linalg.solve(Mp, (p == i).astype(np.float64))


def operator_row(fe: fem.FEProblem, M: sp.spmatrix, rho: int, i: int) -> np.ndarray:
    """Row i of A^(q),loc as a stencil (layout of stencil_rows), entry by
    entry: A^(q)_ij = y^(i)T A y^(j) for the nodes j within 2 rho + 1 steps."""
    m = fe.n - 1
    S = 2 * rho + 1
    W = 2 * S + 1
    ix, iy = divmod(i, m)
    M = sp.csr_matrix(M)
    pi, yi = local_column(M, fe.n, rho, i)
    Ay = sp.csc_matrix(fe.A)[:, pi] @ yi          # A y^(i), dense over all nodes
    out = np.zeros(W * W)
    for dx in range(-S, S + 1):
        for dy in range(-S, S + 1):
            jx, jy = ix + dx, iy + dy
            if 0 <= jx < m and 0 <= jy < m:
                pj, yj = local_column(M, fe.n, rho, jx * m + jy)
                out[(dx + S) * W + dy + S] = Ay[pj] @ yj
    return out
