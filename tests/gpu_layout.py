"""Convert the library's offset-major device layouts into plain matrices
indexed like the oracle (test helper; reads only numpy arrays)."""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def slot_to_index(q: int, k: int) -> np.ndarray:
    """Map level-k slot id (x*2^k + y) to the oracle index (-1 where no unknown)."""
    nk = 1 << k
    x, y = np.meshgrid(np.arange(nk), np.arange(nk), indexing="ij")
    if k < q:
        return (x * nk + y).ravel()
    n = nk
    idx = (x - 1) * (n - 1) + (y - 1)
    idx[(x == 0) | (y == 0)] = -1
    return idx.ravel()


def stencil_to_matrix(A: np.ndarray, q: int, k: int, size: int) -> sp.csr_matrix:
    """A[S][S][nk][nk] -> size x size matrix in oracle indices."""
    S = A.shape[0]
    s = S // 2
    nk = A.shape[2]
    m = slot_to_index(q, k)
    rows, cols, vals = [], [], []
    x, y = np.meshgrid(np.arange(nk), np.arange(nk), indexing="ij")
    for ox in range(S):
        for oy in range(S):
            xx, yy = x + ox - s, y + oy - s
            ok = (xx >= 0) & (yy >= 0) & (xx < nk) & (yy < nk)
            src = (x * nk + y)[ok]
            dst = (xx * nk + yy)[ok]
            v = A[ox, oy][ok]
            r, c = m[src], m[dst]
            keep = (r >= 0) & (c >= 0)
            rows.append(r[keep]); cols.append(c[keep]); vals.append(v[keep])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(size, size))


def subband_map(tree, k: int) -> np.ndarray:
    """GPU subband id (t * np^2 + parent) -> oracle J^(k) row (-1 for padding rows).

    The oracle lists J^(k) parent by parent with m_s - 1 rows each."""
    npar = tree.size(k - 1)
    m = np.array([len(ch) for ch in tree.children[k]])
    start = np.concatenate([[0], np.cumsum(np.maximum(m - 1, 0))[:-1]])
    out = -np.ones(3 * npar, dtype=np.int64)
    for t in range(3):
        ok = t < m - 1
        out[t * npar + np.flatnonzero(ok)] = start[ok] + t
    return out


def block_stencil_to_matrix(B: np.ndarray, tree, k: int) -> sp.csr_matrix:
    """B[T][T][3][3][np][np] -> |J^(k)| x |J^(k)| matrix in oracle order."""
    T = B.shape[0]
    t = T // 2
    npd = B.shape[4]
    npar = npd * npd
    m = subband_map(tree, k)
    size = int(m.max()) + 1
    px, py = np.meshgrid(np.arange(npd), np.arange(npd), indexing="ij")
    rows, cols, vals = [], [], []
    for ox in range(T):
        for oy in range(T):
            qx, qy = px + ox - t, py + oy - t
            ok = (qx >= 0) & (qy >= 0) & (qx < npd) & (qy < npd)
            src = (px * npd + py)[ok]
            dst = (qx * npd + qy)[ok]
            for i in range(3):
                for j in range(3):
                    r = m[i * npar + src]
                    c = m[j * npar + dst]
                    v = B[ox, oy, i, j][ok]
                    keep = (r >= 0) & (c >= 0)
                    rows.append(r[keep]); cols.append(c[keep]); vals.append(v[keep])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(size, size))


def restriction_to_matrix(R: np.ndarray, rho: int, q: int, k: int, nfine: int) -> sp.csr_matrix:
    """R[rw][rw][nc][nc] (rows of R^(k-1,k)) -> |I^(k-1)| x |I^(k)| matrix."""
    rw = R.shape[0]
    nc = R.shape[2]
    nk = 2 * nc
    mf = slot_to_index(q, k)
    cx, cy = np.meshgrid(np.arange(nc), np.arange(nc), indexing="ij")
    rows, cols, vals = [], [], []
    for bx in range(rw):
        for by in range(rw):
            fx, fy = 2 * (cx - rho) + bx, 2 * (cy - rho) + by
            ok = (fx >= 0) & (fy >= 0) & (fx < nk) & (fy < nk)
            r = (cx * nc + cy)[ok]
            c = mf[(fx * nk + fy)[ok]]
            v = R[bx, by][ok]
            keep = c >= 0
            rows.append(r[keep]); cols.append(c[keep]); vals.append(v[keep])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(nc * nc, nfine))
