"""Gamblet hierarchy and subband solve, written out plainly (oracle).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of the paper taken here (each also listed in the design notes):

* Levels.  The fine mesh has ``n = 2^q`` cells per dimension.  Level ``q``
  indexes the interior nodes (the measurement functions of level q are the
  nodal basis functions themselves, the initialisation allowed in the
  discussion of Algorithm 1 in Section 5.2: psi^(q) = phi, so A^(q) = A and
  g^(q) = b).  Levels ``k < q`` index the dyadic cells of side ``2^-k``;
  node ``(i, j)`` belongs to level-(q-1) cell ``(i // 2, j // 2)`` and
  cell ``(cx, cy)`` of level k to cell ``(cx // 2, cy // 2)`` of level k-1
  (nested aggregation of Section 5.1 and Construction 4.2).  Along the two
  low edges some level-(q-1) cells have only one or two children; the index
  tree of Definition 4.1 allows any child count.
  With ``offset=1`` the tree instead follows Example 5.1 exactly (``2^q + 1``
  cells, ``2^q`` interior nodes per dimension, a uniform quad-tree).
* Child order inside a parent: ``t = 2 dx + dy`` with ``(dx, dy)`` the child's
  position in its parent.
* Localization (Algorithm 2, Definition 5.3): the patch of a coarse cell is
  the box of coarse cells within ``rho`` in each coordinate, clipped to the
  domain, with the same ``rho`` at every level.

Index orders: level q uses the interior-node order of ``oracle.fem``;
level k < q uses ``cx * 2^k + cy``; J^(k) lists, parent by parent in level
k-1 order, the ``m_s - 1`` subband indices of each parent.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def helmert(m: int) -> np.ndarray:
    """Rows of the orthogonal matrix U^(m) of Lemma 4.12, normalised (m >= 1).

    U^(2) has rows (1, -1) and (1, 1); U^(m+1) keeps U^(m) in its leading
    block, puts -m in position (m, m+1) (one-based), zeros elsewhere in the new
    column, and a last row of ones.  Returned with unit rows.
    """
    if m == 1:
        return np.ones((1, 1))
    U = np.array([[1.0, -1.0], [1.0, 1.0]])
    for n in range(2, m):
        V = np.zeros((n + 1, n + 1))
        V[:n, :n] = U
        V[n - 1, n] = -float(n)
        V[n, :] = 1.0
        U = V
    return U / np.linalg.norm(U, axis=1, keepdims=True)


@dataclass
class Tree:
    """Index tree (Definition 4.1) of the dyadic measurement hierarchy."""
    q: int
    offset: int = 0
    coords: dict = field(default_factory=dict)     # level -> [|I^(k)|, 2] coordinates
    parent: dict = field(default_factory=dict)     # level k -> [|I^(k)|] index in I^(k-1)
    children: dict = field(default_factory=dict)   # level k -> list over I^(k-1) of child lists (sorted by t)

    def __post_init__(self):
        q = self.q
        if self.offset == 0:
            n = 1 << q
            i, j = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="ij")
        else:
            n = (1 << q) + 1
            i, j = np.meshgrid(np.arange(1, n), np.arange(1, n), indexing="ij")
        self.n_cells = n
        # level-q "slot" coordinates: node (i,j) -> (i - offset, j - offset) in [0, 2^q)
        self.coords[q] = np.stack([i.ravel() - self.offset, j.ravel() - self.offset], axis=1)
        for k in range(q - 1, 0, -1):
            cx, cy = np.meshgrid(np.arange(1 << k), np.arange(1 << k), indexing="ij")
            self.coords[k] = np.stack([cx.ravel(), cy.ravel()], axis=1)
        for k in range(q, 1, -1):
            c = self.coords[k]
            side = 1 << (k - 1)
            par = (c[:, 0] // 2) * side + (c[:, 1] // 2)
            self.parent[k] = par
            t = 2 * (c[:, 0] % 2) + (c[:, 1] % 2)
            kids = [[] for _ in range(side * side)]
            for idx in np.lexsort((t, par)):
                kids[par[idx]].append(int(idx))
            self.children[k] = kids

    def size(self, k: int) -> int:
        return self.coords[k].shape[0]

    def pi(self, k: int) -> sp.csr_matrix:
        """pi^(k-1,k): 0/1 aggregation matrix of Construction 4.2."""
        nk = self.size(k)
        return sp.csr_matrix((np.ones(nk), (self.parent[k], np.arange(nk))),
                             shape=(self.size(k - 1), nk))

    def pibar(self, k: int) -> sp.csr_matrix:
        """pi-bar^(k-1,k): pi with row s divided by its child count m_s (Section 4.7)."""
        P = self.pi(k)
        m = np.asarray(P.sum(axis=1)).ravel()
        return sp.diags(1.0 / m) @ P

    def jparent(self, k: int) -> np.ndarray:
        """Parent (in I^(k-1)) of every subband index of J^(k)."""
        return np.concatenate([np.full(max(len(ch) - 1, 0), s, dtype=np.int64)
                               for s, ch in enumerate(self.children[k])])

    def W(self, k: int, construction: int = 2) -> sp.csr_matrix:
        """W^(k) with rows spanning ker pi^(k-1,k), block-diagonal by parent.

        Construction 4.11 (``construction=1``): row (s,t) = e_t - e_{t+1}.
        Construction 4.13 (``construction=2``): row (s,t) = row t of the
        normalised Helmert matrix of size m_s.
        """
        rows, cols, vals = [], [], []
        r = 0
        for ch in self.children[k]:
            m = len(ch)
            if m < 2:
                continue
            if construction == 1:
                blk = np.zeros((m - 1, m))
                for t in range(m - 1):
                    blk[t, t] = 1.0
                    blk[t, t + 1] = -1.0
            else:
                blk = helmert(m)[: m - 1]
            for t in range(m - 1):
                for tt in range(m):
                    if blk[t, tt] != 0.0:
                        rows.append(r + t)
                        cols.append(ch[tt])
                        vals.append(blk[t, tt])
            r += m - 1
        return sp.csr_matrix((vals, (rows, cols)), shape=(r, self.size(k)))

    def box(self, k: int, i: int, rho: int) -> np.ndarray:
        """Level-k indices whose coordinates lie within rho of index i in each coordinate."""
        c = self.coords[k]
        d = np.abs(c - c[i])
        return np.flatnonzero((d[:, 0] <= rho) & (d[:, 1] <= rho))


@dataclass
class Tree3(Tree):
    """The same index tree on the unit cube (the problem of Section 1 in d = 3):
    level q indexes the interior nodes (order of ``oracle.fem3d``), levels
    k < q the dyadic cubes (index (cx 2^k + cy) 2^k + cz); node (i, j, l)
    belongs to level-(q-1) cube ((i - offset) // 2, ...), a cube to its
    parent by halving every coordinate.  A parent has up to eight children,
    ordered by t = 4 dx + 2 dy + dz."""

    def __post_init__(self):
        q = self.q
        n = (1 << q) + self.offset
        self.n_cells = n
        i = np.arange(1, n)
        I, J, L = np.meshgrid(i, i, i, indexing="ij")
        self.coords[q] = np.stack([I.ravel(), J.ravel(), L.ravel()], axis=1) - self.offset
        for k in range(q - 1, 0, -1):
            c = np.arange(1 << k)
            X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
            self.coords[k] = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
        for k in range(q, 1, -1):
            c = self.coords[k]
            side = 1 << (k - 1)
            par = ((c[:, 0] // 2) * side + (c[:, 1] // 2)) * side + (c[:, 2] // 2)
            self.parent[k] = par
            t = 4 * (c[:, 0] % 2) + 2 * (c[:, 1] % 2) + (c[:, 2] % 2)
            kids = [[] for _ in range(side ** 3)]
            for idx in np.lexsort((t, par)):
                kids[par[idx]].append(int(idx))
            self.children[k] = kids

    def box(self, k: int, i: int, rho: int) -> np.ndarray:
        c = self.coords[k]
        d = np.abs(c - c[i])
        return np.flatnonzero((d[:, 0] <= rho) & (d[:, 1] <= rho) & (d[:, 2] <= rho))


# ----------------------------------------------------------------------------
# Exact gamblet transform (Algorithm 1 with psi^(q) = nodal basis).
# ----------------------------------------------------------------------------

@dataclass
class Level:
    A: np.ndarray | sp.spmatrix          # A^(k)
    W: sp.csr_matrix | None = None       # W^(k)
    B: np.ndarray | sp.spmatrix | None = None   # B^(k) = W A W^T
    R: np.ndarray | sp.spmatrix | None = None   # R^(k-1,k)
    D: np.ndarray | sp.spmatrix | None = None   # D^(k,k-1)


@dataclass
class Hierarchy:
    tree: Tree
    levels: dict            # k -> Level (k = 1..q)
    rho: int | None = None  # None: exact


def exact_hierarchy(A: sp.spmatrix, tree: Tree, construction: int = 2) -> Hierarchy:
    """Dense nested computation of A^(k), B^(k), D, R (Algorithm 1, steps 7-15).

    B^(k) = W A^(k) W^T (eq. for B in Section 4.7), D^(k,k-1) = -B^-1 W A^(k)
    pibar^T (definition of D), R^(k-1,k) = pibar + D^T W (theorem giving R in
    terms of pibar and D), A^(k-1) = R A^(k) R^T (Theorem 4.8).
    """
    q = tree.q
    Ak = A.toarray() if sp.issparse(A) else np.asarray(A, dtype=np.float64)
    levels = {}
    for k in range(q, 1, -1):
        W = tree.W(k, construction)
        Wd = W.toarray()
        pibar = tree.pibar(k).toarray()
        B = Wd @ Ak @ Wd.T
        if B.shape[0] > 0:
            D = -sla.cho_solve(sla.cho_factor(B), Wd @ Ak @ pibar.T)
        else:
            D = np.zeros((0, pibar.shape[0]))
        R = pibar + D.T @ Wd
        levels[k] = Level(A=Ak, W=W, B=B, R=R, D=D)
        Ak = R @ Ak @ R.T
    levels[1] = Level(A=Ak)
    return Hierarchy(tree=tree, levels=levels, rho=None)


# ----------------------------------------------------------------------------
# Localized gamblet transform (Algorithm 2, Definition 5.3).
# ----------------------------------------------------------------------------

def patch_index_set(tree: Tree, k: int, i: int, rho: int, jpar: np.ndarray) -> np.ndarray:
    """i^chi of Definition 5.3: subband indices of J^(k) whose parent is in the box of i."""
    inbox = np.zeros(tree.size(k - 1), dtype=bool)
    inbox[tree.box(k - 1, i, rho)] = True
    return np.flatnonzero(inbox[jpar])


def localized_hierarchy(A: sp.spmatrix, tree: Tree, rho: int, construction: int = 2,
                        keep_D: bool = False) -> Hierarchy:
    """Localized nested computation (Algorithm 2: subband operator, patch systems, R, Galerkin).

    For every coarse index i of level k-1 the patch system
    B^(i,rho) y = -(W A^(k) pibar^T)_{i^chi, i} of Definition 5.3 is solved by a
    dense Cholesky factorisation; y fills column i of D^(k,k-1) on i^chi.
    ``rho`` is one radius for every transition, or a dict k -> rho_(k-1), the
    radius of the patches of the transition from level k to level k-1
    (Algorithm 2 allows a radius per level).
    """
    q = tree.q
    Ak = sp.csr_matrix(A)
    levels = {}
    for k in range(q, 1, -1):
        W = tree.W(k, construction)
        pibar = tree.pibar(k)
        B = (W @ Ak @ W.T).tocsr()
        rhs = -(W @ Ak @ pibar.T).tocsc()
        jpar = tree.jparent(k)
        rows, cols, vals = [], [], []
        rho_k = rho[k] if isinstance(rho, dict) else rho
        for i in range(tree.size(k - 1)):
            chi = patch_index_set(tree, k, i, rho_k, jpar)
            if chi.size == 0:
                continue
            Bp = B[chi][:, chi].toarray()
            bp = rhs[chi, i].toarray().ravel()
            y = sla.cho_solve(sla.cho_factor(Bp), bp)
            rows.append(chi)
            cols.append(np.full(chi.size, i))
            vals.append(y)
        if rows:
            D = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                              shape=(W.shape[0], tree.size(k - 1)))
        else:
            D = sp.csr_matrix((W.shape[0], tree.size(k - 1)))
        R = (pibar + D.T @ W).tocsr()
        levels[k] = Level(A=Ak, W=W, B=B, R=R, D=D if keep_D else None)
        Ak = (R @ Ak @ R.T).tocsr()
    levels[1] = Level(A=Ak)
    return Hierarchy(tree=tree, levels=levels, rho=rho)


def localized_R_by_energy_minimization(A_k: sp.spmatrix, tree: Tree, k: int, rho: int) -> sp.csr_matrix:
    """R^(k-1,k) of the localized transform from its variational characterisation.

    Remark 5.4: the localized psi^(k-1)_i minimises the energy over the span of
    the level-k gamblets whose parents lie in the patch of i, subject to
    int phi^(k-1)_j psi = delta_ij for the coarse indices j of the patch.  In
    level-k coefficients c this is the equality-constrained quadratic problem
    min c^T A_LL c s.t. pi_PL c = e_i, solved here by its KKT system.  W does
    not appear at all.
    """
    A_k = sp.csr_matrix(A_k)
    P = tree.pi(k)
    rows, cols, vals = [], [], []
    for i in range(tree.size(k - 1)):
        patch = tree.box(k - 1, i, rho)
        L = np.flatnonzero(np.isin(tree.parent[k], patch))
        All = A_k[L][:, L].toarray()
        Ppl = P[patch][:, L].toarray()
        nL, nP = L.size, patch.size
        KKT = np.zeros((nL + nP, nL + nP))
        KKT[:nL, :nL] = All
        KKT[:nL, nL:] = Ppl.T
        KKT[nL:, :nL] = Ppl
        rhs = np.zeros(nL + nP)
        rhs[nL + int(np.flatnonzero(patch == i)[0])] = 1.0
        c = np.linalg.solve(KKT, rhs)[:nL]
        rows.append(np.full(nL, i))
        cols.append(L)
        vals.append(c)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(tree.size(k - 1), tree.size(k)))


# ----------------------------------------------------------------------------
# Subband solve (eqs. for w^(k) and U^(1) in Section 4.7, Theorem 4.15).
# ----------------------------------------------------------------------------

def _solve_spd(M, rhs):
    if sp.issparse(M):
        if M.shape[0] == 0:
            return np.zeros_like(rhs)
        return spla.splu(sp.csc_matrix(M)).solve(rhs)
    if M.shape[0] == 0:
        return np.zeros_like(rhs)
    return sla.cho_solve(sla.cho_factor(M), rhs)


def restrict_rhs(h: Hierarchy, b: np.ndarray) -> dict:
    """g^(q) = b, g^(k-1) = R^(k-1,k) g^(k) (eq. for g^(k) in Section 4.7)."""
    q = h.tree.q
    g = {q: np.asarray(b, dtype=np.float64)}
    for k in range(q, 1, -1):
        g[k - 1] = h.levels[k].R @ g[k]
    return g


def subband_coefficients(h: Hierarchy, b: np.ndarray):
    """Solve B^(k) w^(k) = W^(k) g^(k) for k = 2..q and A^(1) U^(1) = g^(1).

    Each system is solved directly (the subband systems are independent).
    """
    q = h.tree.q
    g = restrict_rhs(h, b)
    w = {}
    for k in range(q, 1, -1):
        lv = h.levels[k]
        w[k] = _solve_spd(lv.B, lv.W @ g[k])
    U1 = _solve_spd(h.levels[1].A, g[1])
    return U1, w, g


def prolong(h: Hierarchy, k0: int, v: np.ndarray) -> np.ndarray:
    """Coefficients on the level-k0 gamblets -> nodal coefficients (psi^(q) = phi).

    Uses psi^(k-1) = R^(k-1,k) psi^(k) (eq. defining R), so a coefficient
    vector v on level k-1 equals R^T v on level k.
    """
    for k in range(k0 + 1, h.tree.q + 1):
        v = h.levels[k].R.T @ v
    return v


def solve(h: Hierarchy, b: np.ndarray) -> np.ndarray:
    """u = psi^(1)-part + sum_k chi^(k)-parts (Theorem 4.15), in nodal values.

    Reconstruction v^(1) = U^(1), v^(k) = R^(k,k-1) v^(k-1) + W^(k)T w^(k); the
    subband gamblets are never formed (discussion of Algorithm 1, Section 5.2).
    """
    U1, w, _ = subband_coefficients(h, b)
    v = U1
    for k in range(2, h.tree.q + 1):
        lv = h.levels[k]
        v = lv.R.T @ v + lv.W.T @ w[k]
    return v


def subbands(h: Hierarchy, b: np.ndarray) -> list:
    """Nodal vectors [u^(1), u^(2)-u^(1), ..., u^(q)-u^(q-1)] (eq. of Theorem 4.6)."""
    U1, w, _ = subband_coefficients(h, b)
    out = [prolong(h, 1, U1)]
    for k in range(2, h.tree.q + 1):
        out.append(prolong(h, k, h.levels[k].W.T @ w[k]))
    return out


# ----------------------------------------------------------------------------
# Gamblet transform of a given vector and compression (the representation of
# u in the basis psi^(1)_i / ||psi^(1)_i||_a, chi^(k)_j / ||chi^(k)_j||_a of
# the discussion of Example 5.1 and Figures 10-11).
# ----------------------------------------------------------------------------

def gamblet_transform(h: Hierarchy, u: np.ndarray):
    """Coefficients (U^(1), {k: w^(k)}) of a level-q vector u in the basis
    {psi^(1)_i} + {chi^(k)_j, k = 2..q}.

    The level-(k-1) measurement of a vector is the sum of its level-k
    measurements over the children (R^(k-1,k) pi^(k-1,k)T = I for every
    R = pibar + D W, since pibar pi^T = I and W pi^T = 0), so the level-(k-1)
    coefficients are U^(k-1) = pi U^(k), and the detail U^(k) - R^T U^(k-1)
    lies in the range of W^T: it is W^T w^(k) with w^(k) = (W W^T)^-1 W
    (U^(k) - R^T U^(k-1)).  Telescoping the levels reproduces u through the
    reconstruction of Theorem 4.15 (``inverse_transform``).
    """
    q = h.tree.q
    Uk = np.asarray(u, dtype=np.float64)
    w = {}
    for k in range(q, 1, -1):
        lv = h.levels[k]
        Ukm1 = h.tree.pi(k) @ Uk
        d = Uk - lv.R.T @ Ukm1
        WWt = (lv.W @ lv.W.T).tocsc()
        w[k] = spla.spsolve(WWt, lv.W @ d) if WWt.shape[0] else np.zeros(0)
        Uk = Ukm1
    return Uk, w


def inverse_transform(h: Hierarchy, U1: np.ndarray, w: dict) -> np.ndarray:
    """v^(1) = U^(1), v^(k) = R^(k,k-1) v^(k-1) + W^(k)T w^(k) (Theorem 4.15)."""
    v = np.asarray(U1, dtype=np.float64)
    for k in range(2, h.tree.q + 1):
        lv = h.levels[k]
        v = lv.R.T @ v + lv.W.T @ w[k]
    return v


def energy_scales(h: Hierarchy):
    """||psi^(1)_i||_a = sqrt(A^(1)_ii) and ||chi^(k)_j||_a = sqrt(B^(k)_jj)
    (chi^(k) = W^(k) psi^(k), so the Gram matrix of the chi^(k) is W A^(k) W^T)."""
    def diag(M):
        return M.diagonal() if sp.issparse(M) else np.diag(M)
    s1 = np.sqrt(diag(h.levels[1].A))
    sk = {k: np.sqrt(diag(h.levels[k].B)) for k in range(2, h.tree.q + 1)}
    return s1, sk


def normalized_coefficients(h: Hierarchy, u: np.ndarray):
    """Coefficients of u on psi^(1)/||psi^(1)||_a and chi^(k)/||chi^(k)||_a."""
    U1, w = gamblet_transform(h, u)
    s1, sk = energy_scales(h)
    return U1 * s1, {k: w[k] * sk[k] for k in w}


def compress(c1: np.ndarray, ck: dict, keep: int):
    """Keep the ``keep`` largest normalized coefficients (by magnitude, over all
    levels) and set the others to zero; coefficients equal to the smallest kept
    magnitude are kept as well."""
    allc = np.concatenate([np.abs(c1)] + [np.abs(ck[k]) for k in sorted(ck)])
    if keep <= 0:
        thr = np.inf
    elif keep >= allc.size:
        thr = -np.inf
    else:
        thr = np.sort(allc)[::-1][keep - 1]
    return (np.where(np.abs(c1) >= thr, c1, 0.0),
            {k: np.where(np.abs(ck[k]) >= thr, ck[k], 0.0) for k in ck})


def reconstruct_normalized(h: Hierarchy, c1: np.ndarray, ck: dict) -> np.ndarray:
    """Level-q vector from normalized coefficients."""
    s1, sk = energy_scales(h)
    return inverse_transform(h, c1 / s1, {k: np.divide(ck[k], sk[k], out=np.zeros_like(ck[k]),
                                                           where=sk[k] > 0) for k in ck})


def refine_solve(h: Hierarchy, A: sp.spmatrix, b: np.ndarray, tol: float = 1e-10,
                 max_sweeps: int = 50):
    """Iterative refinement with the localized subband solve as approximate inverse.

    u <- u + S(b - A u) until the correction falls below ``tol`` relative to u
    (the localized solve is inexact; Section 5.4 allows inexact use).  Returns
    (u, sweeps, history of relative corrections).
    """
    u = np.zeros_like(b)
    hist = []
    for it in range(max_sweeps):
        du = solve(h, b - A @ u)
        u = u + du
        rel = float(np.linalg.norm(du) / max(np.linalg.norm(u), 1e-300))
        hist.append(rel)
        if rel <= tol:
            return u, it + 1, hist
    return u, max_sweeps, hist
