"""Seeded synthetic inputs shared, as data, by the CPU oracle and the HIP path.

This module holds no arithmetic of the gamblet method: it only draws
coefficient fields, sources and observation fields of the shapes and value
distributions of the paper's numerical example (Section 5.1, Example 5.1) and
of the rough-coefficient workloads this library is measured on.

Conventions
-----------
* A mesh of ``n`` cells per dimension on the unit square, cell ``(ex, ey)``
  covering ``[ex h, (ex+1) h) x [ey h, (ey+1) h)``; arrays are ``[ex][ey]``,
  C order, float64.
* Every random draw comes from ``numpy.random.default_rng([tag, problem,
  kind, rhs])`` where ``tag`` names the workload, ``kind`` the quantity
  (0 log-coefficient noise, 1 source, 2 observation coefficient noise,
  3 inclusions, 4 level draw, 5 finite-difference cells) and ``rhs`` the
  right-hand side index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

KIND_XI, KIND_G, KIND_OBS, KIND_INCL, KIND_Q, KIND_FD = 0, 1, 2, 3, 4, 5


def rng(tag: int, problem: int = 0, kind: int = 0, rhs: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(tag), int(problem), int(kind), int(rhs)])


def product_field(n: int, K: int = 5, h: float | None = None) -> np.ndarray:
    """Oscillatory product coefficient of Example 5.1 (Section 5.1).

    ``a = prod_{k=1..K} (1 + 0.5 cos(2^k pi (x + y))) (1 + 0.5 sin(2^k pi (y - 3x)))``
    evaluated at the lower-left corner ``(x, y) = (ex h, ey h)`` of every cell.
    ``h`` defaults to ``1/n``; the paper's own example uses ``n = 65``,
    ``h = 1/65`` and ``K = 6``.
    """
    if h is None:
        h = 1.0 / n
    x = np.arange(n, dtype=np.float64)[:, None] * h
    y = np.arange(n, dtype=np.float64)[None, :] * h
    a = np.ones((n, n), dtype=np.float64)
    for k in range(1, K + 1):
        w = (2.0 ** k) * math.pi
        a = a * (1.0 + 0.5 * np.cos(w * (x + y))) * (1.0 + 0.5 * np.sin(w * (y - 3.0 * x)))
    return a


def lognormal_factor(n: int, sigma: float, gen: np.random.Generator) -> np.ndarray:
    """``exp(sigma xi)`` with ``xi ~ N(0, 1)`` iid per cell."""
    return np.exp(sigma * gen.standard_normal((n, n)))


def inclusion_mask(n: int, gen: np.random.Generator, rmin: float = 2.0, rmax: float = 8.0,
                   area: float = 0.10) -> np.ndarray:
    """Union of random discs, drawn until it covers ``area`` of the cells.

    Centres are uniform on the unit square, radii uniform in ``[rmin, rmax]``
    cells; a cell is inside when its centre lies in some disc.
    """
    h = 1.0 / n
    cx = (np.arange(n) + 0.5) * h
    mask = np.zeros((n, n), dtype=bool)
    target = area * n * n
    while mask.sum() < target:
        x0, y0 = gen.uniform(0.0, 1.0, size=2)
        r = gen.uniform(rmin, rmax) * h
        i0, i1 = max(0, int((x0 - r) * n) - 1), min(n, int((x0 + r) * n) + 2)
        j0, j1 = max(0, int((y0 - r) * n) - 1), min(n, int((y0 + r) * n) + 2)
        dx = cx[i0:i1, None] - x0
        dy = cx[None, j0:j1] - y0
        mask[i0:i1, j0:j1] |= (dx * dx + dy * dy) <= r * r
    return mask


def example51_coefficient() -> np.ndarray:
    """Coefficient of Example 5.1: 65 x 65 cells, h = 1/65, K = 6."""
    return product_field(65, K=6, h=1.0 / 65.0)


def example51_nodal_source() -> np.ndarray:
    """Nodal source values of Example 5.1 on the 64 x 64 interior nodes.

    ``g_i = cos(3 z1 + z2) + sin(3 z2) + sin(7 z1 - 5 z2)`` at ``z = (i h, j h)``,
    ``i, j = 1..64``, ``h = 1/65``.
    """
    h = 1.0 / 65.0
    z1 = np.arange(1, 65, dtype=np.float64)[:, None] * h
    z2 = np.arange(1, 65, dtype=np.float64)[None, :] * h
    return np.cos(3 * z1 + z2) + np.sin(3 * z2) + np.sin(7 * z1 - 5 * z2)


def smooth_cell_source(q: int) -> np.ndarray:
    """The source of Example 5.1, g = cos(3 z1 + z2) + sin(3 z2) + sin(7 z1 - 5 z2),
    at the centres of the 2^q x 2^q cells of the unit square (a smooth source for
    the compression measurements; the example itself uses 65 x 65 cells)."""
    n = 1 << q
    z = (np.arange(n, dtype=np.float64) + 0.5) / n
    z1, z2 = z[:, None], z[None, :]
    return np.cos(3 * z1 + z2) + np.sin(3 * z2) + np.sin(7 * z1 - 5 * z2)


@dataclass
class Problem:
    """One synthetic elliptic problem on ``2^q x 2^q`` cells."""
    q: int
    a: np.ndarray                      # [n][n] cell coefficient
    g: np.ndarray                      # [nrhs][n][n] cell source
    rho: int = 3
    tag: int = 0
    problem: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return 1 << self.q

    @property
    def dof(self) -> int:
        return (self.n - 1) ** 2


# Workload tags (used only to seed the generators).
TAG_Q6_EXACT, TAG_Q9_ROUGH, TAG_BATCH, TAG_ADJOINT_Q10, TAG_Q11_INCL = 1, 2, 3, 4, 5


def rough_problem(q: int, sigma: float, tag: int, problem: int = 0, nrhs: int = 1,
                  source: str = "normal", K: int = 5, rho: int = 3) -> Problem:
    """Product field times a lognormal factor, with cell sources.

    ``source`` is ``"normal"`` (iid N(0,1) per cell, one draw per rhs) or
    ``"ones"`` (g = 1).
    """
    n = 1 << q
    a = product_field(n, K=K)
    if sigma != 0.0:
        a = a * lognormal_factor(n, sigma, rng(tag, problem, KIND_XI))
    if source == "ones":
        g = np.ones((nrhs, n, n))
    else:
        g = np.stack([rng(tag, problem, KIND_G, r).standard_normal((n, n)) for r in range(nrhs)])
    return Problem(q=q, a=a, g=g, rho=rho, tag=tag, problem=problem)


def q6_exact_problem() -> Problem:
    """64 x 64 cells, sigma = 1 lognormal product field, g = 1."""
    return rough_problem(6, 1.0, TAG_Q6_EXACT, source="ones", rho=64)


def q9_rough_problem(nrhs: int = 1) -> Problem:
    """512 x 512 cells, sigma = 2 lognormal product field, N(0,1) cell source, radius 3."""
    return rough_problem(9, 2.0, TAG_Q9_ROUGH, nrhs=nrhs, rho=3)


def batch_problems(count: int = 256, nrhs: int = 64, levels=(6, 7, 8)) -> list[Problem]:
    """Independent problems of uneven depth, each with its own seeds."""
    out = []
    for p in range(count):
        q = int(rng(TAG_BATCH, p, KIND_Q).choice(levels))
        out.append(rough_problem(q, 1.0, TAG_BATCH, problem=p, nrhs=nrhs, rho=3))
    return out


def adjoint_problem(q: int = 10, tag: int = TAG_ADJOINT_Q10) -> Problem:
    """Lognormal product field with an observation coefficient drawn from its own stream."""
    pr = rough_problem(q, 1.0, tag, rho=3)
    n = 1 << q
    a_obs = product_field(n) * lognormal_factor(n, 1.0, rng(tag, 0, KIND_OBS))
    pr.extra["a_obs"] = a_obs
    fd = rng(tag, 0, KIND_FD)
    pr.extra["fd_cells"] = fd.choice(n * n, size=min(32, n * n), replace=False)
    return pr


def inclusion_problem(q: int = 11, nrhs: int = 16, tag: int = TAG_Q11_INCL, a_incl: float = 1.0e6) -> Problem:
    """Product field with high-contrast circular inclusions (a = a_incl inside, 1e6 by default)."""
    n = 1 << q
    a = product_field(n)
    mask = inclusion_mask(n, rng(tag, 0, KIND_INCL))
    a[mask] = a_incl
    g = np.stack([rng(tag, 0, KIND_G, r).standard_normal((n, n)) for r in range(nrhs)])
    return Problem(q=q, a=a, g=g, rho=4, tag=tag)
