"""Writes inclusion_direct_noise.txt: how far apart two FP64 direct solves of
the inclusion workload land (discs of a = 1e6 on 10% of the cells over the
oscillatory product field of Section 5.1; 16 N(0,1) cell sources, the first
one solved here).

The stiffness matrix of such a coefficient has condition numbers near 1e10
(128 x 128 cells) and beyond, and its entries next to an inclusion carry the
rounding of sums of terms 1e6 times apart, so FP64 itself fixes the solution
only to some digits.  Two sparse LU solves with different fill-reducing
orderings (and FP64 iterative refinement) measure that floor; a comparison
with the direct solve cannot be asked to go below it.  Calls only the oracle
and the seeded input generator.

Usage: python tests/golden/make_inclusion_noise.py [q ...]   (default 7 9 11)
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic as S  # noqa: E402
from oracle import fem  # noqa: E402


def noise(q: int) -> float:
    pr = S.inclusion_problem(q=q, nrhs=1, a_incl=1e6)
    fe = fem.assemble(pr.a)
    b = fem.load_cellwise(pr.g[0], fe.h)
    u1 = fem.DirectSolver(fe.A, refine=2).solve(b)
    u2 = fem.DirectSolver(fe.A, refine=3, ordering="COLAMD").solve(b)
    return float(np.linalg.norm(u1 - u2) / np.linalg.norm(u1))


def main(qs):
    path = os.path.join(HERE, "inclusion_direct_noise.txt")
    lines = ["# q  relative l2 distance between two FP64 direct solves (MMD_AT_PLUS_A + 2 refinement steps,",
             "#    COLAMD + 3 refinement steps) of the inclusion workload, first right-hand side"]
    for q in qs:
        v = noise(q)
        print(q, v, flush=True)
        lines.append(f"{q} {v:.6e}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main([int(x) for x in sys.argv[1:]] or [7, 9, 11])
