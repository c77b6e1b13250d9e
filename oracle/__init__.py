"""Plain, slow, FP64 CPU oracle for the gamblet hierarchy and solve.

TEST INFRASTRUCTURE ONLY. Nothing on the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline
leg of ``bench.py`` use it, to check and to time against the HIP library.
It shares no code, tables or constants with ``paper_1503_03467_amd``; the
two meet only through the seeded inputs of ``synthetic``.

Modules
-------
``fem``       Q1 finite elements on the unit square (Section 5.1): stiffness,
              load, Dirichlet lifting, direct sparse solve, adjoint gradient
              and a cancellation-free finite-difference check.
``gamblets``  The index tree and measurement aggregation (Definition 4.1,
              Construction 4.2), the subband matrices W (Constructions
              4.11/4.13), the exact gamblet transform (Algorithm 1 with the
              level-q initialisation psi = nodal basis allowed in Section
              5.2), the localized transform (Algorithm 2, Definition 5.3) and
              the subband solve (Theorem 4.15), the gamblet transform and
              compression of the discussion of Example 5.1.
``mass_inverse`` Level-q gamblets from the localized mass inverse
              (Algorithms 1-2, Definition 5.2).

Every function is pinned by a test in ``tests/test_oracle_*.py`` against
something other than itself: closed forms (sine-transform solution of the
constant-coefficient problem, the identities of Theorem 4.8), brute force on
tiny inputs (quadrature of the element integrals, KKT systems of the
constrained energy minimisation, dense exact gamblets), the patch box sizes of
Definition 5.3, and special cases that reduce to the exact hierarchy or to a
direct solve.  No function is left unpinned.
"""
