"""Plain CPU FP64 oracle for the HPS-as-multigrid method (test infrastructure only).

This package is a slow, deliberately unoptimised restatement of the method of
"Towards a Multigrid Preconditioner Interpretation of Hierarchical
Poincare-Steklov Solvers" (Lucero Lorca), written with NumPy/SciPy in complex
double precision.  It exists only to check the HIP implementation: the only
permitted callers are the test suite, the smoke entry point and the CPU-baseline
leg of the benchmark.  Product code must never import it, and it shares no code
with the HIP path (it imports nothing from the product package except the
seeded input generators, which hold none of the method's arithmetic).

Modules, in the paper's order:

* ``gll``       -- 1D GLL nodes, weights, differentiation matrix (Sec. 3.1).
* ``mesh``      -- element/side/box geometry, merge levels, canonical slots
                   (Sec. 3.2, Sec. 4.2 and Fig. 1).
* ``leaf``      -- element operator, impedance rows, leaf ItI map T and load H
                   (Sec. 3.1, eq. ItIOperator).
* ``skeleton``  -- skeleton system M_l g = RHS (Sec. 3.2, eq. faceequations).
* ``merge``     -- pair merge by Schur complement (Sec. 4.1, eqs.
                   localfacesystem/globalfacesystem) and the level hierarchy.
* ``direct``    -- direct HPS: upward merges, downward solve (Sec. 4.2).
* ``multigrid`` -- MG(M) = F + P S^-1 R (I - M F) recursion (Sec. 4.3).
* ``krylov``    -- k-step GMRES (coarse solve) and flexible GMRES (Sec. 4.3/5).
* ``brute``     -- element-DOF brute-force system, independent of ItI maps.

Pins: every function is checked by ``tests/test_oracle_*.py`` against facts
fixed by mathematics or printed in the paper (closed forms, exact polynomial
reproduction, brute force, library routines, the Fig. 1 sparsity patterns).
"""
