"""Plain FP64 CPU oracle for the batched eddy-current UQ hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, links or runs anything from this package; only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark
do.  It shares no code with the GPU path: it re-derives the mesh, the
Karhunen-Loeve basis, the P1 element matrices, the time stepping, Parareal,
the MLMC estimator and the Picard iteration from the paper, in slow and
obviously checkable NumPy/SciPy code (banded Cholesky, LAPACK dpbtrf and
dpbtrs, for every linear solve).

Modules and the passages they follow (Hahn and Schoeps, "Multi-Level Monte
Carlo sampling with Parallel-in-Time Integration for Uncertainty
Quantification in Electric Machine Simulation"):

* ``mesh``       structured P1 triangulation of the unit square.
* ``kl``         separable exponential-covariance Karhunen-Loeve basis.
* ``fem``        Section II-A, Eqs. (1)-(5): M_sigma, K_nu, r.
* ``timestep``   Section II-A, Eqs. (6)-(7): implicit Euler; Section III-B,
                 Eq. (26): mean Joule loss.
* ``mlmc``       Section II-B, Eqs. (8)-(10): MC and MLMC estimators.
* ``parareal``   Section II-C, Eq. (12) with the active window and the
                 per-iteration propagator counts of Eqs. (13)-(14).
* ``picard``     nonlinear reluctivity of Eq. (1) (mu "possibly nonlinear").
* ``costmodel``  Section II-C/II-D, Eqs. (13)-(25) and the finite-core
                 speedup formula.

Every function here is pinned by a `-m "not gpu"` test against something
other than itself (closed forms, brute-force dense solves, identities,
numbers printed in the paper).  The one result with no such pin is the
paper's measured overall FE speedup (1.12), which the cost model does not
reproduce; it is reported as "parity unpinned" by the tests.
"""
