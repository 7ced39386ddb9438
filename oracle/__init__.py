"""FP64 CPU oracle for the space-time multigrid (STMG) method of Appel & Alexandersen,
"Space-Time Multigrid Methods Suitable for Topology Optimisation of Transient Heat
Conduction" (arXiv 2505.10168).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import or call this
package: only the test-suite, the smoke check and the benchmark's CPU-baseline leg
use it.  It is a plain, slow, literal transcription of the paper's definitions in
NumPy float64 and shares no code with the HIP library.

Modules
-------
discretisation : SIMP map, BE-FE all-at-once operator J and its transpose, Dirichlet
                 treatment of Appendix A, load vector, direct (time-stepping) solve.
multigrid      : coarsening strategies (Algorithms 2-4), rediscretisation methods
                 (C/B interpolation, K/D/R/P reassembly), damped Jacobi, Algorithm 1
                 V-cycle and the solve loop with the termination rule of Section 3.1.
sensitivity    : objective, adjoint right-hand side and the discrete-adjoint gradient
                 of Section 7.
design         : optimality-criteria design update and design loop for the
                 optimisation problem of Section 7.

Parity status
-------------
Every function is pinned by a CPU test against something other than itself (closed
forms, brute-force dense algebra, printed values of the paper, invariants), except
the V-cycle iterates themselves: the paper prints no iterates or residual histories,
so their values are "parity unpinned" beyond the pins of each component and the
fixed-point/linearity invariants of the cycle.
"""
from .discretisation import *  # noqa: F401,F403
from .multigrid import *  # noqa: F401,F403
from .sensitivity import *  # noqa: F401,F403
from .design import *  # noqa: F401,F403
