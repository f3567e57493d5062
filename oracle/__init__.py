"""Plain, slow, FP64 CPU oracle of the JFNK hot path — TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import, call or run anything in this package.  The HIP library never does, and
this package shares no code with it; both take their inputs from the seeded
``workloads`` generators only.

Contents, each following the paper (Pasquale & Markidis, "Robust Matrix-Free
Newton-Krylov Solvers via Automatic Differentiation"):

* ``problems``: the discrete residuals F(x^k, x*) (Section 2; Section 3.2;
  Appendix A) — 1D/2D viscous Burgers, Gray-Scott, scalar Helmholtz-Kerr,
  scalar u^3 reaction-diffusion with Dirichlet boundaries.
* ``dual``: forward-mode dual numbers (the AD JVP of Section 2).
* ``jvp``: AD and FD Jacobian-vector products and the FD step rules.
* ``gmres``: restarted GMRES(m), CGS2 Arnoldi, Givens least squares.
* ``bicgstab``: BiCGSTAB, the paper's short-recurrence nonsymmetric method.
* ``cg``: conjugate gradients for the SPD reaction-diffusion linearization.
* ``precond``: the block-diagonal CSLP preconditioner of the Maxwell-Kerr
  problem (Appendix A.4) and its scalar form for the Helmholtz-Kerr
  workload, applied on the right of GMRES.
* ``newton``: inexact Newton with backtracking line search and the
  failure classification of Section 3.4.
* ``sweep``: the Maxwell frequency continuation (Section 3.1's outer loop,
  the Born start of Appendix A.4, the 20% failure rule of Section 3.4).

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against closed forms, independent hand-derived Jacobians, complex-step
derivatives, dense linear solves, FFT/DST closed forms, manufactured solutions
and convergence-order properties.  The line-search constants are the one part
the paper does not fix: they are a reading, pinned only by the Armijo property
(parity of the constants themselves unpinned).
"""

from . import bicgstab, cg, dual, gmres, jvp, newton, precond, problems, sweep  # noqa: F401
from .bicgstab import BicgstabInfo, bicgstab as bicgstab_solve  # noqa: F401
from .cg import CgInfo, cg as cg_solve  # noqa: F401
from .gmres import GmresInfo, gmres as gmres_solve  # noqa: F401
from .jvp import EPS_MACH, EPS_NORMALIZED, EPS_PAPER, fd_step, jvp_ad, jvp_fd  # noqa: F401
from .newton import NewtonInfo, NewtonOptions, newton_solve, run_failed, step_failed  # noqa: F401
from .precond import cslp_diagonal, cslp_solve  # noqa: F401
from .problems import Problem, residual  # noqa: F401
from .sweep import SweepInfo, frequency_sweep  # noqa: F401
