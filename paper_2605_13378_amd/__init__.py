"""MI355X (gfx950) Jacobian-free Newton-Krylov hot path with AD and FD JVPs.

The method is that of Pasquale & Markidis, "Robust Matrix-Free Newton-Krylov
Solvers via Automatic Differentiation": Newton with backtracking line search
around restarted GMRES(m) whose only access to the Jacobian is a
Jacobian-vector product, computed either by forward-mode AD (dual-number
stencil kernels) or by finite differences.  All of it runs in hand-written HIP
kernels behind the C ABI of include/jfnk.h; ``jfnk`` is the Python binding.
"""

from .jfnk import (  # noqa: F401
    EPS_RULES,
    Batch,
    MODES,
    PRECISIONS,
    PROBLEM_IDS,
    Info,
    JfnkError,
    Options,
    Problem,
    Solver,
    default_options,
    exported_symbols,
    footprint_bytes,
    frequency_sweep,
    lib,
    make_problem,
    newton_solve_noalloc,
    problem_size,
)
