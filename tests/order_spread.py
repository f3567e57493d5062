"""How far the oracle's own Newton iterates move when only the summation order of its dot
products and norms changes, and the GPU parity bounds derived from it.

The oracle solves the permuted system P F(P^T y) = 0 (``newton_solve(..., perm=P)``): the same
method and, in exact arithmetic, the same iterates, with every reduction summed in another
order.  For each case below the ceiling is about twice the largest spread measured over seeded
permutations (test_oracle_summation_order pins the spread between ceiling / 1000 and the
ceiling); a GPU run, whose reductions are summed in yet another order, is compared with the
oracle at FACTOR times the ceiling (and never looser than needed: at most the contract's
1e-12 where the ceiling allows it).  On a well-conditioned problem the spread is at rounding
level and the contract bound applies unchanged.
"""

from __future__ import annotations

import numpy as np

import workloads as W

FACTOR = 5.0

# name -> (spec, x_prev, source, options dict, ceiling of max_k |rho_k - rho'_k|,
#          ceiling of max_k ||x_k - x'_k|| / ||x_k||, ceiling of the per-step Krylov-count change)


def _kerr12(cpw, chi):
    spec = dict(W.kerr_spec(12, chi3=chi, cells_per_wavelength=cpw, eps_im=0.05), ny=10)
    return spec, np.zeros(240), W.kerr_gaussian_source(12, amp=1.0, sigma=2.0, ny=10)


def _maxwell(n):
    return W.maxwell_spec(n, omega=2.5), np.zeros(4 * n * n), W.maxwell_source(n, omega=2.5)


def _maxwell12x10():
    spec = W.maxwell_spec(12, omega=2.5, ny=10)
    return spec, np.zeros(4 * 12 * 10), W.maxwell_source(12, omega=2.5, ny=10)


def _kerr_c4(n, chi):
    # the Helmholtz-Kerr workload's physics (k0 = 2 pi / 64 cells, eps_L = 1) on a smaller grid
    return W.kerr_spec(n, chi3=chi, cells_per_wavelength=64.0), np.zeros(2 * n * n), W.kerr_gaussian_source(n)


CASES = {
    "kerr12x10_cpw64_chi0.3": (_kerr12, (64.0, 0.3), dict(max_newton=20), 4e-15, 5e-12, 2),
    "kerr12x10_cpw32_chi1.0": (_kerr12, (32.0, 1.0), dict(max_newton=20), 1.5e-11, 7e-11, 6),
    "maxwell16": (_maxwell, (16,), dict(max_newton=20), 2e-9, 4e-8, 40),
    "maxwell16_cslp": (_maxwell, (16,), dict(max_newton=20, precond="cslp"), 2e-9, 4e-8, 40),
    # measured 3.6e-12 / 1.5e-10 / 5 (three permutations, both Gram-Schmidt forms)
    "maxwell12x10_cslp": (_maxwell12x10, (), dict(precond="cslp", tol_newton=1e-6, tol_krylov=1e-8,
                                                  max_restarts=20, max_newton=8), 8e-12, 3e-10, 8),
    "kerr64_chi0.01": (_kerr_c4, (64, 0.01), dict(max_newton=50), 3e-9, 6e-9, 120),
    "kerr64_chi0.1": (_kerr_c4, (64, 0.1), dict(max_newton=50), 6e-9, 6e-9, 160),
    # with the CSLP preconditioner; measured (three permutations, both Gram-Schmidt forms):
    # 1.2e-11 / 4.8e-11 / 12 on 12 x 10, 5.3e-9 / 4.8e-9 / 62 on 64 x 64
    "kerr12x10_cpw32_chi1.0_cslp": (_kerr12, (32.0, 1.0), dict(max_newton=20, precond="cslp"), 2.5e-11, 1e-10, 24),
    "kerr64_chi0.1_cslp": (_kerr_c4, (64, 0.1), dict(max_newton=50, precond="cslp"), 1.2e-8, 1e-8, 130),
}


def case(name):
    build, args, opts, crho, cx, ck = CASES[name]
    spec, xp, src = build(*args)
    return spec, xp, src, opts, crho, cx, ck


def gpu_bounds(name):
    """(rho bound, x bound) for a GPU-vs-oracle per-iterate comparison in FP64."""
    _, _, _, _, crho, cx, _ = case(name)
    return max(1e-12, FACTOR * crho), max(1e-12, FACTOR * cx)


# Frequency continuation (oracle.frequency_sweep) of the Maxwell-Kerr problem on 16 x 16 at
# omega = 2.5, 3.0, 3.5, 4.0 (Born start at 2.5; FP64 tolerances, Newton cap 20):
# name -> (preconditioner, ceiling of max_i ||E_i - E'_i|| / ||E_i||, ceiling of the
# per-frequency Krylov-count change).  Measured: fields 1.25e-10 / 1.22e-10, counts 89 / 169.
SWEEP_OMEGAS = (2.5, 3.0, 3.5, 4.0)
SWEEP_CASES = {
    "maxwell16_sweep": ("none", 2.5e-10, 200),
    "maxwell16_sweep_cslp": ("cslp", 2.5e-10, 200),
}


def sweep_case(name, n=16):
    """(problem specs, sources, oracle options dict, field ceiling, count ceiling)."""
    pc, cx, ck = SWEEP_CASES[name]
    specs = [W.maxwell_spec(n, omega=om) for om in SWEEP_OMEGAS]
    srcs = [W.maxwell_source(n, omega=om) for om in SWEEP_OMEGAS]
    return specs, srcs, dict(max_newton=20, precond=pc), cx, ck


def sweep_gpu_bounds(name):
    """(field bound, Krylov-count slack) of a GPU-vs-oracle sweep comparison."""
    _, _, _, cx, ck = sweep_case(name)
    return FACTOR * cx, int(FACTOR * ck)
