"""Pins of the oracle's sensitivity to summation order alone (order_spread.CASES): for each
case the iterates of the oracle and of the oracle run on the permuted system P F(P^T y) = 0 are
compared; the spread must lie between ceiling / 1000 (the sensitivity is real, so a tighter
GPU bound would measure rounding order, not correctness) and the recorded ceiling (the GPU
bound, FACTOR times the ceiling, is a small multiple of it).  A well-conditioned control case
stays at rounding level, so its GPU bound keeps the 1e-12 contract."""

import numpy as np
import pytest

import order_spread as OS
from gpu_cases import case as small_case
from oracle import NewtonOptions, Problem, newton_solve


def spread(spec, xp, src, opts, nperm=2, seed=7, orth="cgs2"):
    p = Problem.from_spec(spec)
    o = NewtonOptions.for_precision("f64", orth=orth, **opts)
    _, ref = newton_solve(p, xp, o, source=src, record=True)
    rng = np.random.default_rng(seed)
    d_rho = d_x = 0.0
    d_k = 0
    for _ in range(nperm):
        _, alt = newton_solve(p, xp, o, source=src, record=True, perm=rng.permutation(p.n))
        assert alt.newton_iters == ref.newton_iters and alt.converged == ref.converged
        for k in range(len(ref.rel_res)):
            d_rho = max(d_rho, abs(alt.rel_res[k] - ref.rel_res[k]))
            xr = ref.iterates[k]
            d_x = max(d_x, float(np.linalg.norm(alt.iterates[k] - xr)) / max(float(np.linalg.norm(xr)), 1e-300))
        d_k = max([d_k] + [abs(a - b) for a, b in zip(alt.lin_iters, ref.lin_iters)])
    return ref, d_rho, d_x, d_k


@pytest.mark.parametrize("name", sorted(OS.CASES))
def test_summation_order_spread(name):
    spec, xp, src, opts, c_rho, c_x, c_k = OS.case(name)
    ref, d_rho, d_x, d_k = spread(spec, xp, src, opts)
    assert ref.converged
    assert d_rho <= c_rho and d_x <= c_x and d_k <= c_k, (d_rho, d_x, d_k)
    assert d_x >= c_x / 1000.0, d_x


def test_well_conditioned_control_stays_at_rounding_level():
    spec, xp, src = small_case("grayscott", 64, 64)
    _, d_rho, d_x, d_k = spread(spec, xp, src, {})
    assert d_rho <= 1e-15 and d_x <= 1e-15 and d_k == 0


@pytest.mark.parametrize("n", [4, 6])
def test_tiny_maxwell_at_tight_krylov_tolerance_is_order_independent(n):
    # the grid the Maxwell per-iterate 1e-12 parity case uses (GMRES converges to 1e-13 in a
    # few dozen steps), with and without the CSLP preconditioner
    spec, xp, src = OS._maxwell(n)
    for pre in ("none", "cslp"):
        _, d_rho, d_x, _ = spread(spec, xp, src, dict(max_newton=20, precond=pre, tol_krylov=1e-13,
                                                       tol_newton=1e-10))
        assert d_rho <= 1e-14 and d_x <= 1e-13, (pre, d_rho, d_x)
