"""GPU parity of the Helmholtz-Kerr workload: -Lap E - k0^2 (eps_L + chi3 |E|^2) E = f with PEC
boundary nodes, k0 = 2 pi / 64 cells, eps_L = 1, chi3 in {0.01, 0.1}, Gaussian source, Newton
from E = 0 (the first step is the linear Helmholtz solve).

* 64 x 64 (the workload's cells per wavelength on a smaller grid): every Newton iterate against
  the oracle.  GMRES(30) needs ~900-1500 Arnoldi steps per Newton step on this indefinite
  operator, so the iterates depend on the summation order of the dot products: the oracle
  itself moves by ~3e-9 (FP64 settings) when only that order changes (order_spread,
  test_oracle_summation_order), and FP64 is compared at FACTOR times that ceiling.  FP32
  (complex64 storage and arithmetic, FP64 Givens and Newton update) at the 1e-5 contract
  against the oracle run with the FP32 tolerances.
* 128 x 128 is not compared: there unpreconditioned GMRES(30) does not reach the Krylov
  tolerance of the first (linear Helmholtz) step within 100 restarts, and the oracle itself ends
  50 Newton steps at a relative residual of 0.19, so there is no converged sequence to match.
* 1024 x 1024 (the workload itself): GMRES capped at one and at two restart cycles, the
  iterate against the oracle's capped run from the same state (FP64 1e-10, FP32 1e-5).
"""

import numpy as np
import pytest

import order_spread as OS
import workloads as W
from gpu_cases import dev, gpu_available, host, wdtype
from oracle import Problem, gmres_solve, jvp_ad, residual
from test_gpu_solver import compare_newton, solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("chi", [0.01, 0.1])
def test_kerr_c4_newton_64_f64(chi):
    name = f"kerr64_chi{chi}"
    spec, xp, src, opts, _, _, _ = OS.case(name)
    tol, tol_x = OS.gpu_bounds(name)
    info, ref = compare_newton(spec, xp, src, "f64", "ad", tol, tol_x=tol_x, orth="dcgs2", krylov_slack=0.15,
                               **opts)
    assert info["converged"] and ref.converged


@pytest.mark.parametrize("chi", [0.01, 0.1])
def test_kerr_c4_newton_64_f32(chi):
    """FP32 iterates at 1e-5.  Two FP32 effects are not parity failures and are bounded instead:
    the residual evaluated in FP32 cannot fall below its rounding floor (each of the five
    Laplacian terms, the Kerr term and f rounded at 2^-24, so ||F_fp32(x)|| ~ 3 * 2^-24
    (8 ||E|| + ||f||)), which the relative residual may meet near convergence; and FP32
    GMRES(30) on this indefinite operator stagnates above the 1e-6 Krylov tolerance (the
    paper's FP32 effect), so a step may run to the restart cap where the FP64-arithmetic oracle
    converges: Krylov counts are recorded, not compared."""
    spec, xp, src, opts, _, _, _ = OS.case(f"kerr64_chi{chi}")
    fnorm = float(np.linalg.norm(src))

    def floor(x_ref, f0):
        return 3 * 2.0 ** -24 * (8 * float(np.linalg.norm(x_ref)) + fnorm) / f0

    info, ref = compare_newton(spec, xp, src, "f32", "ad", 1e-5, orth="dcgs2", rho_floor=floor, counts=False,
                               **opts)
    assert info["converged"] and ref.converged
    assert all(a >= 0.5 * b for a, b in zip(info["lin_iters"], ref.lin_iters)), (info["lin_iters"], ref.lin_iters)


@pytest.mark.parametrize("prec,bound", [("f64", 1e-10), ("f32", 1e-5)])
def test_kerr_c4_gmres_capped_1024(prec, bound):
    spec = W.kerr_spec(1024, chi3=0.1, cells_per_wavelength=64.0)
    src = W.kerr_gaussian_source(1024)
    p = Problem.from_spec(spec)
    # a state with |E| > 0 at every node, so that the Kerr term enters J
    E = W.random_vector(p.n, 17, 0.5)
    xw = E if prec == "f64" else E.astype(np.float32).astype(np.float64)
    rhs = -residual(p, xw, None, src)
    if prec == "f32":
        rhs = rhs.astype(np.float32).astype(np.float64)
    mv = lambda v: jvp_ad(p, xw, v, None, src)[1]  # noqa: E731
    s = solver(spec, prec, None, src)
    for cycles in (1, 2):
        ref, ri = gmres_solve(mv, rhs, m=30, tol=1e-300, max_restarts=cycles, orth="dcgs2")
        dx, info = s.gmres(dev(xw, wdtype(prec)), dev(rhs, wdtype(prec)), m=30, tol=1e-300, max_restarts=cycles)
        assert info["krylov_iters"] == ri.iters == 30 * cycles and not info["converged"]
        err = float(np.linalg.norm(host(dx) - ref) / np.linalg.norm(ref))
        assert err <= bound, (cycles, err)
