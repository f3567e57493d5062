"""GPU parity of BiCGSTAB (standalone and inside Newton) against the oracle.

Parity contract:
  * standalone, FP64 AD: the GPU iterate within 1e-8 (relative) of the
    oracle's BiCGSTAB iterate for the same operator and right-hand side,
    iteration counts within one (a tolerance tie can move the stop by one
    iteration or half step), and the GPU iterate's true residual, measured
    with the oracle's FP64 JVP, at most 2 tol ||rhs||;
  * standalone, FP32 AD: the oracle run in FP64 on the FP32-rounded inputs,
    iterate within 1e-4 at tol 1e-5 (FP32 recurrences drift by a few ulps
    per iteration);
  * Newton with BiCGSTAB: per iterate as for GMRES (FP64 AD 1e-10, FP32 AD
    1e-5), the same number of Newton iterates, Krylov counts within 10%;
  * statuses: zero right-hand side, iteration cap, non-finite input, the
    options the library rejects.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, gpu_available, host, wdtype
from oracle import Problem, bicgstab_solve, jvp_ad, residual
from test_gpu_solver import compare_newton, solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def linear_case(kind, nx, ny, prec, seed=81):
    spec, xp, src = case(kind, nx, ny)
    p = Problem.from_spec(spec)
    x = xp + 0.05 * W.random_vector(p.n, seed)
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    rhs = -residual(p, xw, xp, src)
    if prec == "f32":
        rhs = rhs.astype(np.float32).astype(np.float64)
    return spec, xp, src, p, xw, rhs


@pytest.mark.parametrize("kind,nx,ny", [("grayscott", 64, 40), ("grayscott", 130, 37), ("burgers2d", 48, 40),
                                        ("burgers1d", 300, None)])
def test_bicgstab_parity_f64_ad(kind, nx, ny):
    spec, xp, src, p, xw, rhs = linear_case(kind, nx, ny, "f64")
    tol = 1e-10
    matvec = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    ref, rinfo = bicgstab_solve(matvec, rhs, tol=tol, maxiter=400)
    s = solver(spec, "f64", xp, src, m=8)
    dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=tol, max_iters=400)
    assert rinfo.converged and info["converged"], (rinfo, info)
    assert abs(info["krylov_iters"] - rinfo.iters) <= 1, (info["krylov_iters"], rinfo.iters)
    d = host(dx)
    err = np.linalg.norm(d - ref) / np.linalg.norm(ref)
    assert err <= 1e-8, err
    true_res = np.linalg.norm(rhs - matvec(d))
    assert true_res <= 2 * tol * np.linalg.norm(rhs), true_res / np.linalg.norm(rhs)
    assert abs(info["f0_norm"] - np.linalg.norm(rhs)) <= 1e-13 * np.linalg.norm(rhs)


def test_bicgstab_kerr_capped_f64_ad():
    # the Helmholtz-Kerr operator at 8 cells per wavelength is indefinite and
    # BiCGSTAB does not converge on it (residual history with spikes, the
    # paper's robustness remark): compare the iterates after a fixed count.
    # A relative perturbation of one ulp in every JVP moves the oracle's own
    # iterate by ~1e-15 after 6 iterations, ~1e-10 after 8-9 and ~1e-2 after
    # 15, so the counts stay at or below 6.
    spec, xp, src, p, xw, rhs = linear_case("kerr", 40, 36, "f64")
    matvec = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    s = solver(spec, "f64", xp, src, m=8)
    for cap in (3, 6):
        ref, rinfo = bicgstab_solve(matvec, rhs, tol=1e-12, maxiter=cap)
        dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=1e-12, max_iters=cap)
        assert not rinfo.converged and not info["converged"] and info["krylov_iters"] == cap == rinfo.iters
        assert np.linalg.norm(host(dx) - ref) <= 1e-8 * np.linalg.norm(ref)
        assert abs(info["final_res"] - rinfo.res[-1]) <= 1e-8 * rinfo.res[-1]


@pytest.mark.parametrize("kind,nx,ny", [("grayscott", 64, 40), ("burgers2d", 48, 40), ("burgers1d", 300, None)])
def test_bicgstab_parity_f32_ad(kind, nx, ny):
    spec, xp, src, p, xw, rhs = linear_case(kind, nx, ny, "f32")
    tol = 1e-5
    ref, rinfo = bicgstab_solve(lambda v: jvp_ad(p, xw, v, xp, src)[1], rhs, tol=tol, maxiter=400)
    s = solver(spec, "f32", xp, src, m=8)
    dx, info = s.bicgstab(dev(xw, wdtype("f32")), dev(rhs, wdtype("f32")), tol=tol, max_iters=400)
    assert rinfo.converged and info["converged"], (rinfo, info)
    assert abs(info["krylov_iters"] - rinfo.iters) <= 2, (info["krylov_iters"], rinfo.iters)
    err = np.linalg.norm(host(dx) - ref) / np.linalg.norm(ref)
    assert err <= 1e-4, err


@pytest.mark.parametrize("rule", ["paper", "normalized"])
def test_bicgstab_parity_f64_fd(rule):
    from oracle import EPS_MACH, fd_step, jvp_fd

    spec, xp, src, p, xw, rhs = linear_case("grayscott", 64, 40, "f64")
    F0 = residual(p, xw, xp, src)
    tol = 1e-6
    ref, rinfo = bicgstab_solve(lambda v: jvp_fd(p, xw, v, fd_step(rule, EPS_MACH["f64"], xw, v), xp, src, Fx=F0),
                                rhs, tol=tol, maxiter=400)
    s = solver(spec, "f64", xp, src, m=8)
    dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=tol, max_iters=400, mode="fd",
                          eps_rule=rule)
    assert rinfo.converged and info["converged"]
    err = np.linalg.norm(host(dx) - ref) / np.linalg.norm(ref)
    assert err <= 1e-6, err


def test_bicgstab_cap_zero_rhs_and_nonfinite():
    spec, xp, src, p, xw, rhs = linear_case("grayscott", 32, 32, "f64")
    s = solver(spec, "f64", xp, src, m=5)
    matvec = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    # iteration cap: the iterate after exactly three iterations
    ref, rinfo = bicgstab_solve(matvec, rhs, tol=1e-30, maxiter=3)
    dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=1e-30, max_iters=3)
    assert not info["converged"] and info["krylov_iters"] == 3 == rinfo.iters
    assert np.linalg.norm(host(dx) - ref) <= 1e-12 * np.linalg.norm(ref)
    assert abs(info["final_res"] - rinfo.res[-1]) <= 1e-10 * rinfo.res[-1]
    # no iterations allowed
    dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=1e-8, max_iters=0)
    assert not info["converged"] and info["krylov_iters"] == 0 and not host(dx).any()
    # zero right-hand side
    dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(np.zeros(p.n), wdtype("f64")), tol=1e-8)
    assert info["converged"] and info["krylov_iters"] == 0 and not host(dx).any()
    # non-finite right-hand side and non-finite state
    bad = rhs.copy()
    bad[5] = np.nan
    dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(bad, wdtype("f64")), tol=1e-8)
    assert info["nonfinite"] and not info["converged"] and info["krylov_iters"] == 0
    xbad = xw.copy()
    xbad[7] = np.inf
    dx, info = s.bicgstab(dev(xbad, wdtype("f64")), dev(rhs, wdtype("f64")), tol=1e-8)
    assert info["nonfinite"] and not info["converged"]
    # the solver is still usable afterwards
    dx, info = s.bicgstab(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=1e-10, max_iters=400)
    ref, rinfo = bicgstab_solve(matvec, rhs, tol=1e-10, maxiter=400)
    assert info["converged"] and np.linalg.norm(host(dx) - ref) <= 1e-8 * np.linalg.norm(ref)


def test_bicgstab_rejected_configurations():
    from paper_2605_13378_amd import JfnkError

    spec, xp, src, p, xw, rhs = linear_case("grayscott", 32, 32, "f64")
    small = solver(spec, "f64", xp, src, m=4)
    with pytest.raises(JfnkError, match="m >= 5"):
        small.bicgstab(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")))
    with pytest.raises(JfnkError, match="m >= 5"):
        small.newton_solve(dev(xp, wdtype("f64")), krylov="bicgstab", m=4)
    half = solver(spec, "f16s", xp, src, m=8)
    with pytest.raises(JfnkError, match="FP64 or FP32"):
        half.newton_solve(dev(xp, wdtype("f64")), krylov="bicgstab", m=8)
    s = solver(spec, "f64", xp, src, m=8)
    with pytest.raises(JfnkError, match="GMRES only"):
        s.newton_solve(dev(xp, wdtype("f64")), krylov="bicgstab", engine="single", m=8)


@pytest.mark.parametrize("kind,nx,ny,prec,tol", [
    ("grayscott", 64, 64, "f64", 1e-10), ("grayscott", 130, 37, "f64", 1e-10), ("burgers2d", 48, 40, "f64", 1e-10),
    ("burgers1d", 256, None, "f64", 1e-10), ("grayscott", 64, 64, "f32", 1e-5), ("burgers1d", 256, None, "f32", 1e-5),
])
def test_newton_bicgstab(kind, nx, ny, prec, tol):
    spec, xp, src = case(kind, nx, ny)
    info, ref = compare_newton(spec, xp, src, prec, "ad", tol, krylov="bicgstab", krylov_slack=0.1,
                               tol_krylov=1e-10 if prec == "f64" else 1e-6)
    assert info["converged"] and info["restarts"] == 0


def test_newton_bicgstab_kerr_f64():
    # the well-posed small Kerr case of the GMRES tests (Newton from E = 0)
    spec = dict(W.kerr_spec(12, chi3=0.3, cells_per_wavelength=64.0, eps_im=0.05), ny=10)
    src = W.kerr_gaussian_source(12, amp=1.0, sigma=2.0, ny=10)
    info, ref = compare_newton(spec, np.zeros(2 * 12 * 10), src, "f64", "ad", 1e-10, krylov="bicgstab",
                               krylov_slack=0.1, tol_krylov=1e-10, max_newton=20)
    assert info["converged"]


def test_newton_bicgstab_f64_fd():
    # normalized FD step at tol_K 1e-6: above the FD noise floor in every
    # Newton step (with the paper's step the last solve stagnates on FD noise)
    spec, xp, src = case("grayscott", 64, 64)
    info, ref = compare_newton(spec, xp, src, "f64", "fd", 1e-7, eps_rule="normalized", krylov="bicgstab",
                               krylov_slack=0.2, tol_krylov=1e-6)
    assert info["converged"]


def test_full_size_grayscott_f64_ad_bicgstab():
    """Gray-Scott 1024^2, FP64, AD, Newton with BiCGSTAB against the oracle, per iterate."""
    spec, xp, src = W.config("grayscott")
    info, ref = compare_newton(spec, xp, src, "f64", "ad", 1e-10, krylov="bicgstab", krylov_slack=0.1)
    assert info["converged"]
