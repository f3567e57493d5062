"""GPU parity of conjugate gradients and of the reaction-diffusion problem's
Newton solves (CG, GMRES and BiCGSTAB, the paper's twelve-combination
problem) against the oracle.

Parity contract:
  * standalone CG, FP64 AD: iterate within 1e-10 (relative) of the oracle's
    CG iterate for the same operator and right-hand side (the operator is SPD
    and well conditioned, so rounding differences do not grow), iteration
    counts within one, true residual (oracle FP64 JVP) at most 2 tol ||rhs||;
    FP32 AD within 1e-5 at tol 1e-6; FD with both step rules within 1e-6;
  * statuses: cap (exact iterate after three iterations), zero and
    non-finite inputs, the indefinite Helmholtz-Kerr operator reported as a
    breakdown at the same iteration as the oracle, rejected configurations;
  * Newton per iterate on the reaction-diffusion problem with each Krylov
    method (FP64 AD 1e-10, FP32 AD 1e-5, FD with the normalized step 1e-7),
    both engines for GMRES, and the 512^2 workload in FP64.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, gpu_available, host, wdtype
from oracle import Problem, cg_solve, jvp_ad, residual
from test_gpu_solver import compare_newton, solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def linear_case(kind, nx, ny, prec, seed=81):
    spec, xp, src = case(kind, nx, ny)
    p = Problem.from_spec(spec)
    noise = 0.05 * W.random_vector(p.n, seed)
    if kind == "rd2d":
        # keep the homogeneous Dirichlet values: J is then SPD on the iterates
        inner = np.zeros((p.ny, p.nx))
        inner[1:-1, 1:-1] = 1.0
        noise = noise * inner.ravel()
    x = xp + noise
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    rhs = -residual(p, xw, xp, src)
    if prec == "f32":
        rhs = rhs.astype(np.float32).astype(np.float64)
    return spec, xp, src, p, xw, rhs


@pytest.mark.parametrize("nx,ny", [(64, 64), (130, 37), (1024, 12), (3, 3)])
def test_cg_parity_f64_ad(nx, ny):
    spec, xp, src, p, xw, rhs = linear_case("rd2d", nx, ny, "f64")
    tol = 1e-10
    matvec = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    ref, rinfo = cg_solve(matvec, rhs, tol=tol, maxiter=400)
    s = solver(spec, "f64", xp, src, m=4)
    dx, info = s.cg(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=tol, max_iters=400)
    assert rinfo.converged and info["converged"], (rinfo, info)
    assert abs(info["krylov_iters"] - rinfo.iters) <= 1, (info["krylov_iters"], rinfo.iters)
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 1e-10 * np.linalg.norm(ref)
    assert np.linalg.norm(rhs - matvec(d)) <= 2 * tol * np.linalg.norm(rhs)
    assert abs(info["f0_norm"] - np.linalg.norm(rhs)) <= 1e-13 * np.linalg.norm(rhs)


@pytest.mark.parametrize("nx,ny", [(64, 64), (130, 37)])
def test_cg_parity_f32_ad(nx, ny):
    spec, xp, src, p, xw, rhs = linear_case("rd2d", nx, ny, "f32")
    tol = 1e-6
    ref, rinfo = cg_solve(lambda v: jvp_ad(p, xw, v, xp, src)[1], rhs, tol=tol, maxiter=400)
    s = solver(spec, "f32", xp, src, m=4)
    dx, info = s.cg(dev(xw, wdtype("f32")), dev(rhs, wdtype("f32")), tol=tol, max_iters=400)
    assert rinfo.converged and info["converged"], (rinfo, info)
    assert abs(info["krylov_iters"] - rinfo.iters) <= 2
    assert np.linalg.norm(host(dx) - ref) <= 1e-5 * np.linalg.norm(ref)


@pytest.mark.parametrize("rule", ["paper", "normalized"])
def test_cg_parity_f64_fd(rule):
    from oracle import EPS_MACH, fd_step, jvp_fd

    spec, xp, src, p, xw, rhs = linear_case("rd2d", 64, 64, "f64")
    F0 = residual(p, xw, xp, src)
    tol = 1e-6
    ref, rinfo = cg_solve(lambda v: jvp_fd(p, xw, v, fd_step(rule, EPS_MACH["f64"], xw, v), xp, src, Fx=F0), rhs,
                          tol=tol, maxiter=400)
    s = solver(spec, "f64", xp, src, m=4)
    dx, info = s.cg(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=tol, max_iters=400, mode="fd",
                    eps_rule=rule)
    assert rinfo.converged and info["converged"]
    assert np.linalg.norm(host(dx) - ref) <= 1e-6 * np.linalg.norm(ref)


def test_cg_cap_zero_nonfinite_and_indefinite():
    spec, xp, src, p, xw, rhs = linear_case("rd2d", 32, 32, "f64")
    s = solver(spec, "f64", xp, src, m=2)
    matvec = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    ref, rinfo = cg_solve(matvec, rhs, tol=1e-30, maxiter=3)
    dx, info = s.cg(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), tol=1e-30, max_iters=3)
    assert not info["converged"] and info["krylov_iters"] == 3 == rinfo.iters
    assert np.linalg.norm(host(dx) - ref) <= 1e-13 * np.linalg.norm(ref)
    assert abs(info["final_res"] - rinfo.res[-1]) <= 1e-11 * rinfo.res[-1]
    dx, info = s.cg(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), max_iters=0)
    assert not info["converged"] and info["krylov_iters"] == 0 and not host(dx).any()
    dx, info = s.cg(dev(xw, wdtype("f64")), dev(np.zeros(p.n), wdtype("f64")))
    assert info["converged"] and info["krylov_iters"] == 0 and not host(dx).any()
    bad = rhs.copy()
    bad[3] = np.nan
    dx, info = s.cg(dev(xw, wdtype("f64")), dev(bad, wdtype("f64")))
    assert info["nonfinite"] and not info["converged"] and info["krylov_iters"] == 0
    # the indefinite Helmholtz-Kerr operator: (p, J p) < 0 in the second iteration
    spec_k, xp_k, src_k, p_k, xw_k, rhs_k = linear_case("kerr", 40, 36, "f64")
    ref, rinfo = cg_solve(lambda v: jvp_ad(p_k, xw_k, v, xp_k, src_k)[1], rhs_k, tol=1e-10, maxiter=100)
    assert rinfo.breakdown
    sk = solver(spec_k, "f64", xp_k, src_k, m=2)
    dx, info = sk.cg(dev(xw_k, wdtype("f64")), dev(rhs_k, wdtype("f64")), tol=1e-10)
    assert info["breakdown"] and not info["converged"] and info["krylov_iters"] == rinfo.iters
    assert np.linalg.norm(host(dx) - ref) <= 1e-12 * np.linalg.norm(ref)


def test_cg_rejected_configurations():
    from paper_2605_13378_amd import JfnkError

    spec, xp, src, p, xw, rhs = linear_case("rd2d", 16, 16, "f64")
    one = solver(spec, "f64", xp, src, m=1)
    with pytest.raises(JfnkError, match="m >= 2"):
        one.cg(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")))
    half = solver(spec, "f16s", xp, src, m=8)
    with pytest.raises(JfnkError, match="FP64 or FP32"):
        half.newton_solve(dev(xp, wdtype("f64")), krylov="cg", m=8)
    s = solver(spec, "f64", xp, src, m=8)
    with pytest.raises(JfnkError, match="GMRES only"):
        s.newton_solve(dev(xp, wdtype("f64")), krylov="cg", engine="single", m=8)


@pytest.mark.parametrize("krylov", ["cg", "gmres", "bicgstab"])
@pytest.mark.parametrize("nx,ny,prec,tol", [(64, 64, "f64", 1e-10), (130, 37, "f64", 1e-10), (64, 64, "f32", 1e-5)])
def test_newton_reaction_diffusion(krylov, nx, ny, prec, tol):
    spec, xp, src = case("rd2d", nx, ny)
    info, ref = compare_newton(spec, xp, src, prec, "ad", tol, krylov=krylov, krylov_slack=0.1,
                               tol_krylov=1e-10 if prec == "f64" else 1e-6)
    assert info["converged"]


@pytest.mark.parametrize("engine", ["multi", "single"])
def test_newton_reaction_diffusion_gmres_engines(engine):
    spec, xp, src = case("rd2d", 12, 10)
    info, ref = compare_newton(spec, xp, src, "f64", "ad", 1e-12, engine=engine, tol_krylov=1e-12,
                               tol_newton=1e-10)
    assert info["converged"]


def test_newton_cg_f64_fd():
    spec, xp, src = case("rd2d", 64, 64)
    info, ref = compare_newton(spec, xp, src, "f64", "fd", 1e-7, eps_rule="normalized", krylov="cg",
                               krylov_slack=0.2, tol_krylov=1e-6)
    assert info["converged"]


def test_full_size_reaction_diffusion_f64_ad_cg():
    """The paper's GPU reaction-diffusion grid (512^2), FP64, AD, Newton-CG, per iterate."""
    spec, xp, src = W.config("rd2d")
    info, ref = compare_newton(spec, xp, src, "f64", "ad", 1e-10, krylov="cg", krylov_slack=0.1)
    assert info["converged"]
