"""GPU parity of the Su-Olson radiation-diffusion problem (Appendix A.2) against the oracle.

Element-wise residual/JVP parity runs in test_gpu_kernels (the Su-Olson rows);
here: Newton per iterate with GMRES (both Gram-Schmidt forms and both engines)
and BiCGSTAB (FP64 AD 1e-12, FP32 AD 1e-5), the affine residual's property that
the FD JVP equals the AD JVP up to rounding at the paper's 512^2 grid, and FD
Newton reaching the AD iterate.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, gpu_available, host, wdtype
from oracle import EPS_MACH, Problem
from test_gpu_solver import compare_newton, solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("krylov,orth", [("gmres", "dcgs2"), ("gmres", "cgs2"), ("bicgstab", "cgs2")])
@pytest.mark.parametrize("nx,ny,prec,tol", [(64, 64, "f64", 1e-12), (130, 37, "f64", 1e-12), (64, 64, "f32", 1e-5)])
def test_newton_suolson(krylov, orth, nx, ny, prec, tol):
    spec, xp, src = case("suolson", nx, ny)
    info, ref = compare_newton(spec, xp, src, prec, "ad", tol, krylov=krylov, orth=orth, krylov_slack=0.1)
    assert info["converged"] and info["newton_iters"] == 1


@pytest.mark.parametrize("engine", ["multi", "single"])
def test_newton_suolson_engines(engine):
    spec, xp, src = case("suolson", 12, 10)
    compare_newton(spec, xp, src, "f64", "ad", 1e-12, engine=engine)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_suolson_fd_equals_ad_full_size(prec):
    spec, x0, src = W.config("suolson")
    p = Problem.from_spec(spec)
    s = solver(spec, prec, x0, src)
    x = x0 + 0.01 * W.random_vector(p.n, 5)
    v = W.random_vector(p.n, 6)
    xd, vd = dev(x, wdtype(prec)), dev(v, wdtype(prec))
    ja, F = s.jvp(xd, vd, mode="ad", want_F=True)
    jf = s.jvp(xd, vd, mode="fd", eps_rule="paper")
    eps = np.sqrt(EPS_MACH[prec]) * max(1.0, np.linalg.norm(host(xd)))
    u = EPS_MACH[prec] / 2
    S = max(1.0, np.abs(host(F)).max(), np.abs(x).max())
    # affine residual: no truncation term, only rounding amplified by 1 / eps
    assert np.abs(host(jf) - host(ja)).max() <= 64 * u * S / eps


def test_newton_suolson_fd_reaches_the_ad_iterate():
    spec, xp, src = case("suolson", 64, 64)
    s = solver(spec, "f64", xp, src)
    xa, ia = s.newton_solve(dev(xp, wdtype("f64")), mode="ad", tol_krylov=1e-10)
    xf, if_ = s.newton_solve(dev(xp, wdtype("f64")), mode="fd", tol_krylov=1e-10)
    assert ia["converged"] and if_["converged"]
    assert np.linalg.norm(host(xf) - host(xa)) <= 1e-8 * np.linalg.norm(host(xa))


# The classic 1D-profile configuration: rows periodic, the first and last
# columns Dirichlet nodes, cold start with the central box source.


@pytest.mark.parametrize("krylov,orth", [("gmres", "dcgs2"), ("gmres", "cgs2"), ("bicgstab", "cgs2")])
@pytest.mark.parametrize("nx,ny,prec,tol", [(64, 64, "f64", 1e-12), (130, 37, "f64", 1e-12), (64, 64, "f32", 1e-5)])
def test_newton_suolson_periodic_rows(krylov, orth, nx, ny, prec, tol):
    spec, xp, src = case("suolson1d", nx, ny)
    info, ref = compare_newton(spec, xp, src, prec, "ad", tol, krylov=krylov, orth=orth, krylov_slack=0.1)
    assert info["converged"] and info["newton_iters"] == 1


@pytest.mark.parametrize("engine", ["multi", "single"])
def test_newton_suolson_periodic_rows_engines(engine):
    spec, xp, src = case("suolson1d", 12, 10)
    compare_newton(spec, xp, src, "f64", "ad", 1e-12, engine=engine)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_suolson_1d_profile_full_size(prec, tol):
    """512^2 from the cold start: one Newton step per iterate against the oracle, and every row
    of the result the same 1D profile (to rounding: each row sums in the same order)."""
    spec, xp, src = W.config("suolson1d")
    info, ref = compare_newton(spec, xp, src, prec, "ad", tol, krylov_slack=0.1, orth="dcgs2")
    assert info["converged"]
    x = host(info["history"])[-1]
    n = spec["nx"] * spec["ny"]
    U = x[:n].reshape(spec["ny"], spec["nx"])
    assert np.max(np.abs(U - U[0])) <= (1e-12 if prec == "f64" else 1e-5) * np.abs(U).max()
    assert U[0, spec["nx"] // 2] > 0 and U[0, 0] == 0.0
