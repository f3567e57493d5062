"""GPU parity of the CSLP-preconditioned GMRES of the Maxwell-Kerr problem
(Appendix A.4) against the oracle's right-preconditioned GMRES.

Parity contract:
  * GMRES with the preconditioner on a field with |E| > 0 (so M varies from
    node to node) on a non-square grid (hx != hy), a fixed number of Arnoldi
    steps (tolerance out of reach): dx = M^{-1} V y within 1e-9 (FP64 AD,
    both Gram-Schmidt forms, one and several cycles), 1e-3 (FP64 FD, the
    paper's step: rounding-bound on this operator, see the test), 2e-4 (FP32
    AD, oracle in FP64 on the FP32-rounded inputs) of the oracle's; the GPU's true residual norm equals the oracle's;
  * the same at the full 512^2 grid in FP32 (the JVP-row shape);
  * Newton from E = 0 with the preconditioner, per iterate, at FACTOR times
    the oracle's own summation-order spread on the same case (order_spread);
  * the configurations the library rejects, and AUTO running the
    multi-kernel engine for a problem the single-workgroup engine would take.

The same for the preconditioner's scalar form on the Helmholtz-Kerr workload
(M = 2/hx^2 + 2/hy^2 - k0^2 eps(E)(1 - 0.5 i), interleaved (Re, Im) storage):
GMRES on a lossy non-square-cell grid with |E| > 0 (FP64 AD 1e-9 with both
Gram-Schmidt forms, FP32 AD 1e-5 including the 1024^2 workload, FP64 FD under
the paper's step at ten times the oracle's own one-ulp sensitivity), odd and
tiny grids, and Newton per iterate on 12 x 10 and on the workload's physics
at 64 x 64 at FACTOR times the oracle's summation-order spread.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import dev, gpu_available, host, wdtype
from oracle import EPS_MACH, Problem, cslp_solve, fd_step, gmres_solve, jvp_ad, jvp_fd, residual
from test_gpu_solver import compare_newton, solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def linear_case(nx, ny, prec, omega=3.0, seed=5, amp=0.3):
    spec = W.maxwell_spec(nx, omega=omega, ny=ny)
    src = W.maxwell_source(nx, omega=omega, ny=ny)
    p = Problem.from_spec(spec)
    x = amp * W.random_vector(p.n, seed)
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    rhs = -residual(p, xw, None, src)
    if prec == "f32":
        rhs = rhs.astype(np.float32).astype(np.float64)
    return spec, src, p, xw, rhs


def oracle_gmres(p, xw, rhs, src, m, cycles, mode="ad", orth="cgs2"):
    if mode == "ad":
        mv = lambda v: jvp_ad(p, xw, v, None, src)[1]  # noqa: E731
    else:
        F0 = residual(p, xw, None, src)
        eps = fd_step("paper", EPS_MACH["f64"], xw, None)
        mv = lambda v: jvp_fd(p, xw, v, eps, None, src, Fx=F0)  # noqa: E731
    z, info = gmres_solve(lambda v: mv(cslp_solve(p, xw, v)), rhs, m=m, tol=1e-30, max_restarts=cycles, orth=orth)
    return cslp_solve(p, xw, z), info, mv


def run_gpu(spec, src, prec, xw, rhs, m, cycles, mode="ad", orth="dcgs2"):
    s = solver(spec, prec, None, src, m=m)
    s.set_orthogonalization(orth)
    s.set_preconditioner("cslp")
    return s.gmres(dev(xw, wdtype(prec)), dev(rhs, wdtype(prec)), m=m, tol=1e-30, max_restarts=cycles, mode=mode)


@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
@pytest.mark.parametrize("m,cycles", [(8, 1), (6, 3)])
def test_cslp_gmres_f64_ad(orth, m, cycles):
    spec, src, p, xw, rhs = linear_case(40, 36, "f64")
    ref, rinfo, mv = oracle_gmres(p, xw, rhs, src, m, cycles, orth=orth)
    dx, info = run_gpu(spec, src, "f64", xw, rhs, m, cycles, orth=orth)
    assert info["krylov_iters"] == rinfo.iters == m * cycles and not info["converged"]
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 1e-9 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)
    # the update is in the original space: its residual is the one GMRES reports
    true_res = np.linalg.norm(rhs - mv(d))
    assert abs(true_res - np.linalg.norm(rhs - mv(ref))) <= 1e-8 * np.linalg.norm(rhs)
    # the preconditioner did something: unpreconditioned GMRES gives another iterate
    plain, _ = gmres_solve(mv, rhs, m=m, tol=1e-30, max_restarts=cycles)
    assert np.linalg.norm(plain - ref) > 1e-3 * np.linalg.norm(ref)


def test_cslp_gmres_f64_fd_paper_step():
    # FD in FP64 on this operator is rounding-bound: F(x + eps v) - F(x) cancels
    # about eight digits, and a one-ulp change of F(x) alone moves the oracle's
    # own 16-step iterate by 1.1e-4 (measured), about as far as AD is from FD.
    # The bound is ten times that; a JVP that skipped the preconditioner would
    # be off by O(1), as the unpreconditioned iterate shows.
    spec, src, p, xw, rhs = linear_case(40, 36, "f64")
    ref, rinfo, mv = oracle_gmres(p, xw, rhs, src, 8, 2, mode="fd")
    dx, info = run_gpu(spec, src, "f64", xw, rhs, 8, 2, mode="fd")
    assert info["krylov_iters"] == rinfo.iters == 16
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 1e-3 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)
    plain, _ = gmres_solve(mv, rhs, m=8, tol=1e-30, max_restarts=2)
    assert np.linalg.norm(plain - ref) > 1e-2 * np.linalg.norm(ref)


@pytest.mark.parametrize("nx,ny", [(40, 36), (512, 512)])
def test_cslp_gmres_f32_ad(nx, ny):
    spec, src, p, xw, rhs = linear_case(nx, ny, "f32")
    ref, rinfo, _ = oracle_gmres(p, xw, rhs, src, 8, 1, orth="dcgs2")
    dx, info = run_gpu(spec, src, "f32", xw, rhs, 8, 1)
    assert info["krylov_iters"] == rinfo.iters == 8
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 2e-4 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("nx,ny,prec,m,tol", [(512, 512, "f64", 8, 1e-9), (37, 29, "f32", 8, 2e-4),
                                              (37, 29, "f64", 8, 1e-9), (3, 3, "f64", 4, 1e-12),
                                              (4, 3, "f32", 4, 1e-5)])
def test_cslp_gmres_sizes(nx, ny, prec, m, tol):
    """Full size in FP64; an odd width (the scalar, one-column-per-thread path, whose halo words
    cross every wavefront edge); the smallest grids (one or two interior nodes)."""
    spec, src, p, xw, rhs = linear_case(nx, ny, prec)
    ref, rinfo, _ = oracle_gmres(p, xw, rhs, src, m, 1)
    dx, info = run_gpu(spec, src, prec, xw, rhs, m, 1, orth="dcgs2" if nx > 4 else "cgs2")
    assert info["krylov_iters"] == rinfo.iters, (info["krylov_iters"], rinfo.iters)
    d = host(dx)
    assert np.linalg.norm(d - ref) <= tol * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)


def test_cslp_gmres_f16_storage():
    spec, src, p, xw, rhs = linear_case(40, 36, "f32")
    ref, rinfo, _ = oracle_gmres(p, xw, rhs, src, 8, 1)
    dx, info = run_gpu(spec, src, "f16s", xw, rhs, 8, 1, orth="cgs2")
    assert info["krylov_iters"] == 8
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 1e-2 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
def test_newton_maxwell_cslp_from_born(orth):
    # bounds: FACTOR times the oracle's own summation-order spread on this case
    # (order_spread "maxwell16_cslp"); the tiny-grid cases at the contract bound
    # run in test_gpu_maxwell
    import order_spread as OS

    spec, xp, src, opts, _, _, _ = OS.case("maxwell16_cslp")
    tol, tol_x = OS.gpu_bounds("maxwell16_cslp")
    info, ref = compare_newton(spec, xp, src, "f64", "ad", tol, tol_x=tol_x, orth=orth, krylov_slack=0.1, **opts)
    assert info["converged"]


def test_newton_maxwell_cslp_auto_engine_runs_multi_kernel():
    # bounds: FACTOR times the oracle's summation-order spread (order_spread "maxwell12x10_cslp")
    import order_spread as OS

    spec, xp, src, opts, _, _, _ = OS.case("maxwell12x10_cslp")
    tol, tol_x = OS.gpu_bounds("maxwell12x10_cslp")
    info, ref = compare_newton(spec, xp, src, "f64", "ad", tol, tol_x=tol_x, engine="auto", orth="dcgs2",
                               krylov_slack=0.1, **opts)
    assert info["converged"]


def kerr_case(nx, ny, prec, chi=0.3, eps_im=-0.05, cpw=16.0, seed=9, amp=0.4):
    """Helmholtz-Kerr, hx != hy, lossy eps_L, a seeded source zero on the boundary and a state
    with |E| > 0, so that M varies from node to node."""
    spec = dict(kind="kerr", nx=nx, ny=ny, hx=1.0, hy=0.8, dt=0.0, theta=1.0, k0=2 * np.pi / cpw, eps_re=1.0,
                eps_im=eps_im, chi3=chi)
    p = Problem.from_spec(spec)
    src = 0.5 * W.random_vector(p.n, seed + 1)
    src.reshape(ny, nx, 2)[[0, -1], :, :] = 0.0
    src.reshape(ny, nx, 2)[:, [0, -1], :] = 0.0
    x = amp * W.random_vector(p.n, seed)
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    rhs = -residual(p, xw, None, src)
    if prec == "f32":
        rhs = rhs.astype(np.float32).astype(np.float64)
    return spec, src, p, xw, rhs


@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
@pytest.mark.parametrize("m,cycles", [(8, 1), (6, 3)])
def test_kerr_cslp_gmres_f64_ad(orth, m, cycles):
    spec, src, p, xw, rhs = kerr_case(40, 36, "f64")
    ref, rinfo, mv = oracle_gmres(p, xw, rhs, src, m, cycles, orth=orth)
    dx, info = run_gpu(spec, src, "f64", xw, rhs, m, cycles, orth=orth)
    assert info["krylov_iters"] == rinfo.iters == m * cycles and not info["converged"]
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 1e-9 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)
    true_res = np.linalg.norm(rhs - mv(d))
    assert abs(true_res - np.linalg.norm(rhs - mv(ref))) <= 1e-8 * np.linalg.norm(rhs)
    plain, _ = gmres_solve(mv, rhs, m=m, tol=1e-30, max_restarts=cycles)
    assert np.linalg.norm(plain - ref) > 1e-3 * np.linalg.norm(ref)


def test_kerr_cslp_gmres_f64_fd_paper_step():
    # the oracle's own 16-step FD iterate moves by 5.9e-7 when F(x) changes by one ulp
    # (measured); the bound is ten times that, the unpreconditioned iterate is 3.7e-2 away
    spec, src, p, xw, rhs = kerr_case(40, 36, "f64")
    ref, rinfo, mv = oracle_gmres(p, xw, rhs, src, 8, 2, mode="fd")
    dx, info = run_gpu(spec, src, "f64", xw, rhs, 8, 2, mode="fd")
    assert info["krylov_iters"] == rinfo.iters == 16
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 6e-6 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)
    plain, _ = gmres_solve(mv, rhs, m=8, tol=1e-30, max_restarts=2)
    assert np.linalg.norm(plain - ref) > 1e-2 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,chi,cpw", [(40, 0.3, 16.0), (1024, 0.1, 64.0)])
def test_kerr_cslp_gmres_f32_ad(n, chi, cpw):
    """FP32 at the contract bound, on a small grid and on the Helmholtz-Kerr workload's own
    shape and physics (1024^2, k0 = 2 pi / 64, eps_L = 1, chi3 = 0.1), one GMRES(30) cycle."""
    eps_im = -0.05 if n == 40 else 0.0
    spec, src, p, xw, rhs = kerr_case(n, n - 4 if n == 40 else n, "f32", chi=chi, eps_im=eps_im, cpw=cpw)
    m = 8 if n == 40 else 30
    ref, rinfo, _ = oracle_gmres(p, xw, rhs, src, m, 1, orth="dcgs2")
    dx, info = run_gpu(spec, src, "f32", xw, rhs, m, 1)
    assert info["krylov_iters"] == rinfo.iters == m
    d = host(dx)
    assert np.linalg.norm(d - ref) <= 1e-5 * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("nx,ny,prec,m,tol", [(37, 29, "f64", 8, 1e-9), (37, 29, "f32", 8, 1e-5),
                                              (3, 3, "f64", 2, 1e-12), (4, 3, "f32", 4, 1e-5)])
def test_kerr_cslp_gmres_sizes(nx, ny, prec, m, tol):
    """An odd width (the one-column-per-thread path); the smallest grids (one or two interior
    nodes: 2 and 4 real interior unknowns)."""
    spec, src, p, xw, rhs = kerr_case(nx, ny, prec)
    ref, rinfo, _ = oracle_gmres(p, xw, rhs, src, m, 1)
    dx, info = run_gpu(spec, src, prec, xw, rhs, m, 1, orth="dcgs2" if nx > 4 else "cgs2")
    assert info["krylov_iters"] == rinfo.iters, (info["krylov_iters"], rinfo.iters)
    d = host(dx)
    assert np.linalg.norm(d - ref) <= tol * np.linalg.norm(ref), np.linalg.norm(d - ref) / np.linalg.norm(ref)


@pytest.mark.parametrize("name,slack", [("kerr12x10_cpw32_chi1.0_cslp", 0.3), ("kerr64_chi0.1_cslp", 0.15)])
@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
def test_newton_kerr_cslp(name, slack, orth):
    """Newton from E = 0 with the preconditioner, per iterate, at FACTOR times the oracle's
    own summation-order spread (order_spread); 64 x 64 is the Helmholtz-Kerr workload's
    physics (k0 = 2 pi / 64 cells, eps_L = 1, chi3 = 0.1)."""
    import order_spread as OS

    spec, xp, src, opts, _, _, _ = OS.case(name)
    tol, tol_x = OS.gpu_bounds(name)
    info, ref = compare_newton(spec, xp, src, "f64", "ad", tol, tol_x=tol_x, orth=orth, krylov_slack=slack,
                               **opts)
    assert info["converged"] and ref.converged


def test_cslp_rejected_configurations():
    from paper_2605_13378_amd import JfnkError

    spec, xp, src = W.config("grayscott", n=32)
    gs = solver(spec, "f64", xp, src, m=8)
    with pytest.raises(JfnkError, match="Maxwell"):
        gs.set_preconditioner("cslp")
    with pytest.raises(JfnkError, match="Maxwell"):
        gs.newton_solve(dev(xp, wdtype("f64")), precond="cslp", m=8)
    mspec = W.maxwell_spec(16)
    msrc = W.maxwell_source(16)
    s = solver(mspec, "f64", None, msrc, m=8)
    x0 = dev(np.zeros(4 * 16 * 16), wdtype("f64"))
    with pytest.raises(JfnkError, match="GMRES on the multi-kernel engine"):
        s.newton_solve(x0, precond="cslp", krylov="bicgstab", m=8)
    with pytest.raises(JfnkError, match="GMRES on the multi-kernel engine"):
        s.newton_solve(x0, precond="cslp", engine="single", m=8)
    with pytest.raises(JfnkError, match="paper's FD step rule"):
        s.newton_solve(x0, precond="cslp", mode="fd", eps_rule="normalized", m=8)
    s.set_preconditioner("cslp")
    with pytest.raises(JfnkError, match="paper's FD step rule"):
        s.gmres(x0, dev(np.ones(4 * 16 * 16), wdtype("f64")), mode="fd", eps_rule="normalized")
    # back to none: the normalized rule is accepted again
    s.set_preconditioner("none")
    s.gmres(x0, dev(np.ones(4 * 16 * 16), wdtype("f64")), mode="fd", eps_rule="normalized", max_restarts=1)
