"""GPU parity of GMRES and Newton against the oracle, per iterate.

Parity contract:
  * FP64 AD: |rho_k(gpu) - rho_k(oracle)| <= 1e-12 and
    ||x_k(gpu) - x_k(oracle)|| / ||x_k(oracle)|| <= 1e-12 at every Newton
    iterate, same number of iterates, Krylov counts equal or +-1 per step
    (a tolerance tie can flip one Arnoldi step);
  * FP32 AD: the same at 1e-5, the oracle run in FP64 with the FP32
    tolerances (the paper's FP32 settings);
  * FD: the FD JVP carries rounding amplified by 1/eps, which differs between
    any two implementations, so FD iterates are compared at 1e-7 (FP64)
    against the oracle's own FD run, and FD and AD must reach the same root.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, gpu_available, host, wdtype
from oracle import EPS_MACH, NewtonOptions, Problem, gmres_solve, jvp_ad, newton_solve, residual

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def solver(spec, prec, xp, src, m=30):
    from paper_2605_13378_amd import Solver

    s = Solver(spec, prec, m=m)
    s.set_previous(None if xp is None else dev(xp, wdtype("f64")), None if src is None else dev(src, wdtype("f64")))
    return s


def compare_newton(spec, xp, src, prec, mode, tol, x0=None, eps_rule="paper", krylov_slack=None, engine="multi",
                   krylov="gmres", orth="cgs2", precond="none", tol_x=None, rho_floor=None, counts=True, **kw):
    """Newton per iterate against the oracle: |rho_k - rho_k^ref| <= tol (+ rho_floor(x_k^ref), a
    working-precision residual floor, when given) and ||x_k - x_k^ref|| <= tol_x ||x_k^ref||
    (tol_x defaults to tol); Krylov counts per Newton step within the slack unless `counts` is
    False."""
    tol_x = tol if tol_x is None else tol_x
    p = Problem.from_spec(spec)
    o = NewtonOptions.for_precision(prec, mode=mode, eps_rule=eps_rule, krylov=krylov, orth=orth, precond=precond,
                                    **kw)
    x_ref, info_ref = newton_solve(p, xp, o, source=src, x0=x0, record=True)
    s = solver(spec, prec, xp, src, m=o.m)
    start = xp if x0 is None else x0
    s.profile_reset()
    s.profile(True)
    x_gpu, info = s.newton_solve(dev(start, wdtype("f64")), history=True, mode=mode, eps_rule=eps_rule,
                                 m=o.m, tol_newton=o.tol_newton, tol_krylov=o.tol_krylov,
                                 max_newton=o.max_newton, max_restarts=o.max_restarts,
                                 breakdown_tol=o.breakdown_tol, engine=engine, krylov=krylov, orth=orth,
                                 precond=precond)
    prof = s.profile_read()
    s.profile(False)
    # the engine asked for is the one that ran
    if engine == "single":
        assert prof["fused_solve"]["launches"] == 1 and prof["residual"]["launches"] == 0, prof
    elif engine == "multi" or precond != "none":  # AUTO takes the multi-kernel engine with a preconditioner
        assert prof["fused_solve"]["launches"] == 0 and prof["residual"]["launches"] >= 1, prof
    hist = host(info["history"])
    refs = [(orth, info_ref)]
    if orth == "dcgs2" and krylov == "gmres":
        # the delayed second pass and plain CGS2 build the same Krylov basis
        # in exact arithmetic: a mistake shared by the GPU kernel and the
        # oracle's DCGS2 form would show against the plain form
        o2 = NewtonOptions.for_precision(prec, mode=mode, eps_rule=eps_rule, krylov=krylov, orth="cgs2",
                                         precond=precond, **kw)
        refs.append(("cgs2", newton_solve(p, xp, o2, source=src, x0=x0, record=True)[1]))
    for form, ref in refs:
        assert info["newton_iters"] == ref.newton_iters, (form, info, ref)
        assert info["converged"] == ref.converged, form
        for k, (r_gpu, r_ref) in enumerate(zip(info["rel_res"], ref.rel_res)):
            xr = ref.iterates[k]
            fl = 0.0 if rho_floor is None else rho_floor(xr, ref.f0_norm)
            assert abs(r_gpu - r_ref) <= tol + fl, (form, k, r_gpu, r_ref, fl)
            assert np.linalg.norm(hist[k] - xr) <= tol_x * np.linalg.norm(xr), (form, k)
        for a, b in zip(info["lin_iters"], ref.lin_iters) if counts else ():
            slack = 1 if (mode == "ad" and prec == "f64") else (2 if mode == "ad" else 1 + b // 10)
            if krylov_slack is not None:
                slack = max(slack, int(krylov_slack * b))
            assert abs(a - b) <= slack, (form, info["lin_iters"], ref.lin_iters)
    assert np.array_equal(host(x_gpu), hist[-1])
    return info, info_ref


@pytest.mark.parametrize("engine", ["multi", "single"])
def test_newton_burgers1d_config_f64_ad(engine):
    spec, xp, _ = W.config("burgers1d")
    compare_newton(spec, xp, None, "f64", "ad", 1e-12, tol_newton=1e-10, tol_krylov=1e-12, engine=engine)


# Single-workgroup engine (the whole solve in one launch, vectors in LDS) on
# problems small enough for it, at the same per-iterate bounds as the
# multi-kernel path.  The last three are the largest 1D sizes whose LDS
# footprint fits one workgroup's 160 KB (n = 480 in FP64, 896 in FP32) and a
# ragged 2D grid, each with more unknowns than the workgroup has threads.
@pytest.mark.parametrize("kind,nx,ny,prec,mode,rule,tol", [
    ("burgers1d", 256, None, "f32", "ad", "paper", 1e-5),
    ("burgers1d", 256, None, "f64", "fd", "paper", 1e-7),
    ("burgers1d", 200, None, "f64", "fd", "normalized", 1e-7),
    ("grayscott", 16, 12, "f64", "ad", "paper", 1e-12),
    ("grayscott", 16, 16, "f32", "ad", "paper", 1e-5),
    ("burgers2d", 12, 10, "f64", "ad", "paper", 1e-12),
    ("burgers2d", 12, 10, "f64", "fd", "paper", 1e-7),
    ("burgers1d", 480, None, "f64", "ad", "paper", 1e-12),
    ("burgers1d", 896, None, "f32", "ad", "paper", 1e-5),
    ("grayscott", 21, 19, "f32", "ad", "paper", 1e-5),
])
def test_newton_single_workgroup(kind, nx, ny, prec, mode, rule, tol):
    if kind == "burgers1d":
        spec, xp, src = W.burgers1d_spec(nx), W.burgers1d_initial(nx, 0), None
    else:
        spec, xp, src = case(kind, nx, ny)
    compare_newton(spec, xp, src, prec, mode, tol, eps_rule=rule, engine="single")


def test_single_workgroup_statuses_and_fallback():
    spec, xp, src = case("grayscott", 16, 12)
    s = solver(spec, "f64", xp, src)
    x_bad = xp.copy()
    x_bad[17] = np.nan
    _, info = s.newton_solve(dev(x_bad, wdtype("f64")), engine="single")
    assert info["status"] == "nonfinite"
    _, info = s.newton_solve(dev(xp, wdtype("f64")), tol_newton=1e-15, max_newton=1, engine="single")
    assert info["status"] == "not_converged" and info["newton_iters"] == 1
    big, xb, _ = case("grayscott", 64, 64)
    sb = solver(big, "f64", xb, None)
    from paper_2605_13378_amd import JfnkError

    with pytest.raises(JfnkError):
        sb.newton_solve(dev(xb, wdtype("f64")), engine="single")  # does not fit in LDS


@pytest.mark.parametrize("kind,nx,ny", [("grayscott", 64, 64), ("grayscott", 130, 37), ("burgers2d", 48, 40),
                                        ("burgers1d", 1000, None)])
def test_newton_f64_ad(kind, nx, ny):
    spec, xp, src = case(kind, nx, ny)
    compare_newton(spec, xp, src, "f64", "ad", 1e-12)


@pytest.mark.parametrize("name", ["tgv", "dsl"])
def test_newton_paper_burgers_cases(name):
    # the paper's periodic Burgers set-ups (Taylor-Green vortex, double shear layer), CFL step
    spec, x0 = W.burgers2d_paper_case(name, 64)
    compare_newton(spec, x0, None, "f64", "ad", 1e-12)


@pytest.mark.parametrize("engine", ["multi", "single"])
@pytest.mark.parametrize("name,slack", [("kerr12x10_cpw64_chi0.3", None), ("kerr12x10_cpw32_chi1.0", 0.15)])
def test_newton_kerr_f64_ad(name, slack, engine):
    # small cases where GMRES(30) converges in ~30 steps.  -Lap - k0^2 eps is indefinite and
    # Newton runs from E = 0, so the iterates depend on the summation order of the dot
    # products: the oracle itself, run on the permuted system, moves by the spread that
    # order_spread records and test_oracle_summation_order pins (x: 2e-12 and 3e-11 here,
    # rho: 1e-15 and 7e-12), and the bounds are FACTOR times those ceilings (rho back at the
    # 1e-12 contract for the first case).  The second case backtracks through nine Newton
    # steps near the restart length, where the spread moves up to 4 Arnoldi steps between
    # cycles; the per-step count slack is 15%.
    import order_spread as OS

    spec, xp, src, opts, _, _, _ = OS.case(name)
    tol, tol_x = OS.gpu_bounds(name)
    compare_newton(spec, xp, src, "f64", "ad", tol, tol_x=tol_x, krylov_slack=slack, engine=engine, **opts)


@pytest.mark.parametrize("kind,nx,ny", [("grayscott", 64, 64), ("burgers2d", 48, 40), ("burgers1d", 256, None)])
def test_newton_f32_ad(kind, nx, ny):
    spec, xp, src = case(kind, nx, ny)
    compare_newton(spec, xp, src, "f32", "ad", 1e-5)


@pytest.mark.parametrize("rule", ["paper", "normalized"])
def test_newton_f64_fd(rule):
    spec, xp, src = case("grayscott", 64, 48)
    compare_newton(spec, xp, src, "f64", "fd", 1e-7, eps_rule=rule)


def test_fd_and_ad_reach_the_same_root_f64():
    spec, xp, src = case("grayscott", 96, 64)
    s = solver(spec, "f64", xp, src)
    xa, ia = s.newton_solve(dev(xp, wdtype("f64")), mode="ad", tol_newton=1e-8, tol_krylov=1e-9)
    xf, if_ = s.newton_solve(dev(xp, wdtype("f64")), mode="fd", tol_newton=1e-8, tol_krylov=1e-9)
    assert ia["converged"] and if_["converged"]
    # ||J^-1|| <= 1 here (J = I + dt (diffusion + reaction)); both residuals < tol * ||F0||
    assert float(np.linalg.norm(host(xa) - host(xf))) <= 2 * 1e-8 * ia["f0_norm"]


@pytest.mark.parametrize("engine", ["multi", "single"])
def test_line_search_sequence_matches(engine):
    spec = W.burgers1d_spec(24, nu=0.05, dt=1.0)
    xp = 1.0 + 2.0 * np.sin(2 * np.pi * np.arange(24) / 24)
    info, ref = compare_newton(spec, xp, None, "f64", "ad", 1e-12, tol_newton=1e-8, tol_krylov=1e-10,
                               max_newton=40, engine=engine)
    assert info["ls_backtracks"] == ref.ls_backtracks > 0
    assert info["alphas"] == ref.alphas


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_gmres_parity_ad(prec):
    spec, xp, src = case("grayscott", 64, 40)
    p = Problem.from_spec(spec)
    x = xp + 0.05 * W.random_vector(p.n, 81)
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    rhs = -residual(p, xw, xp, src)
    rhs_w = rhs if prec == "f64" else rhs.astype(np.float32).astype(np.float64)
    ktol = 1e-10 if prec == "f64" else 1e-6
    ref, rinfo = gmres_solve(lambda v: jvp_ad(p, xw, v, xp, src)[1], rhs_w, m=20, tol=ktol, max_restarts=50)
    s = solver(spec, prec, xp, src, m=20)
    dx, info = s.gmres(dev(xw, wdtype(prec)), dev(rhs_w, wdtype(prec)), m=20, tol=ktol, max_restarts=50)
    assert info["converged"] and rinfo.converged
    err = np.linalg.norm(host(dx) - ref) / np.linalg.norm(ref)
    assert err <= (1e-10 if prec == "f64" else 1e-5), err
    assert abs(info["krylov_iters"] - rinfo.iters) <= 1


@pytest.mark.parametrize("prec,ktol,bound", [("f64", 1e-6, 1e-6), ("f32", 1e-3, 1e-2)])
def test_gmres_parity_fd(prec, ktol, bound):
    # FD JVPs carry rounding amplified by 1/eps: only tolerances above that
    # noise floor are reachable (FP32 FD stalls near 1e-4, the paper's effect)
    from oracle import fd_step, jvp_fd

    spec, xp, src = case("grayscott", 64, 40)
    p = Problem.from_spec(spec)
    x = xp + 0.05 * W.random_vector(p.n, 81)
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    rhs_w = -residual(p, xw, xp, src)
    if prec == "f32":
        rhs_w = rhs_w.astype(np.float32).astype(np.float64)
    F0 = residual(p, xw, xp, src)
    ref, rinfo = gmres_solve(lambda v: jvp_fd(p, xw, v, fd_step("paper", EPS_MACH[prec], xw, v), xp, src, Fx=F0),
                             rhs_w, m=20, tol=ktol, max_restarts=50)
    s = solver(spec, prec, xp, src, m=20)
    dx, info = s.gmres(dev(xw, wdtype(prec)), dev(rhs_w, wdtype(prec)), m=20, tol=ktol, max_restarts=50, mode="fd")
    assert info["converged"] and rinfo.converged
    err = np.linalg.norm(host(dx) - ref) / np.linalg.norm(ref)
    assert err <= bound, err


def test_gmres_restart_cap_and_zero_rhs():
    spec, xp, src = case("grayscott", 32, 32)
    p = Problem.from_spec(spec)
    s = solver(spec, "f64", xp, src, m=4)
    rhs = W.random_vector(p.n, 91)
    dx, info = s.gmres(dev(xp, wdtype("f64")), dev(rhs, wdtype("f64")), m=1, tol=1e-14, max_restarts=1)
    assert not info["converged"] and info["krylov_iters"] == 1 and info["restarts"] == 1
    ref, rinfo = gmres_solve(lambda v: jvp_ad(p, xp, v, xp)[1], rhs, m=1, tol=1e-14, max_restarts=1)
    assert np.linalg.norm(host(dx) - ref) <= 1e-12 * np.linalg.norm(ref)
    dx0, info0 = s.gmres(dev(xp, wdtype("f64")), dev(np.zeros(p.n), wdtype("f64")), tol=1e-8)
    assert info0["converged"] and info0["krylov_iters"] == 0 and not host(dx0).any()
    # the first cycle's start is not read back: its steps leave on the device and are not
    # counted as a cycle run
    assert info0["restarts"] == 0
    # no cycle allowed: no iterations, dx = 0
    dxn, infn = s.gmres(dev(xp, wdtype("f64")), dev(rhs, wdtype("f64")), m=4, tol=1e-14, max_restarts=0)
    assert not infn["converged"] and infn["krylov_iters"] == 0 and infn["restarts"] == 0 and not host(dxn).any()


def test_nonfinite_and_not_converged_statuses():
    spec, xp, src = case("grayscott", 32, 32)
    s = solver(spec, "f64", xp, src)
    x_bad = xp.copy()
    x_bad[17] = np.nan
    _, info = s.newton_solve(dev(x_bad, wdtype("f64")))
    assert info["status"] == "nonfinite"
    _, info = s.newton_solve(dev(xp, wdtype("f64")), tol_newton=1e-15, max_newton=1)
    assert info["status"] == "not_converged" and info["newton_iters"] == 1


def test_newton_is_deterministic():
    spec, xp, src = case("grayscott", 128, 96)
    s = solver(spec, "f32", xp, src)
    a, ia = s.newton_solve(dev(xp, wdtype("f64")))
    b, ib = s.newton_solve(dev(xp, wdtype("f64")))
    assert np.array_equal(host(a), host(b))
    assert ia["rel_res"] == ib["rel_res"] and ia["lin_iters"] == ib["lin_iters"]


def test_full_size_grayscott_f64_ad_per_iterate():
    """The benchmark workload (Gray-Scott 1024^2, FP64, AD, GMRES(30)) against the oracle."""
    spec, xp, src = W.config("grayscott")
    compare_newton(spec, xp, src, "f64", "ad", 1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_full_size_burgers2d_two_steps_f32_ad(seed):
    """2D Burgers 2048^2, Crank-Nicolson, FP32 AD: two implicit steps, every
    Newton iterate of both against the oracle (each side steps from its own
    previous result).

    The FP32 residual cannot fall below its rounding floor: x - b cancels to
    ~5e-4 per component while x and b carry 2^-24 relative rounding, so
    ||F_fp32(x*)|| ~ 2^-24 ||x|| (4e-5 of ||F0|| here, against the oracle's
    FP64 2.8e-6).  The relative-residual bound is 1e-5 plus twice that floor;
    the iterates themselves match at 1e-5."""
    from oracle import NewtonOptions as NO

    spec, xp, _ = W.config("burgers2d", seed=seed)
    p = Problem.from_spec(spec)
    o = NO.for_precision("f32", mode="ad")
    s = solver(spec, "f32", xp, None)
    x_ref_prev, x_gpu_prev = xp, xp
    for step in range(2):
        x_ref, ref = newton_solve(p, x_ref_prev, o, record=True)
        s.set_previous(dev(x_gpu_prev, wdtype("f64")))
        x_gpu, info = s.newton_solve(dev(x_gpu_prev, wdtype("f64")), history=True, mode="ad")
        assert info["converged"] and ref.converged
        assert info["newton_iters"] == ref.newton_iters, (step, info, ref)
        hist = host(info["history"])
        for k, (r_gpu, r_ref) in enumerate(zip(info["rel_res"], ref.rel_res)):
            xr = ref.iterates[k]
            floor = 2 * 2.0 ** -24 * np.linalg.norm(xr) / ref.f0_norm
            assert abs(r_gpu - r_ref) <= 1e-5 + floor, (step, k, r_gpu, r_ref, floor)
            assert np.linalg.norm(hist[k] - xr) <= 1e-5 * np.linalg.norm(xr), (step, k)
        for a, b in zip(info["lin_iters"], ref.lin_iters):
            assert abs(a - b) <= 2
        x_ref_prev, x_gpu_prev = x_ref, host(x_gpu)


def test_full_size_burgers2d_f16s_ad():
    """2048^2 FP16-stored basis: the result meets the Newton tolerance when its
    residual is evaluated by the oracle in FP64, and lies within the
    tolerance-implied distance of the oracle's root."""
    from oracle import NewtonOptions as NO

    spec, xp, _ = W.config("burgers2d", seed=2)
    p = Problem.from_spec(spec)
    o = NO.for_precision("f32", mode="ad")
    x_ref, ref = newton_solve(p, xp, o)
    s = solver(spec, "f16s", xp, None)
    x, info = s.newton_solve(dev(xp, wdtype("f64")), mode="ad")
    assert info["converged"]
    r = np.linalg.norm(residual(p, host(x), xp))
    assert r <= 1.01 * o.tol_newton * ref.f0_norm, (r, ref.f0_norm)
    assert np.linalg.norm(host(x) - x_ref) <= 2 * o.tol_newton * ref.f0_norm + 1e-6 * np.linalg.norm(x_ref)


@pytest.mark.parametrize("kind,nx,ny", [("grayscott", 64, 64), ("burgers2d", 48, 40), ("grayscott", 1024, 1024)])
@pytest.mark.parametrize("mode", ["ad", "fd"])
@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
def test_newton_f16s(kind, nx, ny, mode, orth):
    """FP16-stored basis and tangent, FP32 arithmetic, FP64 Givens/update/merit.

    Not a per-iterate parity case (FP16 storage perturbs every basis vector by
    ~2^-11 relative); the bound is the tolerance-implied one: both solutions
    satisfy ||F(x)|| <= tol_N ||F0|| and ||J^-1|| <= 1 for these diffusive
    implicit steps, so ||x_gpu - x_ref|| <= 2 tol_N ||F0|| (+ FP32 rounding).
    """
    spec, xp, src = case(kind, nx, ny) if nx < 1024 else W.config("grayscott")
    p = Problem.from_spec(spec)
    o = NewtonOptions.for_precision("f32", mode=mode, eps_rule="normalized")
    x_ref, ref = newton_solve(p, xp, o, source=src)
    s = solver(spec, "f16s", xp, src)
    x, info = s.newton_solve(dev(xp, wdtype("f64")), mode=mode, eps_rule="normalized", orth=orth)
    assert info["converged"] and ref.converged, (info, ref)
    assert info["rel_res"][-1] < o.tol_newton
    bound = 2 * o.tol_newton * ref.f0_norm + 1e-6 * np.linalg.norm(x_ref)
    assert np.linalg.norm(host(x) - x_ref) <= bound
    assert abs(info["newton_iters"] - ref.newton_iters) <= 1
