"""GPU parity of GMRES with the delayed second Gram-Schmidt pass (DCGS2).

The GPU's DCGS2 runs against the oracle's DCGS2 (same algorithm) and against
the oracle's CGS2 (same Krylov iterates in exact arithmetic).  Parity
contract as for CGS2: FP64 AD solutions within 1e-10 and Newton iterates
within 1e-12 (1e-10 on Kerr), FP32 within 1e-5, counts within one per solve
(a tolerance tie can move one step), FD within 1e-7; plus the cycle-end cases
(m = 1, a cap ending mid-cycle, zero and non-finite input), the engine rule,
the Gray-Scott 1024^2 workload per iterate, and the FP16-stored basis of
either form against the oracle with the same binary16 store.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, gpu_available, host, wdtype
from oracle import Problem, gmres_solve, jvp_ad, residual
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


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,nx,ny,m", [("grayscott", 64, 40, 20), ("grayscott", 130, 37, 30),
                                          ("burgers2d", 48, 40, 8), ("burgers1d", 300, None, 30)])
def test_gmres_dcgs2_parity(kind, nx, ny, m, prec):
    spec, xp, src, p, xw, rhs = linear_case(kind, nx, ny, prec)
    ktol = 1e-10 if prec == "f64" else 1e-6
    mv = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    ref_d, rd = gmres_solve(mv, rhs, m=m, tol=ktol, max_restarts=50, orth="dcgs2")
    ref_c, rc = gmres_solve(mv, rhs, m=m, tol=ktol, max_restarts=50)
    s = solver(spec, prec, xp, src, m=m)
    s.set_orthogonalization("dcgs2")
    dx, info = s.gmres(dev(xw, wdtype(prec)), dev(rhs, wdtype(prec)), m=m, tol=ktol, max_restarts=50)
    assert info["converged"] and rd.converged and rc.converged
    bound = 1e-10 if prec == "f64" else 1e-5
    for ref in (ref_d, ref_c):
        assert np.linalg.norm(host(dx) - ref) <= bound * np.linalg.norm(ref)
    assert abs(info["krylov_iters"] - rd.iters) <= 1
    s.set_orthogonalization("cgs2")
    dx2, info2 = s.gmres(dev(xw, wdtype(prec)), dev(rhs, wdtype(prec)), m=m, tol=ktol, max_restarts=50)
    assert np.linalg.norm(host(dx2) - ref_c) <= bound * np.linalg.norm(ref_c)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
def test_gmres_hessenberg_matches_oracle(orth, prec):
    """The unrotated Hessenberg matrix the GPU builds over one full cycle, entry
    by entry, against the oracle's (either Gram-Schmidt form; the two agree in
    exact arithmetic) on a grid that spreads every kernel over many blocks.
    In the delayed form each column's first projection and its completion are
    separate control-block arrays: a completion that read a column its own
    launch had already completed would add the second-pass sums twice."""
    spec, xp, src, p, xw, rhs = linear_case("grayscott", 256, 192, prec)
    m = 20
    mv = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    s = solver(spec, prec, xp, src, m=m)
    s.set_orthogonalization(orth)
    _, info = s.gmres(dev(xw, wdtype(prec)), dev(rhs, wdtype(prec)), m=m, tol=1e-300, max_restarts=1)
    assert info["krylov_iters"] == m and not info["converged"]
    H = s.gmres_hessenberg()
    assert H.shape == (m + 1, m)
    bound = 1e-12 if prec == "f64" else 1e-5
    for form in ("dcgs2", "cgs2"):
        _, ri = gmres_solve(mv, rhs, m=m, tol=1e-300, max_restarts=1, orth=form, record=True)
        Hr = ri.last_H
        assert Hr.shape == H.shape
        scale = float(np.abs(Hr).max())
        assert float(np.abs(H - Hr).max()) <= bound * scale, (form, float(np.abs(H - Hr).max()) / scale)
        assert np.all(np.tril(H, -2) == 0.0)


def test_gmres_dcgs2_cycle_ends():
    spec, xp, src, p, xw, rhs = linear_case("grayscott", 32, 32, "f64")
    mv = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    s = solver(spec, "f64", xp, src, m=6)
    s.set_orthogonalization("dcgs2")
    # m = 1: every column is completed by the V y kernel of its own cycle
    for m, cycles in ((1, 3), (6, 2), (5, 1)):
        ref, ri = gmres_solve(mv, rhs, m=m, tol=1e-14, max_restarts=cycles, orth="dcgs2")
        dx, info = s.gmres(dev(xw, wdtype("f64")), dev(rhs, wdtype("f64")), m=m, tol=1e-14, max_restarts=cycles)
        assert not info["converged"] and info["krylov_iters"] == ri.iters == m * cycles
        assert np.linalg.norm(host(dx) - ref) <= 1e-12 * np.linalg.norm(ref)
    dx, info = s.gmres(dev(xw, wdtype("f64")), dev(np.zeros(p.n), wdtype("f64")), tol=1e-8)
    assert info["converged"] and info["krylov_iters"] == 0 and not host(dx).any()
    bad = rhs.copy()
    bad[9] = np.inf
    dx, info = s.gmres(dev(xw, wdtype("f64")), dev(bad, wdtype("f64")), tol=1e-8)
    assert info["status"] == "nonfinite"


def test_dcgs2_rules():
    # the single-workgroup engine keeps CGS2: same result as CGS2 on it
    spec1, xp1, _ = case("burgers1d", 128)
    s1 = solver(spec1, "f64", xp1, None, m=30)
    a, ia = s1.newton_solve(dev(xp1, wdtype("f64")), engine="single", orth="dcgs2")
    b, ib = s1.newton_solve(dev(xp1, wdtype("f64")), engine="single", orth="cgs2")
    assert np.array_equal(host(a), host(b)) and ia["lin_iters"] == ib["lin_iters"]


@pytest.mark.parametrize("kind,nx,ny,prec,tol", [
    ("grayscott", 64, 64, "f64", 1e-12), ("grayscott", 130, 37, "f64", 1e-12), ("burgers2d", 48, 40, "f64", 1e-12),
    ("burgers1d", 256, None, "f64", 1e-12), ("rd2d", 64, 64, "f64", 1e-12),
    ("grayscott", 64, 64, "f32", 1e-5), ("burgers2d", 48, 40, "f32", 1e-5),
])
def test_newton_dcgs2(kind, nx, ny, prec, tol):
    spec, xp, src = case(kind, nx, ny)
    compare_newton(spec, xp, src, prec, "ad", tol, orth="dcgs2")


def test_newton_dcgs2_kerr_f64():
    # bounds from the oracle's own summation-order spread on this case (order_spread)
    import order_spread as OS

    spec, xp, src, opts, _, _, _ = OS.case("kerr12x10_cpw64_chi0.3")
    tol, tol_x = OS.gpu_bounds("kerr12x10_cpw64_chi0.3")
    compare_newton(spec, xp, src, "f64", "ad", tol, tol_x=tol_x, orth="dcgs2", **opts)


@pytest.mark.parametrize("rule", ["paper", "normalized"])
def test_newton_dcgs2_f64_fd(rule):
    spec, xp, src = case("grayscott", 64, 64)
    compare_newton(spec, xp, src, "f64", "fd", 1e-7, eps_rule=rule, orth="dcgs2")


def test_full_size_grayscott_f64_ad_dcgs2():
    """Gray-Scott 1024^2, FP64, AD, GMRES(30) with DCGS2 against the oracle, per Newton iterate."""
    spec, xp, src = W.config("grayscott")
    compare_newton(spec, xp, src, "f64", "ad", 1e-12, orth="dcgs2")


def test_full_size_grayscott_f32_ad_dcgs2():
    """The benchmark configuration itself (FP32, AD, normalized FD rule irrelevant for AD)."""
    spec, xp, src = W.config("grayscott")
    compare_newton(spec, xp, src, "f32", "ad", 1e-5, orth="dcgs2")


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
def test_gmres_hessenberg_f16s_matches_fp16_store_oracle(orth):
    """FP16-stored basis: the unrotated Hessenberg matrix of one full cycle
    against the oracle run with the same store (every basis vector rounded to
    binary16 under a power-of-two scale), and the solution of a capped run.
    The GPU forms each stored vector in FP32 before rounding it, so an
    element within its FP32 error (~ sqrt(20) * 2^-24 relative over 20 terms)
    of a binary16 rounding boundary can round the other way: probability
    p ~ 2 * 2.7e-7 / 2^-10 ~ 5e-4 per element, one binary16 ulp (2^-10)
    each, ~ sqrt(p) 2^-10 ~ 2e-5 relative per vector.  Bounds: 5e-5 on the
    capped solution (the FP64-store oracle is 3e-4 away: the store's own
    effect) and 2e-5 of max |H| on the Hessenberg matrix."""
    spec, xp, src, p, xw, rhs = linear_case("grayscott", 256, 192, "f32")
    m = 20
    mv = lambda v: jvp_ad(p, xw, v, xp, src)[1]  # noqa: E731
    s = solver(spec, "f16s", xp, src, m=m)
    s.set_orthogonalization(orth)
    dx, info = s.gmres(dev(xw, wdtype("f16s")), dev(rhs, wdtype("f16s")), m=m, tol=1e-300, max_restarts=1)
    assert info["krylov_iters"] == m and not info["converged"]
    H = s.gmres_hessenberg()
    xr, ri = gmres_solve(mv, rhs, m=m, tol=1e-300, max_restarts=1, orth=orth, record=True, store="fp16")
    _, r64 = gmres_solve(mv, rhs, m=m, tol=1e-300, max_restarts=1, orth=orth, record=True)
    scale = float(np.abs(ri.last_H).max())
    err = float(np.abs(H - ri.last_H).max()) / scale
    err64 = float(np.abs(H - r64.last_H).max()) / scale
    print(f"f16s {orth}: H vs fp16-store oracle {err:.3e}, vs fp64 oracle {err64:.3e}")
    assert err <= 2e-5, (err, err64)
    xe = float(np.linalg.norm(host(dx) - xr) / np.linalg.norm(xr))
    print(f"f16s {orth}: dx vs fp16-store oracle {xe:.3e}")
    assert xe <= 5e-5, xe
