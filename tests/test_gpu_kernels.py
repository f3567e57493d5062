"""GPU parity of the residual and JVP kernels against the oracle (element by element).

Sizes span several tiles with ragged tails (nx not a multiple of the vector
width or of the block width, ny not a multiple of the rows per block), the
smallest grids (3 x 3), misaligned pointers (scalar path) and the full
workload sizes.  Tolerances:
  * FP64 residual / AD JVP: 1e-13 relative to max(1, |ref|, |x|) (rounding
    of a few dozen operations);
  * FP32 residual / AD JVP: 1e-5 (the FP32 parity bound);
  * FD JVP: the difference of two residual evaluations divided by eps
    amplifies rounding by 1/eps, so the bound is 32 u S / eps with u the unit
    roundoff of the working precision and S = max(1, |F|, |x|).
"""

import math

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, elem_err, gpu_available, host, local_scale, rel_err, wdtype
from oracle import EPS_MACH, Problem, fd_step, jvp_ad, jvp_fd, residual

pytestmark = pytest.mark.gpu

SIZES = {
    "burgers1d": [(256, None), (1000, None), (3, None), (4097, None)],
    "grayscott": [(64, 64), (130, 37), (3, 3), (1024, 12)],
    "burgers2d": [(48, 40), (33, 17), (256, 9)],
    "kerr": [(40, 24), (17, 9), (3, 3), (130, 11)],
    "rd2d": [(64, 64), (130, 37), (3, 3), (1024, 12)],
    "suolson": [(64, 64), (130, 37), (3, 3), (40, 1030)],
    "suolson1d": [(64, 64), (130, 37), (3, 3), (40, 1030)],
    "maxwell": [(64, 64), (130, 37), (3, 3), (40, 1030)],
}
CASES = [(k, nx, ny) for k, sizes in SIZES.items() for nx, ny in sizes]
TOL = {"f64": 1e-13, "f32": 1e-5}


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def make_solver(spec, prec, xp, src, m=30):
    from paper_2605_13378_amd import Solver

    s = Solver(spec, prec, m=m)
    s.set_previous(None if xp is None else dev(xp, wdtype("f64")), None if src is None else dev(src, wdtype("f64")))
    return s


def state_and_direction(spec, xp, seed):
    n = W.n_unknowns(spec)
    x = xp + 0.1 * W.random_vector(n, seed)
    v = W.random_vector(n, seed + 1)
    return x, v


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,nx,ny", CASES)
def test_residual_parity(kind, nx, ny, prec):
    spec, xp, src = case(kind, nx, ny)
    p = Problem.from_spec(spec)
    x, _ = state_and_direction(spec, xp, 11)
    ref = residual(p, x, xp, src)
    s = make_solver(spec, prec, xp, src)
    got = host(s.residual(dev(x, wdtype(prec))))
    assert rel_err(got, ref, x) <= TOL[prec]
    assert elem_err(got, ref, local_scale(spec, *[a for a in (ref, x, xp, src) if a is not None])) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,nx,ny", CASES)
def test_ad_jvp_parity(kind, nx, ny, prec):
    spec, xp, src = case(kind, nx, ny)
    p = Problem.from_spec(spec)
    x, v = state_and_direction(spec, xp, 21)
    Fref, Jref = jvp_ad(p, x, v, xp, src)
    s = make_solver(spec, prec, xp, src)
    jv, F = s.jvp(dev(x, wdtype(prec)), dev(v, wdtype(prec)), mode="ad", want_F=True)
    assert rel_err(host(jv), Jref, v) <= TOL[prec]
    assert rel_err(host(F), Fref, x) <= TOL[prec]
    assert elem_err(host(jv), Jref, local_scale(spec, Jref, v)) <= TOL[prec]
    assert elem_err(host(F), Fref, local_scale(spec, *[a for a in (Fref, x, xp, src) if a is not None])) <= TOL[prec]
    jv_only = s.jvp(dev(x, wdtype(prec)), dev(v, wdtype(prec)), mode="ad")
    assert np.array_equal(host(jv_only), host(jv))


@pytest.mark.parametrize("rule", ["paper", "normalized"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("kind,nx,ny", [c for c in CASES if c[1] >= 17])
def test_fd_jvp_parity(kind, nx, ny, prec, rule):
    spec, xp, src = case(kind, nx, ny)
    p = Problem.from_spec(spec)
    x, v = state_and_direction(spec, xp, 31)
    em = EPS_MACH[prec]
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    vw = v if prec == "f64" else v.astype(np.float32).astype(np.float64)
    eps = fd_step(rule, em, xw, vw)
    ref = jvp_fd(p, xw, vw, eps, xp, src)
    s = make_solver(spec, prec, xp, src)
    got = host(s.jvp(dev(x, wdtype(prec)), dev(v, wdtype(prec)), mode="fd", eps_rule=rule))
    S = max(1.0, float(np.abs(residual(p, xw, xp, src)).max()), float(np.abs(xw).max()))
    u = em / 2
    bound = 32 * u * S / eps * max(1.0, float(np.abs(vw).max()))
    assert float(np.abs(got - ref).max()) <= bound + TOL[prec] * max(1.0, float(np.abs(ref).max()))


def fp16_stored(v, n):
    """The tangent as an FP16S solver stores it: v (FP32) times the power of two sigma that
    maps a typical entry ||v|| / sqrt(n) near 1, rounded to FP16 (nearest even), divided by
    sigma again (exact).  Computed here from that rule, independently of the kernels."""
    v32 = np.asarray(v, dtype=np.float32)
    nrm = float(np.sqrt(np.sum(v32.astype(np.float64) ** 2)))
    sig = 2.0 ** (-np.rint(np.log2(nrm / np.sqrt(n))))
    return (v32 * np.float32(sig)).astype(np.float16).astype(np.float64) / sig


@pytest.mark.parametrize("mode", ["ad", "fd"])
@pytest.mark.parametrize("kind,nx,ny", [("grayscott", 130, 37), ("burgers2d", 48, 40), ("kerr", 40, 24),
                                        ("burgers1d", 1000, None), ("maxwell", 64, 64), ("grayscott", 1024, 1024)])
def test_f16s_jvp_parity(kind, nx, ny, mode):
    """FP16-storage JVP (the tangent stored in FP16 with a power-of-two scale, FP32 arithmetic)
    element by element against the oracle fed the same FP16-rounded tangent and FP32 state:
    the FP32 bound for AD, the FD rounding bound for FD."""
    spec, xp, src = case(kind, nx, ny) if nx < 1024 else W.config("grayscott")
    p = Problem.from_spec(spec)
    x, v = state_and_direction(spec, xp, 23)
    x32 = x.astype(np.float32).astype(np.float64)
    v16 = fp16_stored(v, p.n)
    s = make_solver(spec, "f16s", xp, src)
    if mode == "ad":
        Fref, Jref = jvp_ad(p, x32, v16, xp, src)
        jv, F = s.jvp(dev(x, wdtype("f32")), dev(v, wdtype("f32")), mode="ad", want_F=True)
        assert rel_err(host(jv), Jref, v16) <= TOL["f32"]
        assert elem_err(host(jv), Jref, local_scale(spec, Jref, v16)) <= TOL["f32"]
        assert rel_err(host(F), Fref, x32) <= TOL["f32"]
    else:
        em = EPS_MACH["f32"]
        eps = fd_step("paper", em, x32, v16)
        ref = jvp_fd(p, x32, v16, eps, xp, src)
        got = host(s.jvp(dev(x, wdtype("f32")), dev(v, wdtype("f32")), mode="fd", eps_rule="paper"))
        S = max(1.0, float(np.abs(residual(p, x32, xp, src)).max()), float(np.abs(x32).max()))
        bound = 32 * (em / 2) * S / eps * max(1.0, float(np.abs(v16).max()))
        assert float(np.abs(got - ref).max()) <= bound + TOL["f32"] * max(1.0, float(np.abs(ref).max()))
    # the FP16 rounding is really applied: the FP32 tangent's product differs beyond the bound
    if mode == "ad" and kind == "grayscott" and nx < 1024:
        J32 = jvp_ad(p, x32, v.astype(np.float32).astype(np.float64), xp, src)[1]
        assert rel_err(J32, Jref, v16) > 10 * TOL["f32"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fixed_eps_fd(prec):
    spec, xp, src = case("grayscott", 64, 40)
    p = Problem.from_spec(spec)
    x, v = state_and_direction(spec, xp, 41)
    xw = x if prec == "f64" else x.astype(np.float32).astype(np.float64)
    vw = v if prec == "f64" else v.astype(np.float32).astype(np.float64)
    eps = 1e-2
    ref = jvp_fd(p, xw, vw, eps, xp, src)
    s = make_solver(spec, prec, xp, src)
    got = host(s.jvp(dev(x, wdtype(prec)), dev(v, wdtype(prec)), mode="fd", eps=eps))
    u = EPS_MACH[prec] / 2
    assert float(np.abs(got - ref).max()) <= 32 * u * 4 / eps + TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_misaligned_pointers_take_the_scalar_path(prec):
    torch = pytest.importorskip("torch")
    spec, xp, src = case("grayscott", 64, 48)
    p = Problem.from_spec(spec)
    x, v = state_and_direction(spec, xp, 51)
    n = p.n
    s = make_solver(spec, prec, xp, src)
    big_x = torch.zeros(n + 1, dtype=wdtype(prec), device="cuda")
    big_x[1:] = dev(x, wdtype(prec))
    big_v = torch.zeros(n + 1, dtype=wdtype(prec), device="cuda")
    big_v[1:] = dev(v, wdtype(prec))
    jv_mis = host(s.jvp(big_x[1:], big_v[1:], mode="ad"))
    jv_al = host(s.jvp(dev(x, wdtype(prec)), dev(v, wdtype(prec)), mode="ad"))
    ref = jvp_ad(p, x, v, xp, src)[1]
    assert rel_err(jv_mis, ref, v) <= TOL[prec]
    assert rel_err(jv_al, ref, v) <= TOL[prec]


@pytest.mark.parametrize("kind,n,prec", [("grayscott", 1024, "f64"), ("grayscott", 1024, "f32"),
                                         ("burgers2d", 2048, "f32"), ("kerr", 1024, "f64"), ("rd2d", 512, "f64"),
                                         ("rd2d", 512, "f32"), ("suolson", 512, "f64"), ("suolson", 512, "f32"),
                                         ("suolson1d", 512, "f64"), ("suolson1d", 512, "f32"),
                                         ("maxwell", 512, "f64"), ("maxwell", 512, "f32")])
def test_full_size_jvp_and_residual(kind, n, prec):
    spec, xp, src = W.config(kind, n=n)
    p = Problem.from_spec(spec)
    x = xp + 0.01 * W.random_vector(p.n, 61)
    v = W.random_vector(p.n, 62)
    s = make_solver(spec, prec, xp, src)
    Fref, Jref = jvp_ad(p, x, v, xp, src)
    jv, F = s.jvp(dev(x, wdtype(prec)), dev(v, wdtype(prec)), mode="ad", want_F=True)
    assert rel_err(host(jv), Jref, v) <= TOL[prec]
    assert rel_err(host(F), Fref, x) <= TOL[prec]
    assert elem_err(host(jv), Jref, local_scale(spec, Jref, v)) <= TOL[prec]
    assert elem_err(host(F), Fref, local_scale(spec, *[a for a in (Fref, x, xp, src) if a is not None])) <= TOL[prec]
    assert rel_err(host(s.residual(dev(x, wdtype(prec)))), Fref, x) <= TOL[prec]


def test_jvp_is_deterministic():
    spec, xp, src = case("burgers2d", 256, 96)
    x, v = state_and_direction(spec, xp, 71)
    s = make_solver(spec, "f32", xp, src)
    a = host(s.jvp(dev(x, wdtype("f32")), dev(v, wdtype("f32")), mode="ad"))
    b = host(s.jvp(dev(x, wdtype("f32")), dev(v, wdtype("f32")), mode="ad"))
    assert np.array_equal(a, b)
    assert math.isfinite(float(np.abs(a).max()))
