"""Pins of the oracle's AD and FD Jacobian-vector products.

* AD JVP columns J e_i equal the hand-derived analytic Jacobian (tests/analytic.py).
* AD JVP equals the complex-step derivative Im F(x + i t v) / t (Squire and
  Trapp, 1998), exact to rounding for these polynomial residuals.
* FD minus AD equals the closed-form truncation term of each residual
  (Burgers quadratic, Gray-Scott and Kerr cubic), taken with a large eps so
  that truncation dominates rounding.
* FD step rules (paper's step-size equation and the normalized variant).
Cited: paper Section 2 (Gateaux-derivative definition of the JVP, the FD JVP,
the FD step, the AD jvp pair).
"""

import math

import numpy as np
import pytest

import analytic
import workloads as W
from oracle import EPS_NORMALIZED, EPS_PAPER, Problem, fd_step, jvp_ad, jvp_fd, residual


def tiny_cases():
    b1 = W.burgers1d_spec(11, nu=0.02, dt=0.05, theta=1.0)
    b2 = W.burgers2d_spec(5, nu=0.1, dt=0.1, theta=0.5)
    b2["ny"] = 4
    gs = W.grayscott_spec(5, D=2e-3, Dv=1e-3, dt=0.8, h=0.05)
    gs["ny"] = 6
    kr = W.kerr_spec(6, chi3=0.4, eps_re=1.1, eps_im=0.07, cells_per_wavelength=5.0)
    kr["ny"] = 5
    return [b1, b2, gs, kr]


def state(spec, seed):
    n = W.n_unknowns(spec)
    return 0.5 + 0.3 * W.random_vector(n, seed)


@pytest.mark.parametrize("spec", tiny_cases(), ids=lambda s: s["kind"])
def test_ad_columns_equal_analytic_jacobian(spec):
    p = Problem.from_spec(spec)
    x = state(spec, 1)
    xp = state(spec, 2)
    src = W.random_vector(p.n, 3, 0.1) if p.kind == "kerr" else None
    J = analytic.DENSE[p.kind](spec, x)
    cols = np.zeros((p.n, p.n))
    for i in range(p.n):
        e = np.zeros(p.n)
        e[i] = 1.0
        cols[:, i] = jvp_ad(p, x, e, xp, src)[1]
    scale = np.abs(J).max()
    np.testing.assert_allclose(cols, J, rtol=0, atol=1e-15 * scale * 8)


@pytest.mark.parametrize("spec", tiny_cases(), ids=lambda s: s["kind"])
def test_ad_equals_complex_step(spec):
    p = Problem.from_spec(spec)
    x = state(spec, 4)
    xp = state(spec, 5)
    v = W.random_vector(p.n, 6)
    src = W.random_vector(p.n, 7, 0.1) if p.kind == "kerr" else None
    t = 1e-30
    cs = residual(p, x + 1j * t * v, xp, src).imag / t
    Fx, Jv = jvp_ad(p, x, v, xp, src)
    np.testing.assert_allclose(Jv, cs, rtol=1e-13, atol=1e-13 * np.abs(cs).max())
    np.testing.assert_array_equal(Fx, residual(p, x, xp, src))


@pytest.mark.parametrize("spec", tiny_cases(), ids=lambda s: s["kind"])
def test_ad_is_linear_in_direction(spec):
    p = Problem.from_spec(spec)
    x = state(spec, 8)
    xp = state(spec, 9)
    v, w = W.random_vector(p.n, 10), W.random_vector(p.n, 11)
    src = W.random_vector(p.n, 12, 0.1) if p.kind == "kerr" else None
    lhs = jvp_ad(p, x, 2.5 * v - 0.75 * w, xp, src)[1]
    rhs = 2.5 * jvp_ad(p, x, v, xp, src)[1] - 0.75 * jvp_ad(p, x, w, xp, src)[1]
    np.testing.assert_allclose(lhs, rhs, rtol=1e-13, atol=1e-13 * np.abs(rhs).max())


def _shift(a, d, axis):
    """a[i + d] along axis with periodic wrap (explicit index arithmetic)."""
    n = a.shape[axis]
    idx = (np.arange(n) + d) % n
    return np.take(a, idx, axis=axis)


def fd_minus_ad_closed_form(spec, x, v, eps):
    """(F(x + eps v) - F(x))/eps - J v, derived by expanding each residual's nonlinearity."""
    c = spec["theta"] * spec["dt"]
    kind = spec["kind"]
    if kind == "burgers1d":
        h = spec["hx"]
        return eps * c * v * (_shift(v, 1, 0) - _shift(v, -1, 0)) / (2 * h)
    if kind == "burgers2d":
        nx, ny = spec["nx"], spec["ny"]
        W2 = v.reshape(2, ny, nx)
        wu, wv = W2
        out = []
        for q in (wu, wv):
            dxq = (_shift(q, 1, 1) - _shift(q, -1, 1)) / (2 * spec["hx"])
            dyq = (_shift(q, 1, 0) - _shift(q, -1, 0)) / (2 * spec["hy"])
            out.append(eps * c * (wu * dxq + wv * dyq))
        return np.concatenate([o.ravel() for o in out])
    if kind == "grayscott":
        nx, ny = spec["nx"], spec["ny"]
        u, vv = x.reshape(2, ny, nx)
        wu, wv = v.reshape(2, ny, nx)
        t = eps * (vv * wu * wu + 2 * u * wu * wv) + eps * eps * wu * wu * wv
        return np.concatenate([(-c * t).ravel(), (c * t).ravel()])
    if kind == "kerr":
        nx, ny = spec["nx"], spec["ny"]
        E = x.reshape(ny, nx, 2)
        Wv = v.reshape(ny, nx, 2)
        Ec = E[..., 0] + 1j * E[..., 1]
        Wc = Wv[..., 0] + 1j * Wv[..., 1]
        k2, chi = spec["k0"] ** 2, spec["chi3"]
        t = -k2 * chi * (eps * (2 * np.real(np.conj(Ec) * Wc) * Wc + np.abs(Wc) ** 2 * Ec)
                         + eps * eps * np.abs(Wc) ** 2 * Wc)
        t[0, :] = t[-1, :] = 0
        t[:, 0] = t[:, -1] = 0
        out = np.zeros((ny, nx, 2))
        out[..., 0] = t.real
        out[..., 1] = t.imag
        return out.ravel()
    raise KeyError(kind)


@pytest.mark.parametrize("spec", tiny_cases(), ids=lambda s: s["kind"])
def test_fd_minus_ad_truncation_closed_form(spec):
    p = Problem.from_spec(spec)
    x = state(spec, 13)
    xp = state(spec, 14)
    v = W.random_vector(p.n, 15)
    src = W.random_vector(p.n, 16, 0.1) if p.kind == "kerr" else None
    eps = 1e-3
    diff = jvp_fd(p, x, v, eps, xp, src) - jvp_ad(p, x, v, xp, src)[1]
    expect = fd_minus_ad_closed_form(spec, x, v, eps)
    scale = np.abs(residual(p, x, xp, src)).max() + np.abs(x).max()
    # what remains is rounding of order u * |F| / eps
    np.testing.assert_allclose(diff, expect, rtol=0, atol=1e-15 * scale / eps * 50)
    assert np.abs(expect).max() > 1e3 * 1e-15 * scale / eps  # truncation really dominates


def test_fd_step_rules():
    em = 2.0 ** -52
    root = math.sqrt(em)
    x_small = np.full(4, 0.1)  # ||x|| = 0.2
    x_big = np.full(4, 1.5)  # ||x|| = 3
    v = np.full(4, 2.0)  # ||v|| = 4
    assert fd_step(EPS_PAPER, em, x_small, v) == pytest.approx(root, rel=1e-15)
    assert fd_step(EPS_PAPER, em, x_big, v) == pytest.approx(3 * root, rel=1e-15)
    assert fd_step(EPS_NORMALIZED, em, x_big, v) == pytest.approx(root * 4 / 4, rel=1e-15)
    assert fd_step(EPS_NORMALIZED, 2.0 ** -23, x_small, v) == pytest.approx(2.0 ** -11.5 * 1.2 / 4, rel=1e-14)


def test_fd_converges_to_ad_at_first_order():
    spec = tiny_cases()[2]
    p = Problem.from_spec(spec)
    x = state(spec, 17)
    xp = state(spec, 18)
    v = W.random_vector(p.n, 19)
    ad = jvp_ad(p, x, v, xp)[1]
    errs = [np.linalg.norm(jvp_fd(p, x, v, e, xp) - ad) for e in (1e-2, 1e-3, 1e-4)]
    assert errs[0] / errs[1] == pytest.approx(10, rel=0.05)
    assert errs[1] / errs[2] == pytest.approx(10, rel=0.05)
