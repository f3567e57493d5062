"""Pins of the oracle's discrete residuals against closed forms.

Each test evaluates the oracle on grid functions whose central differences are
known exactly (discrete Fourier modes, uniform states) and compares with the
closed form written in terms of sin/cos of the grid coordinates, not with the
shifted-array code under test.  Cited: paper Section 2 (residual and
theta-scheme), Appendix A.1 (Burgers, Taylor-Green vortex), A.3
(reaction-diffusion), A.4 (Kerr residual, PEC rows F = E).
"""

import numpy as np
import pytest

import workloads as W
from oracle import Problem, residual
from oracle.problems import N_apply


def fourier_d1(k, h):
    """D_x e^{i k x} = i sin(k h)/h e^{i k x}."""
    return np.sin(k * h) / h


def fourier_d2(k, h):
    """D_xx e^{i k x} = -(4/h^2) sin^2(k h / 2) e^{i k x}."""
    return -4.0 / h**2 * np.sin(k * h / 2) ** 2


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_burgers1d_fourier_mode(theta):
    nx = 48
    spec = W.burgers1d_spec(nx, nu=0.03, dt=0.01, theta=theta)
    p = Problem.from_spec(spec)
    h = spec["hx"]
    xg = np.arange(nx) * h
    kap = 2 * np.pi * 3
    c, A = 0.7, 0.4
    u = c + A * np.sin(kap * xg)
    un = -0.2 + 0.3 * np.cos(2 * np.pi * 2 * xg)  # another level, another mode

    def N_closed(base, amp, mode, kind):
        s1 = fourier_d1(mode, h)
        s2 = fourier_d2(mode, h)
        if kind == "sin":
            val = base + amp * np.sin(mode * xg)
            dx = amp * s1 * np.cos(mode * xg)
            dxx = amp * s2 * np.sin(mode * xg)
        else:
            val = base + amp * np.cos(mode * xg)
            dx = -amp * s1 * np.sin(mode * xg)
            dxx = amp * s2 * np.cos(mode * xg)
        return val * dx - spec["nu"] * dxx

    expect = u - un + spec["dt"] * (theta * N_closed(c, A, kap, "sin")
                                    + (1 - theta) * N_closed(-0.2, 0.3, 2 * np.pi * 2, "cos"))
    got = residual(p, u, un)
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-13)


def test_burgers2d_taylor_green_crank_nicolson():
    n = 32
    spec = W.burgers2d_spec(n, nu=0.05, dt=0.02, theta=0.5)
    p = Problem.from_spec(spec)
    h = spec["hx"]
    c = np.arange(n) * h
    X, Y = c[None, :], c[:, None]
    s1, s2 = fourier_d1(1.0, h), fourier_d2(1.0, h)

    def tgv(a):
        u = a * np.sin(X) * np.cos(Y)
        v = -a * np.cos(X) * np.sin(Y)
        ux, uy = a * s1 * np.cos(X) * np.cos(Y), -a * s1 * np.sin(X) * np.sin(Y)
        vx, vy = a * s1 * np.sin(X) * np.sin(Y), -a * s1 * np.cos(X) * np.cos(Y)
        lap_u, lap_v = 2 * s2 * u, 2 * s2 * v
        Nu = u * ux + v * uy - spec["nu"] * lap_u
        Nv = u * vx + v * vy - spec["nu"] * lap_v
        return np.concatenate([u.ravel(), v.ravel()]), np.concatenate([Nu.ravel(), Nv.ravel()])

    xk, Nk = tgv(0.9)
    xn, Nn = tgv(1.0)
    expect = xk - xn + spec["dt"] / 2 * (Nk + Nn)
    np.testing.assert_allclose(residual(p, xk, xn), expect, rtol=0, atol=1e-13)


def test_grayscott_trivial_state_is_steady():
    spec = W.grayscott_spec(16)
    p = Problem.from_spec(spec)
    x = np.concatenate([np.zeros(256), np.ones(256)])
    assert np.array_equal(residual(p, x, x), np.zeros(512))


def test_grayscott_mode_and_pointwise_terms():
    n = 24
    spec = W.grayscott_spec(n, D=3e-3, Dv=1e-3, F=0.05, k=0.07, dt=0.7, h=0.1)
    p = Problem.from_spec(spec)
    h = spec["hx"]
    c = np.arange(n)
    kx, ky = 2 * np.pi * 2 / n, 2 * np.pi * 3 / n  # modes per grid index
    u = 0.3 + 0.1 * np.cos(kx * c[None, :]) * np.cos(ky * c[:, None])
    v = 0.8 + 0.05 * np.sin(ky * c[:, None]) * np.ones((1, n))
    lam_u = fourier_d2(kx / h, h) + fourier_d2(ky / h, h)
    lam_v = fourier_d2(ky / h, h)
    lap_u = lam_u * (u - 0.3)
    lap_v = lam_v * (v - 0.8)
    Fe, k = spec["F"], spec["k"]
    Nu = -spec["D"] * lap_u - u * u * v + (Fe + k) * u
    Nv = -spec["Dv"] * lap_v + u * u * v - Fe * (1 - v)
    x = np.concatenate([u.ravel(), v.ravel()])
    xn = np.concatenate([(u * 0.5).ravel(), (v * 1.1).ravel()])
    expect = x - xn + spec["dt"] * np.concatenate([Nu.ravel(), Nv.ravel()])
    np.testing.assert_allclose(residual(p, x, xn), expect, rtol=0, atol=1e-13)


def test_source_enters_with_minus_dt():
    spec = W.grayscott_spec(8)
    p = Problem.from_spec(spec)
    x = W.grayscott_initial(8, seed=1)
    s = W.random_vector(p.n, 2)
    # uniform x = x_prev with zero diffusion effect: F = dt N(x) - dt s; compare two sources
    d = residual(p, x, x, source=s) - residual(p, x, x, source=2 * s)
    np.testing.assert_allclose(d, spec["dt"] * s, rtol=1e-14, atol=1e-15)


def test_kerr_sine_mode_closed_form():
    nx, ny = 20, 14
    spec = W.kerr_spec(nx, chi3=0.3, eps_re=1.2, eps_im=-0.1, cells_per_wavelength=6.0)
    spec["ny"] = ny
    p = Problem.from_spec(spec)
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    pm, qm = 2, 3
    mode = np.sin(np.pi * pm * i / (nx - 1)) * np.sin(np.pi * qm * j / (ny - 1))
    a_re, a_im = 0.6, -0.25
    E = np.zeros((ny, nx, 2))
    E[..., 0] = a_re * mode
    E[..., 1] = a_im * mode
    f = W.random_vector(2 * nx * ny, 5, 0.01).reshape(ny, nx, 2)
    lam = 4 * np.sin(np.pi * pm / (2 * (nx - 1))) ** 2 + 4 * np.sin(np.pi * qm / (2 * (ny - 1))) ** 2
    Ec = E[..., 0] + 1j * E[..., 1]
    eps = spec["eps_re"] + 1j * spec["eps_im"] + spec["chi3"] * np.abs(Ec) ** 2
    Fc = lam * Ec - spec["k0"] ** 2 * eps * Ec - (f[..., 0] + 1j * f[..., 1])
    got = residual(p, E.ravel(), None, f.ravel()).reshape(ny, nx, 2)
    inner = (slice(1, -1), slice(1, -1))
    np.testing.assert_allclose(got[inner][..., 0], Fc.real[inner], rtol=0, atol=1e-13)
    np.testing.assert_allclose(got[inner][..., 1], Fc.imag[inner], rtol=0, atol=1e-13)


def test_kerr_boundary_rows_hold_the_field():
    n = 9
    spec = W.kerr_spec(n, chi3=0.2)
    p = Problem.from_spec(spec)
    E = W.random_vector(2 * n * n, 3).reshape(n, n, 2)
    f = W.random_vector(2 * n * n, 4).reshape(n, n, 2)
    got = residual(p, E.ravel(), None, f.ravel()).reshape(n, n, 2)
    b = np.ones((n, n), bool)
    b[1:-1, 1:-1] = False
    assert np.array_equal(got[b], E[b])


def test_theta_one_ignores_previous_operator():
    # with theta = 1 only x - x_prev carries x_prev: F(x; x_prev) - F(x; 0) = -x_prev
    spec = W.burgers1d_spec(32)
    p = Problem.from_spec(spec)
    x = W.burgers1d_initial(32, 0)
    xp = W.random_vector(32, 9)
    np.testing.assert_allclose(residual(p, x, xp) - residual(p, x, np.zeros(32)), -xp, atol=1e-15)


def test_spatial_operator_of_constant_state():
    # constants: all differences vanish; Gray-Scott reduces to its reaction terms
    spec = W.grayscott_spec(6)
    p = Problem.from_spec(spec)
    u0, v0 = 0.2, 0.7
    x = np.concatenate([np.full(36, u0), np.full(36, v0)])
    Nu = -u0 * u0 * v0 + (spec["F"] + spec["k"]) * u0
    Nv = u0 * u0 * v0 - spec["F"] * (1 - v0)
    got = N_apply(p, x)
    np.testing.assert_allclose(got[:36], Nu, rtol=1e-15)
    np.testing.assert_allclose(got[36:], Nv, rtol=1e-15)
