"""Pins of the oracle's inexact Newton solve (paper Section 2: Newton step,
stopping test, backtracking line search; Section 3.4: failure rules).

* Linear special cases: Gray-Scott with F = k = 0 and u = 0 is a backward-Euler
  heat step for v (FFT closed form); Kerr with chi3 = 0 is linear Helmholtz
  with Dirichlet (PEC) nodes (DST-I closed form).
* Discrete manufactured solutions: s := F(x_ex; 0)/dt, then F(x; s) = 0 is
  solved back to x_ex.
* Quadratic local convergence of Newton with the AD JVP.
* Spatially uniform Gray-Scott equals an independent 2x2 Newton per cell.
* Second-order spatial convergence (continuous manufactured solution).
* AD and FD reach the same converged solution (paper, Section 1 and Table 2).
* The line search accepts only Armijo steps and halves otherwise.
* Failure classification forced from the host.
"""

import math

import numpy as np
import pytest
import scipy.fft as sfft

import workloads as W
from oracle import NewtonOptions, Problem, newton_solve, residual, run_failed, step_failed
from oracle.newton import NONFINITE, NOT_CONVERGED, NewtonInfo


def test_grayscott_heat_step_fft_closed_form():
    n = 24
    spec = W.grayscott_spec(n, D=1e-3, Dv=2e-3, F=0.0, k=0.0, dt=0.5, h=0.05)
    p = Problem.from_spec(spec)
    vn = 1.0 + 0.2 * W.random_vector(n * n, 1).reshape(n, n)
    xp = np.concatenate([np.zeros(n * n), vn.ravel()])
    x, info = newton_solve(p, xp, NewtonOptions(tol_newton=1e-13, tol_krylov=1e-14, m=30))
    assert info.converged
    k = np.arange(n)
    lam = (4 / spec["hx"] ** 2) * np.sin(np.pi * k / n)[None, :] ** 2 \
        + (4 / spec["hy"] ** 2) * np.sin(np.pi * k / n)[:, None] ** 2
    v_exact = np.real(np.fft.ifft2(np.fft.fft2(vn) / (1 + spec["dt"] * spec["Dv"] * lam)))
    assert np.array_equal(x[: n * n], np.zeros(n * n))
    np.testing.assert_allclose(x[n * n:].reshape(n, n), v_exact, rtol=0, atol=1e-11)


def test_kerr_linear_helmholtz_dst_closed_form():
    n = 14
    spec = W.kerr_spec(n, chi3=0.0, eps_re=1.0, eps_im=0.3, cells_per_wavelength=7.0)
    p = Problem.from_spec(spec)
    f = W.kerr_gaussian_source(n, amp=1.0, sigma=2.0)
    x, info = newton_solve(p, np.zeros(p.n), NewtonOptions(tol_newton=1e-13, tol_krylov=1e-14, m=200,
                                                            max_newton=3), source=f)
    assert info.converged
    fi = f.reshape(n, n, 2)[1:-1, 1:-1]
    fc = fi[..., 0] + 1j * fi[..., 1]
    q = np.arange(1, n - 1)
    lam1 = 4 * np.sin(np.pi * q / (2 * (n - 1))) ** 2
    lam = lam1[None, :] + lam1[:, None]
    eps = spec["eps_re"] + 1j * spec["eps_im"]
    denom = lam - spec["k0"] ** 2 * eps
    Ec = sfft.idstn(sfft.dstn(fc.real, type=1) / denom, type=1) \
        + 1j * sfft.idstn(sfft.dstn(fc.imag, type=1) / denom, type=1)
    E = x.reshape(n, n, 2)
    np.testing.assert_allclose(E[1:-1, 1:-1, 0] + 1j * E[1:-1, 1:-1, 1], Ec, rtol=0, atol=1e-12)
    assert not E[0].any() and not E[-1].any() and not E[:, 0].any() and not E[:, -1].any()


def manufactured(name, n, seed):
    spec, xp, _ = W.config(name, seed=seed, n=n)
    if name == "burgers2d":
        spec = W.burgers2d_spec(n, nu=0.02, dt=0.01)
    if name == "grayscott":
        xp = W.grayscott_initial(n, seed, side_frac=1 / 8, patches=3)
    p = Problem.from_spec(spec)
    x_ex = xp + 0.05 * np.sin(np.arange(p.n) * 0.37)
    s = residual(p, x_ex, xp) / spec["dt"]
    return p, xp, x_ex, s


@pytest.mark.parametrize("name,n", [("burgers1d", 64), ("burgers2d", 16), ("grayscott", 16)])
def test_discrete_manufactured_solution(name, n):
    p, xp, x_ex, s = manufactured(name, n, 3)
    x, info = newton_solve(p, xp, NewtonOptions(tol_newton=1e-12, tol_krylov=1e-13), source=s)
    assert info.converged
    assert abs(np.linalg.norm(residual(p, x_ex, xp, s))) <= 1e-13 * np.linalg.norm(x_ex)
    np.testing.assert_allclose(x, x_ex, rtol=0, atol=1e-10)


def test_kerr_manufactured_solution():
    n = 12
    spec = W.kerr_spec(n, chi3=0.5, eps_re=1.0, eps_im=0.2, cells_per_wavelength=6.0)
    p = Problem.from_spec(spec)
    i = np.arange(n)[None, :]
    j = np.arange(n)[:, None]
    mode = np.sin(np.pi * i / (n - 1)) * np.sin(np.pi * 2 * j / (n - 1))
    E = np.zeros((n, n, 2))
    E[..., 0] = 0.8 * mode
    E[..., 1] = -0.3 * mode
    e_ex = E.ravel()
    f = residual(p, e_ex, None, np.zeros(p.n))  # F(E_ex; f=0) = N(E_ex) inside, E_ex = 0 on PEC
    x, info = newton_solve(p, np.zeros(p.n), NewtonOptions(tol_newton=1e-12, tol_krylov=1e-13, m=100,
                                                            max_newton=50), source=f)
    assert info.converged
    np.testing.assert_allclose(x, e_ex, rtol=0, atol=1e-10)


def test_quadratic_convergence_ad():
    spec = W.burgers1d_spec(256, nu=0.01, dt=5e-2)
    p = Problem.from_spec(spec)
    xp = W.burgers1d_initial(256, 0)
    x, info = newton_solve(p, xp, NewtonOptions(tol_newton=1e-12, tol_krylov=1e-13, max_newton=15,
                                                max_restarts=200))
    r = info.rel_res
    assert info.converged
    orders = [math.log(r[k + 1] / r[k]) / math.log(r[k] / r[k - 1])
              for k in range(1, len(r) - 1) if r[k + 1] > 1e-12]
    assert len(orders) >= 2, r
    assert min(orders) > 1.6 and max(orders) > 1.9, (orders, r)


def test_uniform_grayscott_equals_per_cell_newton():
    n = 8
    spec = W.grayscott_spec(n, dt=3.0)
    p = Problem.from_spec(spec)
    u0, v0 = 0.3, 0.6
    xp = np.concatenate([np.full(n * n, u0), np.full(n * n, v0)])
    x, info = newton_solve(p, xp, NewtonOptions(tol_newton=1e-14, tol_krylov=1e-15))
    assert info.converged
    # independent 2x2 Newton on G(u, v) = 0
    dt, Fe, k = spec["dt"], spec["F"], spec["k"]
    u, v = u0, v0
    for _ in range(50):
        g1 = u - u0 + dt * (-u * u * v + (Fe + k) * u)
        g2 = v - v0 + dt * (u * u * v - Fe * (1 - v))
        a, b = 1 + dt * (-2 * u * v + Fe + k), -dt * u * u
        c, d = dt * 2 * u * v, 1 + dt * (u * u + Fe)
        det = a * d - b * c
        u, v = u - (d * g1 - b * g2) / det, v - (-c * g1 + a * g2) / det
    np.testing.assert_allclose(x[: n * n], u, rtol=1e-13)
    np.testing.assert_allclose(x[n * n:], v, rtol=1e-13)


def test_second_order_spatial_convergence():
    nu, dt = 0.05, 0.01
    errs = []
    for n in (32, 64, 128):
        spec = W.burgers1d_spec(n, nu=nu, dt=dt)
        p = Problem.from_spec(spec)
        xg = np.arange(n) / n
        tw = 2 * np.pi
        ue = np.sin(tw * xg) + 0.5 * np.cos(2 * tw * xg)
        ue_x = tw * np.cos(tw * xg) - tw * np.sin(2 * tw * xg)
        ue_xx = -tw**2 * np.sin(tw * xg) - 2 * tw**2 * np.cos(2 * tw * xg)
        un = 0.9 * np.sin(tw * xg)
        s = (ue - un) / dt + ue * ue_x - nu * ue_xx
        x, info = newton_solve(p, un, NewtonOptions(tol_newton=1e-13, tol_krylov=1e-14), source=s)
        assert info.converged
        errs.append(np.abs(x - ue).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.85 < o < 2.15 for o in orders), orders


def test_ad_and_fd_reach_the_same_solution():
    spec, xp, _ = W.config("grayscott", n=32)
    p = Problem.from_spec(spec)
    opts = dict(tol_newton=1e-10, tol_krylov=1e-11)
    xa, ia = newton_solve(p, xp, NewtonOptions(mode="ad", **opts))
    xf, if_ = newton_solve(p, xp, NewtonOptions(mode="fd", eps_rule="normalized", **opts))
    assert ia.converged and if_.converged
    bound = 10 * opts["tol_newton"] * ia.f0_norm  # ||J^-1|| <= 1 here: J = I + dt (diffusion + reaction)
    assert np.linalg.norm(xa - xf) <= bound


def test_fd_stalls_where_ad_converges_fp64_tight():
    # the paper's phenomenon in miniature: with a tolerance near FD's accuracy
    # floor the FD Jacobian cannot drive Newton below it, AD can
    spec, xp, _ = W.config("burgers1d")
    p = Problem.from_spec(spec)
    o = dict(tol_newton=1e-10, tol_krylov=1e-12, max_newton=6, max_restarts=20)
    _, ia = newton_solve(p, xp, NewtonOptions(mode="ad", **o))
    _, if_ = newton_solve(p, xp, NewtonOptions(mode="fd", **o))
    assert ia.converged and ia.newton_iters <= 3
    assert not if_.converged and if_.krylov_iters > 20 * ia.krylov_iters


def test_line_search_armijo_and_halving():
    spec = W.burgers1d_spec(64, nu=1e-3, dt=2.0)
    p = Problem.from_spec(spec)
    xp = 1.0 + 2.0 * np.sin(2 * np.pi * np.arange(64) / 64)
    opts = NewtonOptions(tol_newton=1e-8, tol_krylov=1e-10, max_newton=40)
    x, info = newton_solve(p, xp, opts, record=True)
    assert info.ls_backtracks > 0
    for k, alpha in enumerate(info.alphas):
        xk, xk1 = info.iterates[k], info.iterates[k + 1]
        fk = np.linalg.norm(residual(p, xk, xp))
        dx = (xk1 - xk) / alpha
        f_acc = np.linalg.norm(residual(p, xk + alpha * dx, xp))
        if alpha > 2.0 ** -opts.ls_max_backtracks:
            assert f_acc <= (1 - opts.ls_c * alpha) * fk * (1 + 1e-12)
        if alpha < 1.0:
            f_prev = np.linalg.norm(residual(p, xk + 2 * alpha * dx, xp))
            assert not (f_prev <= (1 - opts.ls_c * 2 * alpha) * fk)
        assert math.log2(alpha) == int(math.log2(alpha))


def test_failure_modes_forced_from_host():
    spec, xp, _ = W.config("burgers1d", n=32)
    p = Problem.from_spec(spec)
    bad = xp.copy()
    bad[5] = np.nan
    _, info = newton_solve(p, bad, NewtonOptions())
    assert info.status == NONFINITE
    _, info = newton_solve(p, xp, NewtonOptions(tol_newton=1e-15, max_newton=1))
    assert info.status == NOT_CONVERGED and info.newton_iters == 1
    # residual exactly zero at the start: converged with no iteration
    zero = np.zeros(32)
    _, info = newton_solve(p, zero, NewtonOptions())
    assert info.converged and info.newton_iters == 0 and info.rel_res == [0.0]
    # classification (Section 3.4): > 20% of steps beyond 100 tol fail the run
    ok = NewtonInfo(status="ok", converged=True, rel_res=[1.0, 1e-7])
    slow = NewtonInfo(status=NOT_CONVERGED, rel_res=[1.0, 5e-5])  # within 100x of 1e-6
    badstep = NewtonInfo(status=NOT_CONVERGED, rel_res=[1.0, 1e-3])
    assert not step_failed(slow, 1e-6) and step_failed(badstep, 1e-6)
    assert not run_failed([ok] * 8 + [badstep] * 2, 1e-6)
    assert run_failed([ok] * 7 + [badstep] * 3, 1e-6)
    assert run_failed([ok] * 9 + [NewtonInfo(status=NONFINITE)], 1e-6)
