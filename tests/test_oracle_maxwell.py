"""Pins of the oracle's paper-form Maxwell-Kerr residual (Appendix A.4; 2D TE) (no GPU).

* closed form: with grid sine modes in every plane the central differences
  are known exactly (D_x sin = sin(k h)/h cos, D_xx sin = -(4/h^2) sin^2(k h/2)
  sin), so curl curl E, and with the pointwise permittivity the residual, is
  known elementwise;
* boundary nodes are identity rows;
* the AD JVP equals the complex-step derivative (an independent method) at a
  state with |E| > 0;
* the guard: at E = 0 the AD JVP is the linear (Born) operator, the residual
  with chi = 0 and no source applied to the direction.
"""

import numpy as np
import pytest

import workloads as W
from oracle import Problem, jvp_ad, residual


def grid(nx, ny, omega=2.5, chi=0.05, loss=0.05):
    spec = W.maxwell_spec(nx, omega=omega, chi=chi, loss=loss, ny=ny)
    return spec, Problem.from_spec(spec)


def sines(p, a, b):
    tx = a * np.pi * np.arange(p.nx) / (p.nx - 1)
    ty = b * np.pi * np.arange(p.ny) / (p.ny - 1)
    return np.sin(tx)[None, :], np.sin(ty)[:, None], np.cos(tx)[None, :], np.cos(ty)[:, None], \
        a * np.pi / (p.nx - 1), b * np.pi / (p.ny - 1)


@pytest.mark.parametrize("nx,ny,chi", [(17, 13, 0.05), (24, 24, 0.3), (9, 21, 0.0)])
def test_maxwell_sine_modes_closed_form(nx, ny, chi):
    spec, p = grid(nx, ny, omega=3.1, chi=chi)
    amps = (0.7, -0.3, 0.4, 0.9)
    modes = ((1, 2), (2, 1), (2, 3), (1, 1))
    planes, cc = [], []
    D = []
    for (a, b), A in zip(modes, amps):
        sx, sy, cx, cy, kx, ky = sines(p, a, b)
        planes.append(A * sx * sy)
        D.append(dict(
            dxx=-(4.0 / p.hx ** 2) * np.sin(kx / 2) ** 2 * A * sx * sy,
            dyy=-(4.0 / p.hy ** 2) * np.sin(ky / 2) ** 2 * A * sx * sy,
            dxdy=(np.sin(kx) / p.hx) * (np.sin(ky) / p.hy) * A * cx * cy))
    xr, xi, yr, yi = planes
    m = 1.0 + chi * np.sqrt(xr ** 2 + xi ** 2 + yr ** 2 + yi ** 2)
    w2, L = p.k0 ** 2, p.eps_im
    f = W.maxwell_source(nx, omega=p.k0, ny=ny).reshape(4, ny, nx)
    exp = [D[2]["dxdy"] - D[0]["dyy"] - w2 * m * (xr + L * xi) - f[0],
           D[3]["dxdy"] - D[1]["dyy"] - w2 * m * (xi - L * xr) - f[1],
           D[0]["dxdy"] - D[2]["dxx"] - w2 * m * (yr + L * yi) - f[2],
           D[1]["dxdy"] - D[3]["dxx"] - w2 * m * (yi - L * yr) - f[3]]
    x = np.concatenate([q.ravel() for q in planes])
    got = residual(p, x, x, f.ravel()).reshape(4, ny, nx)
    for q in range(4):
        e = exp[q].copy()
        e[0, :], e[-1, :], e[:, 0], e[:, -1] = planes[q][0, :], planes[q][-1, :], planes[q][:, 0], planes[q][:, -1]
        assert np.max(np.abs(got[q] - e)) <= 1e-12 * max(1.0, np.abs(e).max()), q


def test_maxwell_boundary_rows_are_identity():
    spec, p = grid(11, 9)
    rng = np.random.default_rng(3)
    x, s = rng.standard_normal((2, p.n))
    F = residual(p, x, x, s).reshape(4, p.ny, p.nx)
    X = x.reshape(4, p.ny, p.nx)
    for edge in (np.s_[:, 0, :], np.s_[:, -1, :], np.s_[:, :, 0], np.s_[:, :, -1]):
        assert np.array_equal(F[edge], X[edge])


def test_maxwell_ad_equals_complex_step():
    spec, p = grid(10, 8, omega=4.0, chi=0.2)
    rng = np.random.default_rng(4)
    x = 0.5 + rng.uniform(0.2, 1.0, p.n)  # |E| > 0 everywhere: the residual is analytic there
    v = rng.standard_normal(p.n)
    src = W.maxwell_source(10, omega=4.0, ny=8)
    _, jv = jvp_ad(p, x, v, x, src)
    h = 1e-30
    cs = np.imag(residual(p, x + 1j * h * v, x, src)) / h
    assert np.max(np.abs(jv - cs)) <= 1e-12 * np.abs(cs).max()


def test_maxwell_guard_gives_the_born_operator_at_zero():
    spec, p = grid(12, 10, omega=3.0, chi=0.4)
    v = W.random_vector(p.n, 5)
    F0, jv = jvp_ad(p, np.zeros(p.n), v, np.zeros(p.n), None)
    assert np.all(np.isfinite(jv))
    lin = Problem.from_spec(dict(spec, chi3=0.0))
    born = residual(lin, v, v, None)  # linear in v without chi and source
    assert np.max(np.abs(jv - born)) <= 1e-13 * np.abs(born).max()
