"""Hand-derived dense Jacobians of the discrete residuals (test pins only).

Derived on paper from the stencil formulas, entry by entry, and written with
explicit index loops; they share no code with the oracle's residual functions.
Used to pin the oracle's dual-number JVP ("AD equals the analytic Jacobian,
column by column") on tiny grids.  Entries for neighbours that coincide on
very small periodic grids are accumulated.
"""

from __future__ import annotations

import numpy as np


def burgers1d(spec: dict, u: np.ndarray) -> np.ndarray:
    """dF_i/du_l for F_i = u_i - un_i + th dt [u_i (u_{i+1}-u_{i-1})/(2h) - nu (u_{i+1}-2u_i+u_{i-1})/h^2]."""
    n = spec["nx"]
    h = spec["hx"]
    c = spec["theta"] * spec["dt"]
    nu = spec["nu"]
    J = np.zeros((n, n))
    for i in range(n):
        ip, im = (i + 1) % n, (i - 1) % n
        J[i, i] += 1.0 + c * ((u[ip] - u[im]) / (2 * h) + 2 * nu / h**2)
        J[i, ip] += c * (u[i] / (2 * h) - nu / h**2)
        J[i, im] += c * (-u[i] / (2 * h) - nu / h**2)
    return J


def _idx2(nx, ny):
    def idx(f, j, i):
        return f * nx * ny + (j % ny) * nx + (i % nx)
    return idx


def burgers2d(spec: dict, x: np.ndarray) -> np.ndarray:
    nx, ny = spec["nx"], spec["ny"]
    hx, hy = spec["hx"], spec["hy"]
    c = spec["theta"] * spec["dt"]
    nu = spec["nu"]
    idx = _idx2(nx, ny)
    n = 2 * nx * ny
    J = np.zeros((n, n))
    U = x.reshape(2, ny, nx)
    for j in range(ny):
        for i in range(nx):
            u = U[0, j, i]
            v = U[1, j, i]
            for f in range(2):
                q = U[f]
                row = idx(f, j, i)
                dxq = (q[j, (i + 1) % nx] - q[j, (i - 1) % nx]) / (2 * hx)
                dyq = (q[(j + 1) % ny, i] - q[(j - 1) % ny, i]) / (2 * hy)
                # derivative w.r.t. the same field at the centre and neighbours
                J[row, idx(f, j, i)] += 1.0 + c * (2 * nu / hx**2 + 2 * nu / hy**2)
                J[row, idx(f, j, i + 1)] += c * (u / (2 * hx) - nu / hx**2)
                J[row, idx(f, j, i - 1)] += c * (-u / (2 * hx) - nu / hx**2)
                J[row, idx(f, j + 1, i)] += c * (v / (2 * hy) - nu / hy**2)
                J[row, idx(f, j - 1, i)] += c * (-v / (2 * hy) - nu / hy**2)
                # advecting velocity components u (multiplies D_x q) and v (multiplies D_y q)
                J[row, idx(0, j, i)] += c * dxq
                J[row, idx(1, j, i)] += c * dyq
    return J


def grayscott(spec: dict, x: np.ndarray) -> np.ndarray:
    nx, ny = spec["nx"], spec["ny"]
    hx, hy = spec["hx"], spec["hy"]
    c = spec["theta"] * spec["dt"]
    D, Dv, Fe, k = spec["D"], spec["Dv"], spec["F"], spec["k"]
    idx = _idx2(nx, ny)
    n = 2 * nx * ny
    J = np.zeros((n, n))
    U = x.reshape(2, ny, nx)
    for j in range(ny):
        for i in range(nx):
            u = U[0, j, i]
            v = U[1, j, i]
            for f, Df in ((0, D), (1, Dv)):
                row = idx(f, j, i)
                J[row, idx(f, j, i)] += 1.0 + c * Df * (2 / hx**2 + 2 / hy**2)
                for (dj, di, h) in ((0, 1, hx), (0, -1, hx), (1, 0, hy), (-1, 0, hy)):
                    J[row, idx(f, j + dj, i + di)] += -c * Df / h**2
            ru = idx(0, j, i)
            rv = idx(1, j, i)
            # F_u = ... + c(-u^2 v + (F+k) u);  F_v = ... + c(u^2 v - F (1 - v))
            J[ru, idx(0, j, i)] += c * (-2 * u * v + (Fe + k))
            J[ru, idx(1, j, i)] += c * (-u * u)
            J[rv, idx(0, j, i)] += c * (2 * u * v)
            J[rv, idx(1, j, i)] += c * (u * u + Fe)
    return J


def kerr(spec: dict, x: np.ndarray) -> np.ndarray:
    """Interleaved (re, im) unknowns; PEC boundary rows are identity rows."""
    nx, ny = spec["nx"], spec["ny"]
    hx, hy = spec["hx"], spec["hy"]
    k2 = spec["k0"] ** 2
    er, ei, chi = spec["eps_re"], spec["eps_im"], spec["chi3"]

    def idx(j, i, comp):
        return 2 * (j * nx + i) + comp

    n = 2 * nx * ny
    J = np.zeros((n, n))
    E = x.reshape(ny, nx, 2)
    for j in range(ny):
        for i in range(nx):
            if i == 0 or j == 0 or i == nx - 1 or j == ny - 1:
                J[idx(j, i, 0), idx(j, i, 0)] = 1.0
                J[idx(j, i, 1), idx(j, i, 1)] = 1.0
                continue
            a = E[j, i, 0]
            b = E[j, i, 1]
            diag = 2 / hx**2 + 2 / hy**2
            for comp in (0, 1):
                row = idx(j, i, comp)
                J[row, idx(j, i, comp)] += diag
                J[row, idx(j, i + 1, comp)] += -1 / hx**2
                J[row, idx(j, i - 1, comp)] += -1 / hx**2
                J[row, idx(j + 1, i, comp)] += -1 / hy**2
                J[row, idx(j - 1, i, comp)] += -1 / hy**2
            # F_re = ... - k2 [(er + chi(a^2+b^2)) a - ei b]
            J[idx(j, i, 0), idx(j, i, 0)] += -k2 * (er + chi * (a * a + b * b) + 2 * chi * a * a)
            J[idx(j, i, 0), idx(j, i, 1)] += -k2 * (2 * chi * a * b - ei)
            # F_im = ... - k2 [(er + chi(a^2+b^2)) b + ei a]
            J[idx(j, i, 1), idx(j, i, 1)] += -k2 * (er + chi * (a * a + b * b) + 2 * chi * b * b)
            J[idx(j, i, 1), idx(j, i, 0)] += -k2 * (2 * chi * a * b + ei)
    return J


DENSE = {"burgers1d": burgers1d, "burgers2d": burgers2d, "grayscott": grayscott, "kerr": kerr}
