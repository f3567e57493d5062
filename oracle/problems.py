"""Discrete nonlinear residuals F(x^k, x*) of the benchmark problems (oracle).

Written once, generically: the functions accept NumPy arrays, complex arrays
(for complex-step checks) and ``Dual`` numbers (for the forward-mode JVP), so
F, the FD JVP and the AD JVP all evaluate the same residual code, as the
paper's methodology requires (Section 3.1).

Discretization (paper, Section 3.2 and Appendix A): second-order central
differences, D_x f = (f_{i+1} - f_{i-1}) / (2h) and
D_xx f = (f_{i+1} - 2 f_i + f_{i-1}) / h^2, periodic wrap for the
time-dependent problems.  Time discretization is the theta scheme
(Crank-Nicolson at theta = 1/2, as in Appendix A.1; backward Euler at 1):

    F(x; x^n) = x - x^n + dt [theta N(x) + (1 - theta) N(x^n)] - dt s

with N the spatial operator written as u_t = -N(u) and ``s`` an optional source.

The Helmholtz-Kerr boundary value problem (scalar form of the workload, PEC
boundary nodes held by F = E as in the paper's Appendix A.4):

    interior:  F = -Lap E - k0^2 (eps_L + chi3 |E|^2) E - f
    boundary:  F = E

with |E|^2 = Re(E)^2 + Im(E)^2 written on the real and imaginary parts, so the
residual is a polynomial in real unknowns and forward-mode AD differentiates
through |E|^2 componentwise.

The scalar reaction-diffusion problem (Section 3.2; Appendix A.3)
u_t = D Lap u - u^3 with homogeneous Dirichlet conditions: N(u) = -D Lap u + u^3
in the theta scheme above at the interior nodes, F = u at the boundary nodes
(which hold the zero boundary value).  Its Jacobian on the interior nodes is
I + theta dt (-D L + 3 diag(u^2)), symmetric positive definite.

The paper-form Maxwell-Kerr boundary value problem (Appendix A.4): the 2D TE
field E = (Ex, Ey) (complex) with mu0 = eps0 = 1, frequency omega (the field
k0), source f = i omega J:

    interior:  F = curl curl E - omega^2 eps(E) E - f,
               eps(E) = (1 - i loss) (1 + chi |E|),  |E| = sqrt(|Ex|^2 + |Ey|^2)
    boundary:  F = E (PEC nodes held)

with (curl curl E)_x = D_x D_y Ey - D_yy Ex and (curl curl E)_y = D_x D_y Ex -
D_xx Ey (central differences; D_x D_y reaches the four diagonal neighbours),
loss = 0.05 (the field eps_im) and chi the field chi3.  |E| is not
differentiable at E = 0: the AD tangent of |E| is taken as 0 there (the guard),
so the JVP at E = 0 is the linear (Born) operator.

The Su-Olson non-equilibrium radiation diffusion system (Appendix A.2),
U_t = (1/3) Lap U - (U - V) + Q, V_t = xi (U - V): N = (-(1/3) Lap U + (U - V),
-xi (U - V)), source (Q, 0), Dirichlet boundary nodes (F = x there).  The
residual is affine in the state, so the FD difference quotient equals the
Jacobian product up to rounding.  Its two configurations: the dynamic one with
Dirichlet nodes all round, and the classic 1D profile on a 2D grid whose rows
wrap (``periodic_y``): only the first and last columns are boundary nodes.

Layouts are those of the ``workloads`` module: 1D ``u[i]``; two-field 2D
problems as two row-major planes of shape (ny, nx); Kerr as interleaved
(re, im) pairs of shape (ny, nx, 2).
"""

from __future__ import annotations

from dataclasses import dataclass, field, fields as dc_fields

import numpy as np

from .dual import Dual, concatenate, roll, stack_last


@dataclass(frozen=True)
class Problem:
    """A benchmark problem: kind, grid and physical parameters."""

    kind: str  # 'burgers1d' | 'burgers2d' | 'grayscott' | 'kerr' | 'rd2d' | 'suolson' | 'maxwell'
    nx: int
    ny: int = 1
    hx: float = 1.0
    hy: float = 1.0
    dt: float = 0.0
    theta: float = 1.0
    nu: float = 0.0  # Burgers viscosity
    D: float = 0.0  # Gray-Scott diffusivity of u; reaction-diffusion diffusivity
    Dv: float = 0.0  # Gray-Scott diffusivity of v
    F: float = 0.0  # Gray-Scott feed rate
    k: float = 0.0  # Gray-Scott kill rate
    k0: float = 0.0  # Kerr wavenumber
    eps_re: float = 1.0  # Kerr linear permittivity (real part)
    eps_im: float = 0.0  # Kerr linear permittivity (imaginary part)
    chi3: float = 0.0  # Kerr coefficient
    xi: float = 0.0  # Su-Olson material coupling
    periodic_y: bool = False  # Su-Olson's 1D-profile configuration: periodic rows, Dirichlet columns

    @classmethod
    def from_spec(cls, spec: dict) -> "Problem":
        names = {f.name for f in dc_fields(cls)}
        return cls(**{k: v for k, v in spec.items() if k in names})

    @property
    def n(self) -> int:
        """Number of real unknowns."""
        cells = self.nx * self.ny
        if self.kind == "maxwell":
            return 4 * cells
        return cells if self.kind in ("burgers1d", "rd2d") else 2 * cells

    @property
    def is_ibvp(self) -> bool:
        return self.kind not in ("kerr", "maxwell")


# ---------------------------------------------------------------------------
# Central differences (periodic wrap by np.roll: roll(f, -1)[i] = f[i+1])
# ---------------------------------------------------------------------------


def d1(f, h: float, axis: int):
    """First derivative, (f_{i+1} - f_{i-1}) / (2h)."""
    return (roll(f, -1, axis) - roll(f, 1, axis)) / (2.0 * h)


def d2(f, h: float, axis: int):
    """Second derivative, (f_{i+1} - 2 f_i + f_{i-1}) / h^2."""
    return (roll(f, -1, axis) - 2.0 * f + roll(f, 1, axis)) / (h * h)


def lap(f, p: Problem):
    """Five-point Laplacian D_xx + D_yy on a (ny, nx) array."""
    return d2(f, p.hx, 1) + d2(f, p.hy, 0)


# ---------------------------------------------------------------------------
# Field views
# ---------------------------------------------------------------------------


def split(p: Problem, x):
    """Flat state -> list of field arrays (or Duals)."""
    if p.kind == "burgers1d":
        return [x]
    if p.kind == "rd2d":
        return [x.reshape(p.ny, p.nx)]
    if p.kind == "maxwell":
        planes = x.reshape(4, p.ny, p.nx)
        return [planes[0], planes[1], planes[2], planes[3]]
    if p.kind == "kerr":
        e = x.reshape(p.ny, p.nx, 2)
        return [e[..., 0], e[..., 1]]
    planes = x.reshape(2, p.ny, p.nx)
    return [planes[0], planes[1]]


def join(p: Problem, parts):
    """List of field arrays -> flat state (inverse of ``split``)."""
    if p.kind == "burgers1d":
        return parts[0]
    if p.kind == "rd2d":
        return parts[0].ravel()
    if p.kind == "maxwell":
        return concatenate([q.ravel() for q in parts])
    if p.kind == "kerr":
        return stack_last(parts).ravel()
    return concatenate([parts[0].ravel(), parts[1].ravel()])


# ---------------------------------------------------------------------------
# Spatial operators N (time-dependent problems: u_t = -N(u))
# ---------------------------------------------------------------------------


def N_burgers1d(p: Problem, f):
    """N(u) = u D_x u - nu D_xx u (1D analogue of Appendix A.1)."""
    (u,) = f
    return [u * d1(u, p.hx, 0) - p.nu * d2(u, p.hx, 0)]


def N_burgers2d(p: Problem, f):
    """N(U) = Adv(U) - nu Lap(U), Adv(U) = u D_x U + v D_y U (Appendix A.1)."""
    u, v = f
    adv_u = u * d1(u, p.hx, 1) + v * d1(u, p.hy, 0)
    adv_v = u * d1(v, p.hx, 1) + v * d1(v, p.hy, 0)
    return [adv_u - p.nu * lap(u, p), adv_v - p.nu * lap(v, p)]


def N_grayscott(p: Problem, f):
    """Gray-Scott: u_t = D Lap u + u^2 v - (F+k) u,  v_t = Dv Lap v - u^2 v + F (1 - v)."""
    u, v = f
    uuv = u * u * v
    return [-p.D * lap(u, p) - uuv + (p.F + p.k) * u,
            -p.Dv * lap(v, p) + uuv - p.F * (1.0 - v)]


def N_rd2d(p: Problem, f):
    """Scalar reaction-diffusion: u_t = D Lap u - u^3 (Appendix A.3)."""
    (u,) = f
    return [-p.D * lap(u, p) + u * u * u]


def N_suolson(p: Problem, f):
    """Su-Olson: U_t = (1/3) Lap U - (U - V), V_t = xi (U - V) (Appendix A.2; the source enters as s)."""
    U, V = f
    d = U - V
    return [-(1.0 / 3.0) * lap(U, p) + d, -p.xi * d]


SPATIAL = {"burgers1d": N_burgers1d, "burgers2d": N_burgers2d, "grayscott": N_grayscott, "rd2d": N_rd2d,
           "suolson": N_suolson}


def N_apply(p: Problem, x):
    """Spatial operator on a flat state."""
    return join(p, SPATIAL[p.kind](p, split(p, x)))


# ---------------------------------------------------------------------------
# Helmholtz-Kerr
# ---------------------------------------------------------------------------


def interior_mask(p: Problem) -> np.ndarray:
    """1 on interior nodes, 0 on the boundary nodes (PEC or Dirichlet), shape (ny, nx).

    With ``periodic_y`` (Su-Olson's 1D-profile configuration) the rows wrap, so
    only the first and last columns are boundary nodes."""
    m = np.zeros((p.ny, p.nx))
    if p.periodic_y:
        m[:, 1:-1] = 1.0
    else:
        m[1:-1, 1:-1] = 1.0
    return m


def kerr_residual(p: Problem, x, source):
    """F = -Lap E - k0^2 (eps_L + chi3 |E|^2) E - f inside, F = E on the boundary."""
    re, im = split(p, x)
    f_re, f_im = split(p, source) if source is not None else (0.0, 0.0)
    a = p.eps_re + p.chi3 * (re * re + im * im)  # real part of the permittivity
    b = p.eps_im  # imaginary part (constant)
    k2 = p.k0 * p.k0
    n_re = -lap(re, p) - k2 * (a * re - b * im) - f_re
    n_im = -lap(im, p) - k2 * (a * im + b * re) - f_im
    m = interior_mask(p)
    return join(p, [m * n_re + (1.0 - m) * re, m * n_im + (1.0 - m) * im])


# ---------------------------------------------------------------------------
# Maxwell-Kerr, 2D TE
# ---------------------------------------------------------------------------


def guarded_norm(s):
    """|E| = sqrt(s) for s = |Ex|^2 + |Ey|^2; on duals the tangent is 0 where s = 0."""
    if isinstance(s, Dual):
        v = np.sqrt(s.val)
        pos = v > 0
        return Dual(v, np.where(pos, s.tan / (2.0 * np.where(pos, v, 1.0)), 0.0))
    return np.sqrt(s)


def maxwell_residual(p: Problem, x, source):
    """F = curl curl E - omega^2 eps(E) E - f inside, F = E on the boundary."""
    exr, exi, eyr, eyi = split(p, x)
    fxr, fxi, fyr, fyi = split(p, source) if source is not None else (0.0, 0.0, 0.0, 0.0)

    def dxdy(f):
        return d1(d1(f, p.hx, 1), p.hy, 0)

    w2 = p.k0 * p.k0
    loss = p.eps_im
    m = 1.0 + p.chi3 * guarded_norm(exr * exr + exi * exi + eyr * eyr + eyi * eyi)
    nxr = dxdy(eyr) - d2(exr, p.hy, 0) - w2 * (m * (exr + loss * exi)) - fxr
    nxi = dxdy(eyi) - d2(exi, p.hy, 0) - w2 * (m * (exi - loss * exr)) - fxi
    nyr = dxdy(exr) - d2(eyr, p.hx, 1) - w2 * (m * (eyr + loss * eyi)) - fyr
    nyi = dxdy(exi) - d2(eyi, p.hx, 1) - w2 * (m * (eyi - loss * eyr)) - fyi
    mk = interior_mask(p)
    return join(p, [mk * nxr + (1.0 - mk) * exr, mk * nxi + (1.0 - mk) * exi,
                    mk * nyr + (1.0 - mk) * eyr, mk * nyi + (1.0 - mk) * eyi])


# ---------------------------------------------------------------------------
# The residual F(x; x*)
# ---------------------------------------------------------------------------


def residual(p: Problem, x, x_prev, source=None):
    """Discrete residual F(x; x*) (paper, Section 2 and Appendix A).

    Time-dependent problems: x* = x^n is the previous time level; the theta
    scheme above.  Kerr: x* is only the Newton starting guess and the residual
    does not depend on it.
    """
    if p.kind == "kerr":
        return kerr_residual(p, x, source)
    if p.kind == "maxwell":
        return maxwell_residual(p, x, source)
    out = x - x_prev + (p.dt * p.theta) * N_apply(p, x)
    if p.theta != 1.0:
        out = out + (p.dt * (1.0 - p.theta)) * N_apply(p, x_prev)
    if source is not None:
        out = out - p.dt * source
    if p.kind == "rd2d":
        # homogeneous Dirichlet: boundary nodes are identity rows
        m = interior_mask(p).ravel()
        out = m * out + (1.0 - m) * x
    elif p.kind == "suolson":
        m = np.tile(interior_mask(p).ravel(), 2)
        out = m * out + (1.0 - m) * x
    return out


def as_dual(x, v) -> Dual:
    return Dual(np.asarray(x, dtype=np.float64), np.asarray(v, dtype=np.float64))
