"""Block-diagonal complex shifted-Laplacian (CSLP) preconditioner of the 2D TE
Maxwell-Kerr problem and of the scalar Helmholtz-Kerr workload (oracle; TEST
INFRASTRUCTURE).

Paper, Appendix A.4 ("Preconditioning"): a matrix-free diagonal preconditioner
built from the curl-curl operator's own diagonal and a damped permittivity.
At an interior node, with the permittivity of the current Newton iterate
eps(E) = (1 - loss i)(1 + chi |E|) (eps0 = mu0 = 1) damped to
eps_p = eps(E) (1 - 0.5 i):

    Ex component:  M_xx = 2 / hy^2 - omega^2 eps_p
    Ey component:  M_yy = 2 / hx^2 - omega^2 eps_p

(2 / hy^2 is the diagonal of -d_yy acting on Ex in curl curl E, 2 / hx^2 that
of -d_xx acting on Ey.)  Each entry multiplies the complex component
(Re + i Im) of its node, so on the real unknowns it is a 2 x 2 block per
component and node.  Readings: the PEC boundary rows are F = E, whose
Jacobian is the identity, so M = 1 there; |E| is taken at the Newton iterate
and frozen for the whole linear solve (M depends on the state, not on the
Krylov vector).

Helmholtz-Kerr (reading: the paper defines the preconditioner for the TE
problem only; the same construction on the scalar operator
-Lap E - k0^2 eps(E) E, eps(E) = eps_L + chi3 |E|^2): the diagonal of -Lap is
2 / hx^2 + 2 / hy^2, so

    M = 2 / hx^2 + 2 / hy^2 - k0^2 eps(E) (1 - 0.5 i)

on the one complex component of an interior node, 1 on the boundary.

It is applied on the right: GMRES runs on z -> J M^{-1} z and the update is
dx = M^{-1} z, so the residual GMRES minimizes and tests is that of
J dx = rhs.
"""

from __future__ import annotations

import numpy as np

from .problems import Problem, interior_mask, join, split

DAMPING = 0.5  # the paper's damping of the preconditioner's permittivity, eps (1 - 0.5 i)


def cslp_diagonal(p: Problem, x, damping: float = DAMPING):
    """The complex diagonal entries at the state x, one (ny, nx) array per complex component
    (1 on the boundary): (M_xx, M_yy) for Maxwell-Kerr, (M,) for Helmholtz-Kerr."""
    inner = interior_mask(p) > 0
    if p.kind == "maxwell":
        exr, exi, eyr, eyi = split(p, np.asarray(x, dtype=np.float64))
        absE = np.sqrt(exr * exr + exi * exi + eyr * eyr + eyi * eyi)
        eps = (1.0 - 1j * p.eps_im) * (1.0 + p.chi3 * absE)
        eps_p = eps * (1.0 - 1j * damping)
        w2 = p.k0 * p.k0
        mxx = np.where(inner, 2.0 / (p.hy * p.hy) - w2 * eps_p, 1.0 + 0j)
        myy = np.where(inner, 2.0 / (p.hx * p.hx) - w2 * eps_p, 1.0 + 0j)
        return mxx, myy
    if p.kind == "kerr":
        re, im = split(p, np.asarray(x, dtype=np.float64))
        eps = (p.eps_re + p.chi3 * (re * re + im * im)) + 1j * p.eps_im
        eps_p = eps * (1.0 - 1j * damping)
        diag = 2.0 / (p.hx * p.hx) + 2.0 / (p.hy * p.hy)
        return (np.where(inner, diag - p.k0 * p.k0 * eps_p, 1.0 + 0j),)
    raise ValueError("the CSLP preconditioner is defined for the Maxwell-Kerr and Helmholtz-Kerr problems")


def cslp_solve(p: Problem, x, v, damping: float = DAMPING):
    """M^{-1} v for the preconditioner frozen at the state x."""
    diags = cslp_diagonal(p, x, damping)
    parts = split(p, np.asarray(v, dtype=np.float64))
    out = []
    for k, m in enumerate(diags):
        c = (parts[2 * k] + 1j * parts[2 * k + 1]) / m
        out += [c.real, c.imag]
    return join(p, out)
