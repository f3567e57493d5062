"""BiCGSTAB (oracle).

The paper's second Krylov method for nonsymmetric Jacobians (Section 2: the
short-recurrence method of van der Vorst, lower memory than GMRES, less
monotone convergence; Section 3.3: its iteration cap is the same 100 as the
GMRES restart cap).  The standard stabilized bi-conjugate gradient
iteration, with the conventions shared with the GMRES oracle:

* initial guess x0 = 0, so r0 = rhs; the shadow residual is r0 itself;
* tolerance relative to ||rhs||: the solve stops when ||s|| (half step) or
  ||r|| (full step) falls to tol ||rhs||; at most ``maxiter`` iterations;
* one iteration: rho = (r0, r); beta = (rho / rho_prev) (alpha / omega);
  p = r + beta (p - omega v) (p = r in the first iteration); v = J p;
  alpha = rho / (r0, v); s = r - alpha v; [stop with x += alpha p if s is
  small]; t = J s; omega = (t, s) / (t, t); x += alpha p + omega s;
  r = s - omega t;
* breakdown (rho, (r0, v) or (t, t) exactly zero, or omega zero) ends the
  solve unconverged; a non-finite scalar ends it with ``nonfinite``.

"Iterations" counts completed iterations (two JVPs each; one when the half
step converged).
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class BicgstabInfo:
    converged: bool = False
    iters: int = 0
    nonfinite: bool = False
    breakdown: bool = False
    res: list = field(default_factory=list)  # ||r|| (or ||s|| at a half-step stop) after each iteration


def bicgstab(matvec, rhs: np.ndarray, tol: float = 1e-8, maxiter: int = 100):
    """Solve J x = rhs; returns (x, BicgstabInfo)."""
    n = rhs.shape[0]
    x = np.zeros(n)
    info = BicgstabInfo()
    bnorm = float(np.linalg.norm(rhs))
    if not math.isfinite(bnorm):
        info.nonfinite = True
        return x, info
    if bnorm == 0.0:
        info.converged = True
        return x, info
    target = tol * bnorm
    r = rhs.copy()
    r0 = rhs.copy()
    p = np.zeros(n)
    v = np.zeros(n)
    rho_prev = alpha = omega = 1.0
    for it in range(1, maxiter + 1):
        rho = float(np.dot(r0, r))
        if not math.isfinite(rho):
            info.nonfinite = True
            return x, info
        if rho == 0.0:
            info.breakdown = True
            return x, info
        if it == 1:
            p = r.copy()
        else:
            beta = (rho / rho_prev) * (alpha / omega)
            p = r + beta * (p - omega * v)
        v = matvec(p)
        r0v = float(np.dot(r0, v))
        if not math.isfinite(r0v):
            info.nonfinite = True
            return x, info
        if r0v == 0.0:
            info.breakdown = True
            return x, info
        alpha = rho / r0v
        s = r - alpha * v
        snorm = float(np.linalg.norm(s))
        if not math.isfinite(snorm):
            info.nonfinite = True
            return x, info
        if snorm <= target:
            x = x + alpha * p
            info.iters = it
            info.res.append(snorm)
            info.converged = True
            return x, info
        t = matvec(s)
        tt = float(np.dot(t, t))
        ts = float(np.dot(t, s))
        if not (math.isfinite(tt) and math.isfinite(ts)):
            info.nonfinite = True
            return x, info
        if tt == 0.0:
            info.breakdown = True
            return x, info
        omega = ts / tt
        x = x + alpha * p + omega * s
        r = s - omega * t
        rnorm = float(np.linalg.norm(r))
        info.iters = it
        info.res.append(rnorm)
        if not math.isfinite(rnorm):
            info.nonfinite = True
            return x, info
        if rnorm <= target:
            info.converged = True
            return x, info
        if omega == 0.0:
            info.breakdown = True
            return x, info
        rho_prev = rho
    return x, info
