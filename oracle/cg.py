"""Conjugate gradients (oracle).

The paper's Krylov method for symmetric positive-definite Jacobians (Section
2: Hestenes and Stiefel's method, short recurrences, valid only for SPD
systems; Section 3.3: used on the reaction-diffusion problem, whose
linearization is SPD, with the same iteration cap as the other methods).
The textbook iteration, with the conventions shared with the other oracles:

* initial guess x0 = 0, so r0 = rhs and p0 = r0;
* tolerance relative to ||rhs||: stop when ||r|| <= tol ||rhs||, at most
  ``maxiter`` iterations (one JVP each);
* one iteration: alpha = (r, r) / (p, J p); x += alpha p; r -= alpha J p;
  beta = (r_new, r_new) / (r, r); p = r_new + beta p;
* (p, J p) <= 0 means J is not positive definite along p: the solve ends
  unconverged with ``breakdown``; a non-finite scalar ends it with
  ``nonfinite``.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CgInfo:
    converged: bool = False
    iters: int = 0
    nonfinite: bool = False
    breakdown: bool = False
    res: list = field(default_factory=list)  # ||r|| after each iteration


def cg(matvec, rhs: np.ndarray, tol: float = 1e-8, maxiter: int = 100):
    """Solve J x = rhs for SPD J; returns (x, CgInfo)."""
    n = rhs.shape[0]
    x = np.zeros(n)
    info = CgInfo()
    bnorm = float(np.linalg.norm(rhs))
    if not math.isfinite(bnorm):
        info.nonfinite = True
        return x, info
    if bnorm == 0.0:
        info.converged = True
        return x, info
    target = tol * bnorm
    r = rhs.copy()
    p = r.copy()
    rr = float(np.dot(r, r))
    for it in range(1, maxiter + 1):
        Jp = matvec(p)
        pJp = float(np.dot(p, Jp))
        if not math.isfinite(pJp):
            info.nonfinite = True
            return x, info
        if pJp <= 0.0:
            info.breakdown = True
            return x, info
        alpha = rr / pJp
        x = x + alpha * p
        r = r - alpha * Jp
        rr_new = float(np.dot(r, r))
        rn = math.sqrt(rr_new) if rr_new >= 0.0 else float("nan")
        info.iters = it
        info.res.append(rn)
        if not math.isfinite(rn):
            info.nonfinite = True
            return x, info
        if rn <= target:
            info.converged = True
            return x, info
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, info
