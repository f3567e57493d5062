"""Jacobian-vector products of the discrete residual (oracle).

* AD (paper, Section 2, the ``jvp`` pair): forward-mode dual numbers pushed
  through the same residual function; returns (F(x), J(x) v).
* FD (paper, Section 2, the finite-difference JVP): (F(x + eps v) - F(x)) / eps,
  the residual evaluated twice with the same code, nothing cancelled by hand.
* FD step size: the paper's rule eps = sqrt(eps_mach) * max(1, ||x||) (its
  step-size equation, no clipping), and the normalized variant
  eps = sqrt(eps_mach) * (1 + ||x||) / ||v|| used by the Gray-Scott workload.
  ``eps_mach`` is the machine epsilon of the arithmetic the perturbed state is
  formed in (2^-52 for FP64, 2^-23 for FP32).
"""

from __future__ import annotations

import math

import numpy as np

from .dual import Dual
from .problems import Problem, residual

EPS_PAPER = "paper"
EPS_NORMALIZED = "normalized"

EPS_MACH = {"f64": 2.0 ** -52, "f32": 2.0 ** -23, "f16s": 2.0 ** -23}


def jvp_ad(p: Problem, x, v, x_prev, source=None):
    """(F(x), J(x) v) by forward-mode AD."""
    d = residual(p, Dual(np.asarray(x, float), np.asarray(v, float)), x_prev, source)
    return d.val, d.tan


def fd_step(rule: str, eps_mach: float, x, v) -> float:
    """FD perturbation size under ``rule`` (2-norms of the whole state vectors)."""
    xn = float(np.linalg.norm(x))
    root = math.sqrt(eps_mach)
    if rule == EPS_PAPER:
        return root * max(1.0, xn)
    if rule == EPS_NORMALIZED:
        vn = float(np.linalg.norm(v))
        return root * (1.0 + xn) / vn
    raise ValueError(rule)


def jvp_fd(p: Problem, x, v, eps: float, x_prev, source=None, Fx=None):
    """(F(x + eps v) - F(x)) / eps; ``Fx`` may pass F(x) already computed."""
    if Fx is None:
        Fx = residual(p, x, x_prev, source)
    return (residual(p, x + eps * v, x_prev, source) - Fx) / eps
