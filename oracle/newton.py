"""Inexact Newton with backtracking line search (oracle).

Paper, Section 2: linearize F(x^k) at each iterate, solve J(x^k) dx = -F(x^k)
with the Krylov method (GMRES or BiCGSTAB; J only through JVPs), stop when
||F(x^k, x*)|| / ||F(x*, x*)|| < tol_Newton, and damp the update to
x^{k+1} = x^k + alpha dx with alpha reduced until the residual norm decreases
sufficiently.  The paper leaves the line-search constants open; the reading
taken here: Armijo condition ||F(x + alpha dx)|| <= (1 - c alpha) ||F(x)||
with c = 1e-4, alpha halved at most ``ls_max_backtracks`` times, and if no
trial passes the last one (alpha = 2^-ls_max_backtracks) is taken and counted
as a line-search failure.  A non-finite residual at an accepted iterate, or in
the Krylov solve, fails the solve.

Run-level failure rule (Section 3.4): an implicit step "fails" when its final
relative residual exceeds 100 tol_Newton; a run of several steps fails when
more than 20% of its steps fail, or on non-finite values.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import gmres as gm
from .bicgstab import bicgstab
from .cg import cg
from .jvp import EPS_MACH, EPS_PAPER, fd_step, jvp_ad, jvp_fd
from .precond import cslp_solve
from .problems import Problem, residual

OK = "ok"
NONFINITE = "nonfinite"
NOT_CONVERGED = "not_converged"


@dataclass
class NewtonOptions:
    mode: str = "ad"  # 'ad' | 'fd'
    m: int = 30
    tol_newton: float = 1e-6
    tol_krylov: float = 1e-8
    max_newton: int = 15
    max_restarts: int = 100
    ls_c: float = 1e-4
    ls_max_backtracks: int = 10
    eps_rule: str = EPS_PAPER
    eps_mach: float = EPS_MACH["f64"]
    fd_eps: float = 0.0  # > 0: fixed FD step
    breakdown_tol: float = 1e-14
    krylov: str = "gmres"  # 'gmres' | 'bicgstab' | 'cg' (the last two capped at max_restarts iterations)
    orth: str = "cgs2"  # GMRES Gram-Schmidt: 'cgs2' or 'dcgs2' (second pass delayed one step)
    precond: str = "none"  # 'none' | 'cslp' (Maxwell-Kerr, GMRES only: right preconditioning)
    store: str | None = None  # GMRES basis storage: None (FP64) or 'fp16' (see oracle.gmres)

    @classmethod
    def for_precision(cls, precision: str, **kw) -> "NewtonOptions":
        """Tolerances per precision (paper Section 3.3): FP64 1e-6 / 1e-8, FP32 1e-4 / 1e-6."""
        if precision == "f64":
            base = dict(tol_newton=1e-6, tol_krylov=1e-8, eps_mach=EPS_MACH["f64"], breakdown_tol=1e-14)
        else:
            base = dict(tol_newton=1e-4, tol_krylov=1e-6, eps_mach=EPS_MACH[precision], breakdown_tol=1e-6)
        base.update(kw)
        return cls(**base)


@dataclass
class NewtonInfo:
    status: str = NOT_CONVERGED
    converged: bool = False
    newton_iters: int = 0
    krylov_iters: int = 0
    restarts: int = 0
    ls_backtracks: int = 0
    ls_failures: int = 0
    rel_res: list = field(default_factory=list)  # rho_k = ||F(x_k)|| / ||F(x_0)||, k = 0..
    alphas: list = field(default_factory=list)
    lin_iters: list = field(default_factory=list)
    iterates: list = field(default_factory=list)  # x_k (when record=True)
    f0_norm: float = 0.0


def newton_solve(p: Problem, x_prev: np.ndarray, opts: NewtonOptions, source=None,
                 x0: np.ndarray | None = None, record: bool = False, perm: np.ndarray | None = None):
    """Solve F(x; x*) = 0 starting from x0 (default x* = x_prev); returns (x, NewtonInfo).

    ``perm`` (a permutation of the unknowns, test use) runs the same method on the
    reordered system P F(P^T y) = 0: the Krylov solve sees P J P^T and -P F, and the merit
    norms are taken over P F.  In exact arithmetic nothing changes; in floating point every
    dot product and norm is summed in another order, which measures how much the iterates
    depend on summation order alone."""
    if perm is None:
        def fwd(v):
            return v

        bwd = fwd
    else:
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm))

        def fwd(v):  # P v
            return v[perm]

        def bwd(y):  # P^T y
            return y[inv]

    def merit(F):
        return float(np.linalg.norm(fwd(F)))

    x = (x_prev if x0 is None else x0).astype(np.float64).copy()
    info = NewtonInfo()
    F = residual(p, x, x_prev, source)
    n0 = merit(F)
    info.f0_norm = n0
    fk = n0
    if record:
        info.iterates.append(x.copy())
    k = 0
    while True:
        if not math.isfinite(fk):
            info.status = NONFINITE
            return x, info
        rho = fk / n0 if n0 > 0.0 else 0.0
        info.rel_res.append(rho)
        if rho < opts.tol_newton:
            info.status = OK
            info.converged = True
            return x, info
        if k == opts.max_newton:
            info.status = NOT_CONVERGED
            return x, info

        if opts.mode == "ad":
            def jv(v, _x=x):
                return jvp_ad(p, _x, v, x_prev, source)[1]
        else:
            Fx = F

            def jv(v, _x=x, _F=Fx):
                eps = opts.fd_eps if opts.fd_eps > 0.0 else fd_step(opts.eps_rule, opts.eps_mach, _x, v)
                return jvp_fd(p, _x, v, eps, x_prev, source, Fx=_F)

        def matvec(y, _jv=jv):  # the Krylov solver's operator (P J P^T; J itself without perm)
            return fwd(_jv(bwd(y)))

        rhs = -fwd(F)
        if opts.precond == "cslp":
            # right preconditioning (Appendix A.4): GMRES on J M^{-1}, dx = M^{-1} z
            if opts.krylov != "gmres":
                raise ValueError("the CSLP preconditioner is applied with GMRES")

            def minv(v, _x=x):
                return cslp_solve(p, _x, v)

            def pmatvec(z, _mv=matvec, _minv=minv):
                return _mv(fwd(_minv(bwd(z))))

            z, ginfo = gm.gmres(pmatvec, rhs, m=opts.m, tol=opts.tol_krylov, max_restarts=opts.max_restarts,
                                breakdown_tol=opts.breakdown_tol, orth=opts.orth, store=opts.store)
            dx = minv(bwd(z))
            info.restarts += ginfo.cycles
        elif opts.precond != "none":
            raise ValueError(opts.precond)
        elif opts.krylov == "bicgstab":
            dy, ginfo = bicgstab(matvec, rhs, tol=opts.tol_krylov, maxiter=opts.max_restarts)
            dx = bwd(dy)
        elif opts.krylov == "cg":
            dy, ginfo = cg(matvec, rhs, tol=opts.tol_krylov, maxiter=opts.max_restarts)
            dx = bwd(dy)
        else:
            dy, ginfo = gm.gmres(matvec, rhs, m=opts.m, tol=opts.tol_krylov,
                                 max_restarts=opts.max_restarts, breakdown_tol=opts.breakdown_tol, orth=opts.orth,
                                 store=opts.store)
            dx = bwd(dy)
            info.restarts += ginfo.cycles
        info.krylov_iters += ginfo.iters
        info.lin_iters.append(ginfo.iters)
        if ginfo.nonfinite:
            info.status = NONFINITE
            return x, info

        alpha = 1.0
        accepted = False
        for t in range(opts.ls_max_backtracks + 1):
            xt = x + alpha * dx
            Ft = residual(p, xt, x_prev, source)
            ft = merit(Ft)
            if math.isfinite(ft) and ft <= (1.0 - opts.ls_c * alpha) * fk:
                accepted = True
                break
            if t < opts.ls_max_backtracks:
                alpha *= 0.5
                info.ls_backtracks += 1
        if not accepted:
            info.ls_failures += 1
        info.alphas.append(alpha)
        x, F, fk = xt, Ft, ft
        k += 1
        info.newton_iters = k
        if record:
            info.iterates.append(x.copy())


def step_failed(info: NewtonInfo, tol_newton: float) -> bool:
    """A time step fails if its final relative residual is above 100 tol_Newton or non-finite."""
    if info.status == NONFINITE or not info.rel_res:
        return True
    return not (info.rel_res[-1] <= 100.0 * tol_newton)


def run_failed(step_infos: list, tol_newton: float) -> bool:
    """A multi-step run fails when more than 20% of its steps fail, or on a non-finite step."""
    if any(i.status == NONFINITE for i in step_infos):
        return True
    bad = sum(step_failed(i, tol_newton) for i in step_infos)
    return bad > 0.2 * len(step_infos)
