"""Restarted GMRES(m) with CGS2 Arnoldi and Givens rotations (oracle).

The Krylov method of the paper's Section 2 (minimal residual over the Krylov
space K_m = span{r0, J r0, ..., J^{m-1} r0}, restarted) in its classical form:

* initial guess x0 = 0; the tolerance is relative to ||rhs||;
* each restart cycle starts from the true residual r = rhs - J x and stops the
  whole solve when ||r|| <= tol ||rhs||; at most ``max_restarts`` cycles (the
  paper's "maximum Krylov iteration count" counts restart cycles);
* Arnoldi step: w = J v_j, classical Gram-Schmidt applied twice
  (h = V^T w, w -= V h, h2 = V^T w, w -= V h2, column = h + h2),
  H[j+1, j] = ||w||;
* the Hessenberg column is reduced by the previous Givens rotations, a new
  rotation zeroes H[j+1, j] (c = a/r, s = b/r, r = hypot(a, b); (1, 0) when
  b = 0) and g is rotated; |g[j+1]| is the residual estimate;
* the cycle ends when |g[j+1]| <= tol ||rhs||, on a happy breakdown
  (||w|| <= breakdown_tol * ||J v_j||) or after m steps; then R y = g is
  back-substituted and x += V y.

``orth="dcgs2"`` selects the same Arnoldi process with the second
Gram-Schmidt pass delayed by one step (the low-synchronization form the
paper's GPU bottleneck discussion motivates; the paper fixes no variant).
Step j takes the once-orthogonalized vector u left by step j-1 and

* completes column j-1: a = V^T u, beta = sqrt(u.u - a.a) (the norm of the
  reorthogonalized vector), H[:j, j-1] += a, H[j, j-1] = beta, then the Givens
  update and the stop tests exactly as above;
* with u^ = u / beta and a^ = a / beta, the new basis vector is
  v_j = u^ - V a^, and the product w = J u^ stands in for J v_j through the
  Arnoldi relation J v_j = w - V_{j+1} (H a^);
* projects once: with b = V^T w and d = u^.w, h_i = b_i - (H a^)_i (i < j),
  gamma = d - a^.b, h_j = gamma - (H a^)_j, and the next pending vector is
  w - sum_i ((H a^)_i + h_i - gamma a^_i) v_i - gamma u^ (= J v_j - V h).

In exact arithmetic both forms give the same basis and Hessenberg matrix;
the delayed form reads the basis twice per step instead of three times.
After the last step the pending vector completes the last column.

``store="fp16"`` keeps the basis as a reduced-precision store would (the
paper's reduced-precision discussion; the storage format is this package's
reading): every vector written to the basis is rounded to binary16 after
scaling by a power of two that brings its typical entry near 1 (the scale
changes no significand for entries in binary16's normal range).  What is
written: r (then v_0 = stored r / ||r||, the norm of r before rounding),
with CGS2 each new w (v_{j+1} = stored w / ||w||), with DCGS2 each pending
u (its second pass and norm are taken over the stored u) and each v_j.
Everything else stays in FP64.

"Krylov iterations" counts Arnoldi steps.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresInfo:
    converged: bool = False
    iters: int = 0  # Arnoldi steps over all cycles
    cycles: int = 0  # restart cycles run
    nonfinite: bool = False
    breakdowns: int = 0
    true_res: list = field(default_factory=list)  # ||rhs - J x|| at the top of each cycle
    est_res: list = field(default_factory=list)  # |g[j+1]| after every Arnoldi step
    last_V: list | None = None  # basis of the last cycle (when record=True)
    last_H: np.ndarray | None = None  # unrotated Hessenberg of the last cycle
    last_k: int = 0


def givens(a: float, b: float) -> tuple[float, float]:
    """Rotation (c, s) with [c s; -s c] [a; b] = [r; 0]."""
    if b == 0.0:
        return 1.0, 0.0
    r = math.hypot(a, b)
    return a / r, b / r


def back_substitute(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve the upper-triangular system R y = g."""
    k = g.shape[0]
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        s = g[i]
        for l in range(i + 1, k):
            s -= R[i, l] * y[l]
        y[i] = s / R[i, i]
    return y


def store_fp16(v: np.ndarray) -> np.ndarray:
    """v as held by an FP16 store: rounded to binary16 (nearest even) after
    scaling by 2^-round(log2(||v|| / sqrt(n))), returned unscaled in FP64."""
    nrm = float(np.linalg.norm(v))
    if not (nrm > 0.0 and math.isfinite(nrm)):
        return v.copy()
    sig = 2.0 ** -round(math.log2(nrm / math.sqrt(v.shape[0])))
    return (v * sig).astype(np.float16).astype(np.float64) / sig


def _store_fn(store):
    if store is None:
        return lambda v: v
    if store == "fp16":
        return store_fp16
    raise ValueError(store)


def gmres(matvec, rhs: np.ndarray, m: int = 30, tol: float = 1e-8, max_restarts: int = 100,
          breakdown_tol: float = 1e-14, record: bool = False, orth: str = "cgs2", store: str | None = None):
    """Solve J x = rhs; returns (x, GmresInfo).  orth: 'cgs2' or 'dcgs2';
    store: None (FP64 basis) or 'fp16' (basis rounded as stored in binary16)."""
    st = _store_fn(store)
    if orth == "dcgs2":
        return _gmres_dcgs2(matvec, rhs, m, tol, max_restarts, breakdown_tol, record, st)
    if orth != "cgs2":
        raise ValueError(orth)
    n = rhs.shape[0]
    x = np.zeros(n)
    info = GmresInfo()
    bnorm = float(np.linalg.norm(rhs))
    if not math.isfinite(bnorm):
        info.nonfinite = True
        return x, info
    if bnorm == 0.0:
        info.converged = True
        info.true_res.append(0.0)
        return x, info
    target = tol * bnorm
    for cycle in range(max_restarts + 1):
        r = rhs.copy() if cycle == 0 else rhs - matvec(x)
        beta = float(np.linalg.norm(r))
        info.true_res.append(beta)
        if not math.isfinite(beta):
            info.nonfinite = True
            return x, info
        if beta <= target:
            info.converged = True
            return x, info
        if cycle == max_restarts:
            return x, info
        info.cycles += 1
        V = [st(r) / beta]
        H = np.zeros((m + 1, m))  # rotated in place
        Hraw = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k = 0
        for j in range(m):
            w = matvec(V[j])
            jv_norm = float(np.linalg.norm(w))
            # classical Gram-Schmidt, twice
            h = np.array([np.dot(V[i], w) for i in range(j + 1)])
            for i in range(j + 1):
                w = w - h[i] * V[i]
            h2 = np.array([np.dot(V[i], w) for i in range(j + 1)])
            for i in range(j + 1):
                w = w - h2[i] * V[i]
            col = h + h2
            wnorm = float(np.linalg.norm(w))
            Hraw[: j + 1, j] = col
            Hraw[j + 1, j] = wnorm
            H[: j + 1, j] = col
            H[j + 1, j] = wnorm
            if not (np.all(np.isfinite(col)) and math.isfinite(wnorm)):
                info.nonfinite = True
                return x, info
            # previous rotations
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            info.iters += 1
            info.est_res.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= target:
                break
            if wnorm <= breakdown_tol * jv_norm:
                info.breakdowns += 1
                break
            V.append(st(w) / wnorm)
        y = back_substitute(H[:k, :k], g[:k])
        for i in range(k):
            x = x + y[i] * V[i]
        if record:
            info.last_V = [vv.copy() for vv in V]
            info.last_H = Hraw[: k + 1, :k].copy()
            info.last_k = k
    return x, info


def _rotate_column(H, cs, sn, g, j):
    """Apply the previous rotations to column j, form rotation j, update g."""
    for i in range(j):
        t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
        H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
        H[i, j] = t
    cs[j], sn[j] = givens(H[j, j], H[j + 1, j])
    H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
    H[j + 1, j] = 0.0
    g[j + 1] = -sn[j] * g[j]
    g[j] = cs[j] * g[j]


def _gmres_dcgs2(matvec, rhs, m, tol, max_restarts, breakdown_tol, record, st):
    n = rhs.shape[0]
    x = np.zeros(n)
    info = GmresInfo()
    bnorm = float(np.linalg.norm(rhs))
    if not math.isfinite(bnorm):
        info.nonfinite = True
        return x, info
    if bnorm == 0.0:
        info.converged = True
        info.true_res.append(0.0)
        return x, info
    target = tol * bnorm
    for cycle in range(max_restarts + 1):
        r = rhs.copy() if cycle == 0 else rhs - matvec(x)
        beta0 = float(np.linalg.norm(r))
        info.true_res.append(beta0)
        if not math.isfinite(beta0):
            info.nonfinite = True
            return x, info
        if beta0 <= target:
            info.converged = True
            return x, info
        if cycle == max_restarts:
            return x, info
        info.cycles += 1
        V = [st(r) / beta0]
        H = np.zeros((m + 1, m))  # rotated in place
        Hraw = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta0
        jv_norms = []
        u = None  # once-orthogonalized vector pending for the column before it

        def complete(col, u):
            """Second pass for the pending vector; completes column col. Returns (a, beta, stop)."""
            a = np.array([np.dot(V[i], u) for i in range(col + 1)])
            c = float(np.dot(u, u))
            b2 = c - float(np.dot(a, a))
            beta = math.sqrt(b2) if b2 > 0.0 else 0.0
            Hraw[: col + 1, col] += a
            Hraw[col + 1, col] = beta
            H[: col + 2, col] = Hraw[: col + 2, col]
            if not (np.all(np.isfinite(Hraw[: col + 2, col])) and math.isfinite(c)):
                return a, beta, "nonfinite"
            _rotate_column(H, cs, sn, g, col)
            info.iters += 1
            info.est_res.append(abs(g[col + 1]))
            if abs(g[col + 1]) <= target:
                return a, beta, "converged"
            if beta <= breakdown_tol * jv_norms[col]:
                info.breakdowns += 1
                return a, beta, "breakdown"
            return a, beta, None

        k = 0
        stopped = False
        for j in range(m):
            if j == 0:
                uh = V[0]
                ah = np.zeros(0)
            else:
                a, beta, stop = complete(j - 1, u)
                k = j
                if stop == "nonfinite":
                    info.nonfinite = True
                    return x, info
                if stop is not None:
                    stopped = True
                    break
                uh = u / beta
                ah = a / beta
            w = matvec(uh)
            jv_norms.append(float(np.linalg.norm(w)))
            b = np.array([np.dot(V[i], w) for i in range(j)])
            d = float(np.dot(uh, w))
            if j == 0:
                h = np.array([d])
                u = st(w - d * V[0])
            else:
                Ha = Hraw[: j + 1, :j] @ ah  # J v_j = w - sum_i Ha_i v_i
                gamma = d - float(np.dot(ah, b))
                h = np.zeros(j + 1)
                h[:j] = b - Ha[:j]
                h[j] = gamma - Ha[j]
                vj = uh.copy()
                for i in range(j):
                    vj = vj - ah[i] * V[i]
                u = w - gamma * uh
                for i in range(j):
                    u = u - (Ha[i] + h[i] - gamma * ah[i]) * V[i]
                u = st(u)
                V.append(st(vj))
            Hraw[: j + 1, j] = h
        if not stopped:
            a, beta, stop = complete(m - 1, u)
            k = m
            if stop == "nonfinite":
                info.nonfinite = True
                return x, info
            if stop is None and beta > 0.0:
                V.append((u - sum(a[i] * V[i] for i in range(m))) / beta)
        y = back_substitute(H[:k, :k], g[:k])
        for i in range(k):
            x = x + y[i] * V[i]
        if record:
            info.last_V = [vv.copy() for vv in V]
            info.last_H = Hraw[: k + 1, :k].copy()
            info.last_k = k
    return x, info
