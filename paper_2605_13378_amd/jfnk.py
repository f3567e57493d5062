"""ctypes binding of libjfnk.so (include/jfnk.h).

Argument marshalling only: tensors are checked (device, dtype, length,
contiguity) and their device pointers handed to the C ABI; every step of the
method runs in the library's HIP kernels.  PyTorch provides device memory and
the current HIP stream.  There is no fallback: if the library is not built or
cannot be loaded, every call raises.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjfnk.so")

MAX_ITERS = 64

PROBLEM_IDS = {"burgers1d": 0, "burgers2d": 1, "grayscott": 2, "kerr": 3, "rd2d": 4, "suolson": 5, "maxwell": 6}
PRECISIONS = {"f64": 0, "f32": 1, "f16s": 2}
MODES = {"ad": 0, "fd": 1}
EPS_RULES = {"paper": 0, "normalized": 1}
ENGINES = {"auto": 0, "multi": 1, "single": 2, "graph": 3}
KRYLOV = {"gmres": 0, "bicgstab": 1, "cg": 2}
ORTH = {"cgs2": 0, "dcgs2": 1}
PRECOND = {"none": 0, "cslp": 1}
STATUS = {0: "ok", 1: "invalid argument", 2: "out of memory", 3: "hip error", 4: "nonfinite",
          5: "breakdown", 6: "not_converged"}
PROFILE_KERNELS = {"residual": 0, "jvp_ad": 1, "jvp_fd": 2, "cgs_a": 3, "cgs_b": 4, "cgs_c": 5, "vy": 6,
                   "cycle_start": 7, "newton_trial": 8, "fused_solve": 9, "bicgstab": 10, "cg": 11, "dcgs_update": 12}


class Problem(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double),
                ("dt", ctypes.c_double), ("theta", ctypes.c_double),
                ("p", ctypes.c_double * 8)]


class Options(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int), ("max_restarts", ctypes.c_int), ("max_newton", ctypes.c_int),
                ("ls_max_backtracks", ctypes.c_int),
                ("tol_krylov", ctypes.c_double), ("tol_newton", ctypes.c_double), ("ls_c", ctypes.c_double),
                ("fd_eps", ctypes.c_double), ("breakdown_tol", ctypes.c_double),
                ("mode", ctypes.c_int), ("eps_rule", ctypes.c_int),
                ("history", ctypes.c_void_p), ("engine", ctypes.c_int), ("krylov", ctypes.c_int),
                ("orth", ctypes.c_int), ("precond", ctypes.c_int)]


class Info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("converged", ctypes.c_int), ("newton_iters", ctypes.c_int),
                ("krylov_iters", ctypes.c_int), ("restarts", ctypes.c_int), ("ls_backtracks", ctypes.c_int),
                ("ls_failures", ctypes.c_int), ("lin_iters", ctypes.c_int * MAX_ITERS),
                ("rel_res", ctypes.c_double * (MAX_ITERS + 1)), ("alpha", ctypes.c_double * MAX_ITERS),
                ("f0_norm", ctypes.c_double), ("final_res", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self) -> dict:
        k = self.newton_iters
        return dict(status=STATUS.get(self.status, str(self.status)), converged=bool(self.converged),
                    newton_iters=k, krylov_iters=self.krylov_iters, restarts=self.restarts,
                    ls_backtracks=self.ls_backtracks, ls_failures=self.ls_failures,
                    lin_iters=list(self.lin_iters[:k]), rel_res=list(self.rel_res[: k + 1]),
                    alphas=list(self.alpha[:k]), f0_norm=self.f0_norm, final_res=self.final_res,
                    seconds=self.seconds)


class BatchConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int), ("precision", ctypes.c_int),
                ("m", ctypes.c_int), ("keep_workspaces", ctypes.c_int)]


class BatchStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong), ("failed", ctypes.c_longlong),
                ("workspaces_created", ctypes.c_longlong), ("workspaces_released", ctypes.c_longlong),
                ("max_running", ctypes.c_int), ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("frees_while_running", ctypes.c_longlong)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class JfnkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None

# (name, restype, argtypes)
_SIGNATURES = [
    ("jfnk_create", ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_void_p)]),
    ("jfnk_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("jfnk_footprint_bytes", ctypes.c_size_t, [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_int]),
    ("jfnk_problem_size", ctypes.c_size_t, [ctypes.POINTER(Problem)]),
    ("jfnk_set_previous", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("jfnk_residual", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("jfnk_jvp", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int]),
    ("jfnk_gmres", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_int, ctypes.POINTER(Info)]),
    ("jfnk_gmres_hessenberg", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                             ctypes.POINTER(ctypes.c_int)]),
    ("jfnk_bicgstab", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                     ctypes.POINTER(Info)]),
    ("jfnk_cg", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                               ctypes.POINTER(Info)]),
    ("jfnk_newton_solve", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Options),
                                         ctypes.POINTER(Info)]),
    ("jfnk_newton_solve_noalloc", ctypes.c_int, [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_void_p,
                                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(Options),
                                                 ctypes.POINTER(Info), ctypes.c_void_p]),
    ("jfnk_cycle_graphs", ctypes.c_int, [ctypes.c_void_p]),
    ("jfnk_frequency_sweep", ctypes.c_int, [ctypes.POINTER(Problem), ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                            ctypes.c_int, ctypes.POINTER(Options), ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.POINTER(Info), ctypes.POINTER(ctypes.c_int)]),
    ("jfnk_default_options", None, [ctypes.c_int, ctypes.POINTER(Options)]),
    ("jfnk_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("jfnk_last_error", ctypes.c_char_p, [ctypes.c_void_p]),
    ("jfnk_profile_enable", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("jfnk_profile_read", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    ("jfnk_profile_reset", ctypes.c_int, [ctypes.c_void_p]),
    ("jfnk_set_stream", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    ("jfnk_set_orthogonalization", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("jfnk_set_preconditioner", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("jfnk_batch_create", ctypes.c_int, [ctypes.POINTER(BatchConfig), ctypes.POINTER(ctypes.c_void_p)]),
    ("jfnk_batch_destroy", ctypes.c_int, [ctypes.c_void_p]),
    ("jfnk_batch_submit", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.c_void_p,
                                         ctypes.c_void_p, ctypes.POINTER(Options),
                                         ctypes.POINTER(ctypes.c_longlong)]),
    ("jfnk_batch_poll", ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong]),
    ("jfnk_batch_wait", ctypes.c_int, [ctypes.c_void_p, ctypes.c_longlong, ctypes.c_void_p,
                                       ctypes.POINTER(Info), ctypes.c_void_p]),
    ("jfnk_batch_clock", ctypes.c_double, [ctypes.c_void_p]),
    ("jfnk_batch_get_stats", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(BatchStats)]),
]


def lib() -> ctypes.CDLL:
    """Load libjfnk.so (built in place); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2605_13378_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, res, args in _SIGNATURES:
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def exported_symbols() -> list[str]:
    return [name for name, _, _ in _SIGNATURES]


def make_problem(spec: dict) -> Problem:
    """Problem struct from a workload spec dict (see the workloads module)."""
    kind = spec["kind"]
    p = Problem()
    p.id = PROBLEM_IDS[kind]
    p.nx = int(spec["nx"])
    p.ny = int(spec.get("ny", 1))
    p.hx = float(spec["hx"])
    p.hy = float(spec.get("hy", 1.0))
    p.dt = float(spec.get("dt", 0.0))
    p.theta = float(spec.get("theta", 1.0))
    if kind in ("burgers1d", "burgers2d"):
        vals = [spec["nu"]]
    elif kind == "grayscott":
        vals = [spec["D"], spec["Dv"], spec["F"], spec["k"]]
    elif kind == "rd2d":
        vals = [spec["D"]]
    elif kind == "suolson":
        vals = [spec["xi"], 1.0 if spec.get("periodic_y") else 0.0]
    elif kind == "maxwell":
        vals = [spec["k0"], spec["eps_im"], spec["chi3"]]
    else:
        vals = [spec["k0"], spec.get("eps_re", 1.0), spec.get("eps_im", 0.0), spec["chi3"]]
    for i, v in enumerate(vals):
        p.p[i] = float(v)
    return p


def default_options(precision: str = "f64", **kw) -> Options:
    o = Options()
    lib().jfnk_default_options(PRECISIONS[precision], ctypes.byref(o))
    for key, val in kw.items():
        if key == "mode":
            val = MODES[val]
        elif key == "eps_rule":
            val = EPS_RULES[val]
        elif key == "engine":
            val = ENGINES[val]
        elif key == "krylov":
            val = KRYLOV[val]
        elif key == "orth":
            val = ORTH[val]
        elif key == "precond":
            val = PRECOND[val]
        elif key == "history":
            val = None if val is None else val.data_ptr()
        setattr(o, key, val)
    return o


def footprint_bytes(spec: dict, precision: str = "f64", m: int = 30) -> int:
    p = make_problem(spec)
    return int(lib().jfnk_footprint_bytes(ctypes.byref(p), PRECISIONS[precision], m))


def problem_size(spec: dict) -> int:
    p = make_problem(spec)
    return int(lib().jfnk_problem_size(ctypes.byref(p)))


class Solver:
    """One problem shape and precision on the current HIP stream."""

    def __init__(self, spec: dict, precision: str = "f64", m: int = 30, stream=None):
        import torch

        self._torch = torch
        self.spec = dict(spec)
        self.precision = precision
        self.m = m
        self.n = problem_size(spec)
        self.wdtype = torch.float64 if precision == "f64" else torch.float32
        st = torch.cuda.current_stream() if stream is None else stream
        self.stream = st
        prob = make_problem(spec)
        h = ctypes.c_void_p()
        rc = lib().jfnk_create(ctypes.byref(prob), PRECISIONS[precision], m, ctypes.c_void_p(st.cuda_stream),
                               ctypes.byref(h))
        if rc != 0:
            raise JfnkError(rc, lib().jfnk_last_error(None).decode())
        self._h = h

    # -- helpers -----------------------------------------------------------
    def _check(self, rc: int, allowed=(0,)):
        if rc not in allowed:
            raise JfnkError(rc, lib().jfnk_last_error(self._h).decode())
        return rc

    def _vec(self, t, dtype, name):
        torch = self._torch
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
        if t.numel() != self.n or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {self.n} elements")
        return t

    def _new(self, dtype=None):
        return self._torch.empty(self.n, dtype=dtype or self.wdtype, device="cuda")

    # -- the C ABI calls -------------------------------------------------------
    def set_previous(self, x_prev, source=None):
        torch = self._torch
        self._prev = self._vec(x_prev, torch.float64, "x_prev") if x_prev is not None else None
        self._src = self._vec(source, torch.float64, "source")
        self._check(lib().jfnk_set_previous(self._h, None if self._prev is None else self._prev.data_ptr(),
                                            None if self._src is None else self._src.data_ptr()))

    def residual(self, x, out=None):
        x = self._vec(x, self.wdtype, "x")
        out = self._new() if out is None else self._vec(out, self.wdtype, "out")
        self._check(lib().jfnk_residual(self._h, x.data_ptr(), out.data_ptr()))
        return out

    def jvp(self, x, v, mode="ad", eps=0.0, eps_rule="paper", want_F=False, out=None):
        x = self._vec(x, self.wdtype, "x")
        v = self._vec(v, self.wdtype, "v")
        jv = self._new() if out is None else self._vec(out, self.wdtype, "out")
        F = self._new() if (want_F and mode == "ad") else None
        self._check(lib().jfnk_jvp(self._h, x.data_ptr(), v.data_ptr(), jv.data_ptr(),
                                   None if F is None else F.data_ptr(), MODES[mode], float(eps),
                                   EPS_RULES[eps_rule]))
        return (jv, F) if want_F else jv

    def cycle_graphs(self) -> int:
        """Captured GMRES-cycle graphs this solver holds (MULTI_KERNEL_GRAPH engine)."""
        return int(lib().jfnk_cycle_graphs(self._h))

    def set_orthogonalization(self, orth: str):
        """Gram-Schmidt form of later gmres() calls: 'cgs2' or 'dcgs2' (the default)."""
        self._check(lib().jfnk_set_orthogonalization(self._h, ORTH[orth]))

    def set_preconditioner(self, precond: str):
        """Right preconditioner of later gmres() calls: 'none' (default) or 'cslp' (Maxwell-Kerr, Helmholtz-Kerr)."""
        self._check(lib().jfnk_set_preconditioner(self._h, PRECOND[precond]))

    def gmres(self, x, rhs, m=None, tol=1e-8, max_restarts=100, mode="ad", eps=0.0, eps_rule="paper"):
        x = self._vec(x, self.wdtype, "x")
        rhs = self._vec(rhs, self.wdtype, "rhs")
        dx = self._new()
        info = Info()
        self._check(lib().jfnk_gmres(self._h, x.data_ptr(), rhs.data_ptr(), dx.data_ptr(),
                                     self.m if m is None else m, tol, max_restarts, MODES[mode], float(eps),
                                     EPS_RULES[eps_rule], ctypes.byref(info)), allowed=(0, 4))
        d = info.as_dict()
        d["converged"] = bool(info.converged)
        return dx, d

    def gmres_hessenberg(self):
        """Unrotated (k + 1) x k Hessenberg matrix of the last GMRES cycle (numpy, FP64)."""
        import numpy as np

        k = ctypes.c_int(0)
        ld = self.m + 1
        H = np.zeros((self.m, ld), dtype=np.float64)  # column-major: row l of this array is column l
        self._check(lib().jfnk_gmres_hessenberg(self._h, H.ctypes.data, ld, ctypes.byref(k)))
        kk = k.value
        return np.ascontiguousarray(H[:kk, : kk + 1].T)

    def bicgstab(self, x, rhs, tol=1e-8, max_iters=100, mode="ad", eps=0.0, eps_rule="paper"):
        """BiCGSTAB solve of J(x) dx = rhs; returns (dx, info dict with 'breakdown')."""
        return self._short_recurrence(lib().jfnk_bicgstab, x, rhs, tol, max_iters, mode, eps, eps_rule)

    def cg(self, x, rhs, tol=1e-8, max_iters=100, mode="ad", eps=0.0, eps_rule="paper"):
        """Conjugate-gradient solve of J(x) dx = rhs (SPD J); returns (dx, info dict with 'breakdown')."""
        return self._short_recurrence(lib().jfnk_cg, x, rhs, tol, max_iters, mode, eps, eps_rule)

    def _short_recurrence(self, fn, x, rhs, tol, max_iters, mode, eps, eps_rule):
        x = self._vec(x, self.wdtype, "x")
        rhs = self._vec(rhs, self.wdtype, "rhs")
        dx = self._new()
        info = Info()
        rc = self._check(fn(self._h, x.data_ptr(), rhs.data_ptr(), dx.data_ptr(), float(tol), int(max_iters),
                            MODES[mode], float(eps), EPS_RULES[eps_rule], ctypes.byref(info)), allowed=(0, 4, 5))
        d = info.as_dict()
        d["converged"] = bool(info.converged)
        d["breakdown"] = rc == 5
        d["nonfinite"] = rc == 4
        return dx, d

    def newton_solve(self, x0, history: bool = False, **opts):
        torch = self._torch
        x = self._vec(x0, torch.float64, "x0").clone()
        hist = None
        if history:
            mn = opts.get("max_newton", 15)
            hist = torch.zeros((mn + 1) * self.n, dtype=torch.float64, device="cuda")
            opts["history"] = hist
        o = default_options(self.precision, **opts)
        if o.m > self.m:
            raise ValueError("options.m exceeds the solver's m")
        info = Info()
        # converged, non-finite and not-converged solves all report through info
        self._check(lib().jfnk_newton_solve(self._h, x.data_ptr(), ctypes.byref(o), ctypes.byref(info)),
                    allowed=(0, 4, 6))
        d = info.as_dict()
        if history:
            d["history"] = hist.view(-1, self.n)[: info.newton_iters + 1]
        return x, d

    # -- profiling ------------------------------------------------------------
    def profile(self, on: bool = True):
        self._check(lib().jfnk_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self):
        self._check(lib().jfnk_profile_reset(self._h))

    def profile_read(self) -> dict:
        out = {}
        for name, kid in PROFILE_KERNELS.items():
            n = ctypes.c_longlong()
            ms = ctypes.c_double()
            by = ctypes.c_double()
            self._check(lib().jfnk_profile_read(self._h, kid, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
            out[name] = dict(launches=n.value, ms=ms.value, bytes=by.value)
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().jfnk_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def newton_solve_noalloc(spec: dict, precision: str, x_prev, source, x_inout, history=None, stream=None,
                         **opts) -> dict:
    """jfnk_newton_solve_noalloc: the single-workgroup Newton solve with no
    solver handle and no device allocation.  x_prev, source (nullable) and
    x_inout (updated in place) are FP64 CUDA (HIP) tensors of the problem's
    length; history (nullable) an FP64 tensor of (max_newton + 1) * n entries
    the caller provides.  Returns the info dict; raises JfnkError on argument
    errors (jfnk_last_error(NULL) text)."""
    import torch

    n = problem_size(spec)
    for name, t in (("x_prev", x_prev), ("source", source), ("x_inout", x_inout), ("history", history)):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float64:
            raise TypeError(f"{name} must be an FP64 CUDA (HIP) tensor")
        if not t.is_contiguous() or (name != "history" and t.numel() != n):
            raise ValueError(f"{name} must be contiguous with {n} elements")
    if history is not None:
        opts["history"] = history
    o = default_options(precision, **opts)
    info = Info()
    prob = make_problem(spec)
    st = torch.cuda.current_stream() if stream is None else stream
    rc = lib().jfnk_newton_solve_noalloc(ctypes.byref(prob), PRECISIONS[precision],
                                         None if x_prev is None else x_prev.data_ptr(),
                                         None if source is None else source.data_ptr(), x_inout.data_ptr(),
                                         ctypes.byref(o), ctypes.byref(info), ctypes.c_void_p(st.cuda_stream))
    if rc not in (0, 4, 6):
        raise JfnkError(rc, lib().jfnk_last_error(None).decode())
    return info.as_dict()


def frequency_sweep(specs: list, sources: list, precision: str = "f64", stream=None, **opts):
    """jfnk_frequency_sweep: the problems of `specs` (one per frequency, in order)
    with their host FP64 sources (numpy, or None) by frequency continuation.
    Returns (fields: numpy array [count, n], infos: list of dicts, run_failed)."""
    import numpy as np
    import torch

    count = len(specs)
    n = problem_size(specs[0])
    probs = (Problem * count)(*[make_problem(sp) for sp in specs])
    srcs = [None if f is None else np.ascontiguousarray(f, dtype=np.float64) for f in sources]
    for f in srcs:
        if f is not None and f.size != n:
            raise ValueError(f"every source must have {n} entries")
    ptrs = (ctypes.c_void_p * count)(*[None if f is None else f.ctypes.data for f in srcs])
    fields = np.empty((count, n), dtype=np.float64)
    infos = (Info * count)()
    failed = ctypes.c_int(0)
    o = default_options(precision, **opts)
    st = torch.cuda.current_stream() if stream is None else stream
    rc = lib().jfnk_frequency_sweep(probs, ptrs, count, PRECISIONS[precision], ctypes.byref(o),
                                    ctypes.c_void_p(st.cuda_stream), fields.ctypes.data, infos, ctypes.byref(failed))
    if rc != 0:
        raise JfnkError(rc, lib().jfnk_last_error(None).decode())
    return fields, [i.as_dict() for i in infos], bool(failed.value)


class Batch:
    """Continuous batching of independent Newton solves (jfnk_batch_* calls).

    Requests carry host FP64 arrays (numpy); `submit` copies them and returns
    a ticket at once, `wait` blocks for the result.  The library's worker
    threads run admitted requests concurrently, each on its own HIP stream.
    """

    def __init__(self, precision: str = "f32", m: int = 30, max_slots: int = 4,
                 budget_bytes: int = 16 << 30, keep_workspaces: bool = True):
        self.precision = precision
        self.m = m
        cfg = BatchConfig(budget_bytes=int(budget_bytes), max_slots=int(max_slots),
                          precision=PRECISIONS[precision], m=int(m), keep_workspaces=1 if keep_workspaces else 0)
        h = ctypes.c_void_p()
        rc = lib().jfnk_batch_create(ctypes.byref(cfg), ctypes.byref(h))
        if rc != 0:
            raise JfnkError(rc, "jfnk_batch_create rejected the configuration")
        self._h = h
        self._n = {}

    def submit(self, spec: dict, x_prev, source=None, **opts) -> int:
        import numpy as np

        prob = make_problem(spec)
        n = problem_size(spec)
        xp = np.ascontiguousarray(x_prev, dtype=np.float64)
        if xp.size != n:
            raise ValueError(f"x_prev must have {n} entries")
        src = None if source is None else np.ascontiguousarray(source, dtype=np.float64)
        if src is not None and src.size != n:
            raise ValueError(f"source must have {n} entries")
        o = default_options(self.precision, **opts)
        if o.m > self.m:
            raise ValueError("options.m exceeds the batch's m")
        t = ctypes.c_longlong()
        rc = lib().jfnk_batch_submit(self._h, ctypes.byref(prob), xp.ctypes.data,
                                     None if src is None else src.ctypes.data, ctypes.byref(o), ctypes.byref(t))
        if rc != 0:
            raise JfnkError(rc, "jfnk_batch_submit rejected the request")
        self._n[t.value] = n
        return t.value

    def poll(self, ticket: int) -> bool:
        return lib().jfnk_batch_poll(self._h, ticket) == 1

    def wait(self, ticket: int):
        """(x, info dict with 'times' = (submit, start, finish) on the batch clock)."""
        import numpy as np

        n = self._n.pop(ticket)
        x = np.empty(n, dtype=np.float64)
        info = Info()
        times = (ctypes.c_double * 3)()
        rc = lib().jfnk_batch_wait(self._h, ticket, x.ctypes.data, ctypes.byref(info), times)
        d = info.as_dict()
        d["rc"] = rc
        d["times"] = (times[0], times[1], times[2])
        return x, d

    def clock(self) -> float:
        return float(lib().jfnk_batch_clock(self._h))

    def stats(self) -> dict:
        st = BatchStats()
        lib().jfnk_batch_get_stats(self._h, ctypes.byref(st))
        return st.as_dict()

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().jfnk_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
