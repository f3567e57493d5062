"""Shared helpers of the GPU parity tests: seeded cases and tensor plumbing.

Inputs come from the ``workloads`` generators only; expected values come from
the oracle only.
"""

from __future__ import annotations

import numpy as np

import workloads as W


def torch_mod():
    import torch

    return torch


def gpu_available() -> bool:
    try:
        torch = torch_mod()
        return torch.cuda.is_available()
    except Exception:
        return False


def dev(a, dtype):
    torch = torch_mod()
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.double().cpu().numpy()


def wdtype(prec):
    torch = torch_mod()
    return torch.float64 if prec == "f64" else torch.float32


def case(kind: str, nx: int, ny: int | None = None, seed: int = 0):
    """(spec, x_prev, source) of a small problem of the given kind and grid."""
    if kind == "burgers1d":
        spec = W.burgers1d_spec(nx)
        return spec, W.burgers1d_initial(nx, seed), None
    ny = nx if ny is None else ny
    if kind == "grayscott":
        spec = dict(W.grayscott_spec(nx), ny=ny)
        return spec, W.grayscott_initial(nx, seed, ny=ny, side_frac=1 / 8, patches=6), None
    if kind == "burgers2d":
        spec = dict(W.burgers2d_spec(nx, nu=0.02, dt=0.01), ny=ny, hy=2 * np.pi / ny)
        u = W.random_vector(2 * nx * ny, seed, 0.5)
        return spec, u, None
    if kind == "rd2d":
        spec = W.rd2d_spec(nx, ny=ny)
        return spec, W.rd2d_initial(nx, seed, ny=ny), None
    if kind == "maxwell":
        spec = W.maxwell_spec(nx, ny=ny)
        return spec, np.zeros(4 * nx * ny), W.maxwell_source(nx, ny=ny)
    if kind == "suolson":
        x0, src = W.suolson_initial(nx, seed, ny=ny)
        return W.suolson_spec(nx, ny=ny), x0, src
    if kind == "suolson1d":
        # periodic rows; a y-dependent start so that the row wrap matters
        x0, src = W.suolson_box_initial(nx, ny=ny)
        x0 = x0 + 0.1 * W.random_vector(2 * nx * ny, seed + 3)
        m = np.zeros((ny, nx))
        m[:, 1:-1] = 1.0
        return W.suolson_spec(nx, ny=ny, periodic_y=True), x0 * np.tile(m.ravel(), 2), src
    if kind == "kerr":
        spec = dict(W.kerr_spec(nx, chi3=0.3, cells_per_wavelength=8.0, eps_im=0.05), ny=ny)
        src = W.kerr_gaussian_source(nx, amp=1.0, sigma=max(1.0, nx / 8), ny=ny)
        return spec, np.zeros(2 * nx * ny), src
    raise KeyError(kind)


def rel_err(got, ref, x=None):
    scale = max(1.0, float(np.abs(ref).max()))
    if x is not None:
        scale = max(scale, float(np.abs(x).max()))
    return float(np.abs(got - ref).max()) / scale


def _node_planes(spec, a):
    """View of a state vector as (fields, ny, nx) planes (Kerr's interleaved pairs as two planes)."""
    nx, ny = spec["nx"], spec["ny"]
    if spec["kind"] == "kerr":
        return a.reshape(ny, nx, 2).transpose(2, 0, 1)
    return a.reshape(-1, ny, nx)


def local_scale(spec, *arrays):
    """Per element: the largest |value| of any of `arrays` over every field of
    the node's 3 x 3 neighbourhood (the operands a stencil output at that node
    is formed from), laid out like a state vector."""
    from scipy.ndimage import maximum_filter

    nx, ny = spec["nx"], spec["ny"]
    nf = None
    s = None
    for a in arrays:
        pl = np.abs(_node_planes(spec, np.asarray(a, dtype=np.float64)))
        nf = pl.shape[0]
        m = maximum_filter(pl.max(axis=0), size=3, mode="wrap")
        s = m if s is None else np.maximum(s, m)
    if spec["kind"] == "kerr":
        return np.repeat(s.reshape(-1), 2)
    return np.tile(s.reshape(-1), nf)


def elem_err(got, ref, scale):
    """max_i |got_i - ref_i| / max(|ref_i|, scale_i): a per-element relative
    error, so that a mistake confined to small entries is not hidden by the
    largest ones (scale_i, from local_scale, keeps nodes where the output
    cancels to near zero from demanding more than their operands' rounding)."""
    den = np.maximum(np.abs(ref), scale)
    den = np.where(den > 0.0, den, 1.0)
    return float((np.abs(got - ref) / den).max())
