"""The allocation-free Newton solve (jfnk_newton_solve_noalloc) against the
solver-handle solve on the same single-workgroup engine.

Both run the same kernels on the same constant part, so the iterates, the
per-step records and the final state must be bitwise equal.  Two calls in a
row share the static device workspace; the second is smaller than the first
(its entries beyond the second problem's length hold the first call's values,
which nothing may read).  Sizes beyond the workspace, FP16 storage and the
multi-kernel engine are rejected with a message.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, gpu_available, host, wdtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def _handle_solve(spec, prec, xp, src, **opts):
    from paper_2605_13378_amd import Solver

    s = Solver(spec, prec, m=opts.get("m", 30))
    s.set_previous(None if xp is None else dev(xp, wdtype("f64")), None if src is None else dev(src, wdtype("f64")))
    start = np.zeros(W.n_unknowns(spec)) if xp is None else xp
    x, info = s.newton_solve(dev(start, wdtype("f64")), history=True, engine="single", **opts)
    s.close()
    return host(x), info


def _noalloc_solve(spec, prec, xp, src, **opts):
    import torch

    from paper_2605_13378_amd import newton_solve_noalloc

    n = W.n_unknowns(spec)
    start = np.zeros(n) if xp is None else xp
    x = dev(start, torch.float64)
    mn = opts.get("max_newton", 15)
    hist = torch.zeros((mn + 1) * n, dtype=torch.float64, device="cuda")
    info = newton_solve_noalloc(spec, prec, None if xp is None else dev(xp, torch.float64),
                                None if src is None else dev(src, torch.float64), x, history=hist,
                                engine="single", **opts)
    torch.cuda.synchronize()
    return host(x), info, host(hist).reshape(mn + 1, n)[: info["newton_iters"] + 1]


def _kerr_case():
    spec = dict(W.kerr_spec(12, chi3=0.3, cells_per_wavelength=64.0, eps_im=0.05), ny=10)
    return spec, None, W.kerr_gaussian_source(12, amp=1.0, sigma=2.0, ny=10)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_noalloc_equals_handle_solve_two_calls(prec):
    calls = [case("grayscott", 16, 12), (W.burgers1d_spec(200), W.burgers1d_initial(200, 3), None)]
    if prec == "f64":
        calls.append(_kerr_case())
    sizes = []
    for spec, xp, src in calls:
        x_ref, ref = _handle_solve(spec, prec, xp, src)
        x, info, hist = _noalloc_solve(spec, prec, xp, src)
        sizes.append(W.n_unknowns(spec))
        assert ref["converged"] and info["converged"], (spec["kind"], info, ref)
        assert np.array_equal(x, x_ref), spec["kind"]
        assert np.array_equal(hist, host(ref["history"])), spec["kind"]
        for key in ("newton_iters", "krylov_iters", "restarts", "ls_backtracks", "rel_res", "lin_iters", "alphas",
                    "f0_norm", "status"):
            assert info[key] == ref[key], (spec["kind"], key, info[key], ref[key])
    assert sizes[1] < sizes[0]


def test_noalloc_rejections():
    import torch

    from paper_2605_13378_amd import JfnkError, newton_solve_noalloc

    spec, xp, src = case("grayscott", 64, 64)  # 8192 unknowns: above the static workspace
    x = dev(xp, torch.float64)
    with pytest.raises(JfnkError, match="4096 unknowns"):
        newton_solve_noalloc(spec, "f64", dev(xp, torch.float64), None, x, engine="single")
    spec, xp, src = case("grayscott", 16, 16)
    x = dev(xp, torch.float64)
    with pytest.raises(JfnkError, match="FP64 or FP32"):
        newton_solve_noalloc(spec, "f16s", dev(xp, torch.float64), None, x)
    with pytest.raises(JfnkError, match="single-workgroup"):
        newton_solve_noalloc(spec, "f64", dev(xp, torch.float64), None, x, engine="multi")
    assert np.array_equal(host(x), xp)  # nothing ran
