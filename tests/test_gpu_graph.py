"""The MULTI_KERNEL_GRAPH engine: each GMRES restart cycle launched as one
captured HIP graph.  It launches the same kernels with the same arguments in
the same order as MULTI_KERNEL, so every result must be bitwise the same:
the Newton iterate, the Newton and Krylov counts, the residual history.
Replays of a cached graph are checked again after other (eager) solves on
the same solver, and the engine falls back to direct launches on the null
stream, which cannot be captured."""

import numpy as np
import pytest

import workloads as W
from gpu_cases import case, dev, gpu_available, host, torch_mod, wdtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def run(s, xp, **kw):
    torch = torch_mod()
    x, info = s.newton_solve(dev(xp, wdtype("f64")), **kw)
    torch.cuda.synchronize()
    return host(x), info


@pytest.mark.parametrize("name,prec,kw", [
    ("gs64-f64", "f64", dict()),
    ("gs64-f32", "f32", dict()),
    ("gs64-f32-fd", "f32", dict(mode="fd", eps_rule="normalized")),
    ("gs64-f32-cgs2", "f32", dict(orth="cgs2")),
    ("gs64-f16s", "f16s", dict()),
    ("burgers2d", "f64", dict()),
    ("kerr-restarts", "f64", dict(max_newton=20)),
    ("maxwell-cslp", "f64", dict(max_newton=20, precond="cslp")),
    ("gs1024-f32", "f32", dict(eps_rule="normalized")),
])
def test_graph_engine_equals_multi_kernel_bitwise(name, prec, kw):
    from paper_2605_13378_amd import Solver

    torch = torch_mod()
    if name.startswith("gs64"):
        spec, xp, src = case("grayscott", 64, 64)
    elif name == "burgers2d":
        spec, xp, src = case("burgers2d", 48, 40)
    elif name == "kerr-restarts":
        import order_spread as OS

        spec, xp, src, _, _, _, _ = OS.case("kerr12x10_cpw32_chi1.0")
    elif name == "maxwell-cslp":
        spec, xp, src = W.maxwell_spec(16, omega=2.5), np.zeros(4 * 16 * 16), W.maxwell_source(16, omega=2.5)
    else:
        spec, xp, src = W.config("grayscott")
    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        s = Solver(spec, prec, m=30, stream=st)
        s.set_previous(None if name in ("kerr-restarts", "maxwell-cslp") else dev(xp, wdtype("f64")),
                       None if src is None else dev(src, wdtype("f64")))
        xm, im = run(s, xp, engine="multi", **kw)
        assert s.cycle_graphs() == 0
        outs = []
        for rep in range(3):
            outs.append(run(s, xp, engine="graph", **kw))
            if rep == 0:
                ncap = s.cycle_graphs()
                assert ncap >= 1, "the graph engine captured no cycle"
            run(s, xp, engine="multi", **kw)  # eager work between replays
        assert s.cycle_graphs() == ncap  # replays reuse the captured graphs
        s.close()
    torch.cuda.synchronize()
    for xg, ig in outs:
        assert np.array_equal(xg, xm), name
        for key in ("newton_iters", "krylov_iters", "restarts", "lin_iters", "rel_res", "converged"):
            assert ig[key] == im[key], (name, key, ig[key], im[key])


def test_graph_engine_rules():
    from paper_2605_13378_amd import JfnkError, Solver

    torch = torch_mod()
    spec, xp, src = case("grayscott", 32, 32)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        s = Solver(spec, "f64", m=30, stream=st)
        s.set_previous(dev(xp, wdtype("f64")))
        with pytest.raises(JfnkError, match="graph"):
            s.newton_solve(dev(xp, wdtype("f64")), engine="graph", krylov="bicgstab")
        # profiling on: cycles run directly (timing events are not captured), same result
        s.profile(True)
        xa, ia = run(s, xp, engine="graph")
        s.profile(False)
        assert s.cycle_graphs() == 0
        xb, ib = run(s, xp, engine="graph")
        assert s.cycle_graphs() >= 1
        assert np.array_equal(xa, xb) and ia["krylov_iters"] == ib["krylov_iters"]
        s.close()
    torch.cuda.synchronize()
