"""Serving (jfnk_batch_*): continuous batching of independent Newton solves.

Contract:
  * a request's result is bitwise the same alone (one slot, one request on
    the device) and in a mix (several slots, requests of different shapes
    overlapping on the device), with the same Newton and Krylov counts;
  * it is bitwise the same as the standalone solver's result for the same
    problem, precision and options;
  * it matches the oracle to the FP32 bound (1e-5 relative per iterate is
    checked elsewhere for the standalone path; here the final iterate);
  * the device-memory budget binds: workspaces held never exceed it, and a
    request larger than the budget is rejected at submission.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import dev, gpu_available, host, wdtype
from oracle import NewtonOptions, Problem, newton_solve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


def small_stream(count=12, seed=3):
    """Serving-mix requests restricted to small sizes (1D N <= 4096, GS side <= 128)."""
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        if r % 2 == 0:
            req = dict(id=r, kind="burgers1d", size=int(2 ** rng.integers(8, 13)), seed=int(rng.integers(0, 2**31 - 1)))
        else:
            req = dict(id=r, kind="grayscott", size=int(2 ** rng.integers(6, 8)), seed=int(rng.integers(0, 2**31 - 1)))
        out.append(req)
    return out


def run_alone(reqs, prec="f32"):
    from paper_2605_13378_amd import Batch

    b = Batch(prec, m=30, max_slots=1)
    res = []
    for req in reqs:
        spec, xp = W.serving_request_inputs(req)
        t = b.submit(spec, xp)
        res.append(b.wait(t))
    b.close()
    return res


def test_mix_equals_alone_bitwise():
    from paper_2605_13378_amd import Batch

    reqs = small_stream()
    alone = run_alone(reqs)
    b = Batch("f32", m=30, max_slots=4)
    tickets = []
    for req in reqs:
        spec, xp = W.serving_request_inputs(req)
        tickets.append(b.submit(spec, xp))
    mixed = [b.wait(t) for t in tickets]
    st = b.stats()
    b.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["max_running"] >= 2, st  # requests did overlap on the device
    for req, (xa, ia), (xm, im) in zip(reqs, alone, mixed):
        assert ia["rc"] == 0 and im["rc"] == 0, (req, ia["status"], im["status"])
        assert np.array_equal(xa, xm), req
        assert ia["newton_iters"] == im["newton_iters"] and ia["krylov_iters"] == im["krylov_iters"], req
        assert ia["rel_res"] == im["rel_res"], req


def test_batch_equals_standalone_solver():
    from paper_2605_13378_amd import Batch, Solver

    req = dict(id=0, kind="grayscott", size=128, seed=11)
    spec, xp = W.serving_request_inputs(req)
    b = Batch("f32", m=30, max_slots=2)
    xb, ib = b.wait(b.submit(spec, xp))
    b.close()
    s = Solver(spec, "f32", m=30)
    s.set_previous(dev(xp, wdtype("f64")))
    xs, is_ = s.newton_solve(dev(xp, wdtype("f64")))
    assert np.array_equal(xb, host(xs))
    assert ib["krylov_iters"] == is_["krylov_iters"]


@pytest.mark.parametrize("req", [dict(id=0, kind="burgers1d", size=256, seed=5),
                                 dict(id=1, kind="grayscott", size=64, seed=6)])
def test_batch_result_matches_oracle_f32(req):
    from paper_2605_13378_amd import Batch

    spec, xp = W.serving_request_inputs(req)
    b = Batch("f32", m=30, max_slots=2)
    x, info = b.wait(b.submit(spec, xp))
    b.close()
    o = NewtonOptions.for_precision("f32")
    x_ref, info_ref = newton_solve(Problem.from_spec(spec), xp, o)
    assert info["converged"] and info_ref.converged
    assert info["newton_iters"] == info_ref.newton_iters
    assert np.linalg.norm(x - x_ref) <= 1e-5 * np.linalg.norm(x_ref)


def test_budget_binds_and_results_stay_equal():
    from paper_2605_13378_amd import Batch, footprint_bytes

    reqs = small_stream(count=8, seed=9)
    biggest = 0
    for req in reqs:
        spec, _ = W.serving_request_inputs(req)
        n = W.n_unknowns(spec)
        biggest = max(biggest, footprint_bytes(spec, "f32", 30) + 2 * 8 * n)
    budget = int(1.5 * biggest)
    alone = run_alone(reqs)
    b = Batch("f32", m=30, max_slots=4, budget_bytes=budget)
    tickets = []
    for req in reqs:
        spec, xp = W.serving_request_inputs(req)
        tickets.append(b.submit(spec, xp))
    mixed = [b.wait(t) for t in tickets]
    st = b.stats()
    b.close()
    assert st["peak_bytes"] <= budget, st
    assert st["completed"] == len(reqs)
    # the budget forced releases, and every device free waited for an idle device
    assert st["workspaces_released"] > 0 and st["frees_while_running"] == 0, st
    for (xa, _), (xm, _) in zip(alone, mixed):
        assert np.array_equal(xa, xm)


def test_no_cache_frees_wait_for_idle_device():
    """keep_workspaces = 0: every finished request's workspace is released, but its
    device memory goes back only while no request runs; results unchanged."""
    from paper_2605_13378_amd import Batch

    reqs = small_stream(count=10, seed=4)
    alone = run_alone(reqs)
    b = Batch("f32", m=30, max_slots=4, keep_workspaces=False)
    tickets = []
    for req in reqs:
        spec, xp = W.serving_request_inputs(req)
        tickets.append(b.submit(spec, xp))
    mixed = [b.wait(t) for t in tickets]
    st = b.stats()
    b.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["workspaces_released"] == len(reqs) and st["frees_while_running"] == 0, st
    for (xa, _), (xm, _) in zip(alone, mixed):
        assert np.array_equal(xa, xm)


def test_full_serving_range_alone_equals_mix():
    """The serving stream itself (1D Burgers N = 2^8..2^16, Gray-Scott side 2^6..2^10,
    Gray-Scott 1024^2 included): each result bitwise the same alone and among 8 slots."""
    from paper_2605_13378_amd import Batch

    reqs = W.serving_stream(count=2000, seed=0, rate=1.0)[:24]
    sizes = {(r["kind"], r["size"]) for r in reqs}
    assert ("grayscott", 1024) in sizes and max(r["size"] for r in reqs if r["kind"] == "burgers1d") >= 2 ** 15
    alone = run_alone(reqs)
    b = Batch("f32", m=30, max_slots=8)
    tickets = []
    for req in reqs:
        spec, xp = W.serving_request_inputs(req)
        tickets.append(b.submit(spec, xp))
    mixed = [b.wait(t) for t in tickets]
    st = b.stats()
    b.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0 and st["max_running"] >= 2, st
    for req, (xa, ia), (xm, im) in zip(reqs, alone, mixed):
        assert ia["rc"] == 0 and im["rc"] == 0, req
        assert np.array_equal(xa, xm), req
        assert ia["krylov_iters"] == im["krylov_iters"], req


def test_submit_rejects_oversized_and_invalid():
    from paper_2605_13378_amd import Batch, JfnkError

    b = Batch("f32", m=30, max_slots=1, budget_bytes=1 << 20)
    spec, xp = W.serving_request_inputs(dict(id=0, kind="grayscott", size=256, seed=1))
    with pytest.raises(JfnkError):
        b.submit(spec, xp)  # needs far more than 1 MiB
    bad = dict(spec, nx=0)
    with pytest.raises(JfnkError):
        b.submit(bad, np.zeros(0))
    b.close()


def mixed_kind_requests():
    """Every problem kind (both Su-Olson configurations), Krylov method and the CSLP
    preconditioner in one stream (FP64)."""
    reqs = []
    spec, xp = W.rd2d_spec(48), W.rd2d_initial(48, 1)
    reqs.append((spec, xp, None, dict(krylov="cg")))
    xs, src = W.suolson_initial(40, 2)
    reqs.append((W.suolson_spec(40), xs, src, dict(krylov="bicgstab")))
    spec, xp = dict(W.grayscott_spec(64)), W.grayscott_initial(64, 3, side_frac=1 / 8, patches=6)
    reqs.append((spec, xp, None, dict(orth="dcgs2")))
    reqs.append((W.maxwell_spec(16, omega=2.5), np.zeros(4 * 16 * 16), W.maxwell_source(16, omega=2.5),
                 dict(max_newton=20)))
    spec, x0 = W.burgers2d_paper_case("dsl", 32)
    reqs.append((spec, x0, None, dict(orth="cgs2")))
    reqs.append((W.rd2d_spec(32), W.rd2d_initial(32, 4), None, dict(krylov="bicgstab")))
    reqs.append((W.maxwell_spec(16, omega=2.5), np.zeros(4 * 16 * 16), W.maxwell_source(16, omega=2.5),
                 dict(max_newton=20, precond="cslp")))
    x1, src1 = W.suolson_box_initial(40, ny=24)
    reqs.append((W.suolson_spec(40, ny=24, periodic_y=True), x1, src1, dict(orth="dcgs2")))
    return reqs


def test_mixed_problem_kinds_and_methods_alone_equals_mix():
    from paper_2605_13378_amd import Batch

    reqs = mixed_kind_requests()
    alone = []
    b1 = Batch("f64", m=30, max_slots=1)
    for spec, xp, src, o in reqs:
        alone.append(b1.wait(b1.submit(spec, xp, src, **o)))
    b1.close()
    b8 = Batch("f64", m=30, max_slots=8)
    tickets = [b8.submit(spec, xp, src, **o) for spec, xp, src, o in reqs]
    mixed = [b8.wait(t) for t in tickets]
    b8.close()
    for (spec, xp, src, o), (xa, ia), (xm, im) in zip(reqs, alone, mixed):
        assert np.array_equal(xa, xm), spec["kind"]
        assert ia["krylov_iters"] == im["krylov_iters"] and ia["newton_iters"] == im["newton_iters"]
        assert ia["converged"], (spec["kind"], ia)
        # against the oracle with the same method and Gram-Schmidt form
        p = Problem.from_spec(spec)
        opts = NewtonOptions.for_precision("f64", krylov=o.get("krylov", "gmres"), orth=o.get("orth", "dcgs2"),
                                           max_newton=o.get("max_newton", 15), precond=o.get("precond", "none"))
        xr, ir = newton_solve(p, xp, opts, source=src)
        assert ir.converged and ir.newton_iters == ia["newton_iters"], (spec["kind"], ir.newton_iters, ia)
        tol = 1e-6 if spec["kind"] == "maxwell" else 1e-10
        assert np.linalg.norm(xa - xr) <= tol * max(1.0, np.linalg.norm(xr)), spec["kind"]


def test_graph_engine_in_a_mix_equals_multi_kernel_alone():
    """Requests on the graph engine (each worker captures its cycles while the others run and
    allocate workspaces) give bitwise the multi-kernel engine's results alone."""
    from paper_2605_13378_amd import Batch

    reqs = W.serving_stream(count=2000, seed=0, rate=1.0)[:40]
    b1 = Batch("f32", m=30, max_slots=1)
    alone = []
    for req in reqs:
        spec, xp = W.serving_request_inputs(req)
        alone.append(b1.wait(b1.submit(spec, xp, engine="multi")))
    b1.close()
    b = Batch("f32", m=30, max_slots=8)
    tickets = []
    for req in reqs:
        spec, xp = W.serving_request_inputs(req)
        tickets.append(b.submit(spec, xp, engine="graph"))
    mixed = [b.wait(t) for t in tickets]
    st = b.stats()
    b.close()
    assert st["failed"] == 0 and st["max_running"] >= 2, st
    for req, (xa, ia), (xm, im) in zip(reqs, alone, mixed):
        assert ia["rc"] == 0 and im["rc"] == 0, (req, ia["status"], im["status"])
        assert np.array_equal(xa, xm), req
        assert ia["krylov_iters"] == im["krylov_iters"], req
