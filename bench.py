"""Benchmark of the JFNK hot path on one MI355X.

Workload: implicit (backward-Euler) step of the two-species Gray-Scott
reaction-diffusion system on a 1024 x 1024 periodic grid (D = 2e-5,
Dv = 1e-5, F = 0.04, k = 0.06, dt = 1, h = sqrt(D dt)), seeded random square
patches, solved by Newton with line search around GMRES(30) with classical
Gram-Schmidt applied twice, the second pass delayed one step (DCGS2, two
passes over the basis per Arnoldi step; --orth cgs2 runs the three-pass form),
and FP64 Givens.  One step = one whole Newton solve of that implicit step
(residuals, JVPs, every Arnoldi pass, Givens, V y updates, line search), with
the inputs resident in HBM before the timed region starts.

The headline line is the AD JVP in FP32 working precision (FP64 Givens,
Newton update and merit norm); FP64 and FD variants, the JVP bandwidth of
the AD and FD kernels, per-solve latency percentiles, the roofline of the
kernel that takes most of the time, and the CPU oracle timed on the host
are reported on the same JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E peak
CONFIG_NAME = "grayscott-1024x1024-backward-euler"

# Calibrated HBM traffic / algorithmic bytes of the dominant kernel class, from the
# rocprofv3 FETCH_SIZE / WRITE_SIZE runs summarized in profiles/, valid only for the
# kernel sources and launch shapes they were taken with (hash of the device headers and
# of the host file that sizes the grids).
MEASURED_TRAFFIC = {
    "jvp_ad": {"sources": "10a839899f5cf92b", "orth": "dcgs2", "ratio": 1.108},
    "dcgs_update": {"sources": "10a839899f5cf92b", "orth": "dcgs2", "ratio": 1.019},
}

def kernel_sources_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in ("common.hpp", "krylov.hpp", "problems.hpp", "stencil.hpp", "launch.hpp", "launch_impl.hpp",
              "launch_stencil.hpp", "stencil_inst.hip", "solver.hip"):
        with open(os.path.join(HERE, "paper_2605_13378_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, bytes_per_launch: float, orth: str, sources: str | None = None):
    """HBM bytes per launch of `kernel` from the calibrated counter ratio, or None when no
    measurement exists for it, or the kernel sources or the Gram-Schmidt form differ from the
    ones the counters were taken with."""
    meas = MEASURED_TRAFFIC.get(kernel)
    if meas is None or meas["orth"] != orth:
        return None
    if meas["sources"] != (kernel_sources_hash() if sources is None else sources):
        return None
    return round(meas["ratio"] * bytes_per_launch)


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    s = sorted(xs)
    if not s:
        return float("nan")
    k = (len(s) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return s[lo] + (s[hi] - s[lo]) * (k - lo)


def make_solver(spec, prec, xp, torch):  # prec: f64 | f32 | f16s
    from paper_2605_13378_amd import Solver

    s = Solver(spec, prec, m=30)
    s.set_previous(torch.tensor(xp, dtype=torch.float64, device="cuda"))
    return s


ORTH = "dcgs2"  # GMRES Gram-Schmidt form of the headline and variant rows (--orth)


def options_for(prec: str, mode: str) -> dict:
    # the Gray-Scott workload takes the normalized FD step rule
    return dict(mode=mode, eps_rule="normalized", orth=ORTH)


def run_solves(s, x0, torch, count, opts, sync_each=True):
    """Run `count` Newton solves; returns (elapsed seconds, per-solve latencies, last info)."""
    lat = []
    info = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(count):
        t1 = time.perf_counter()
        _, info = s.newton_solve(x0, **opts)
        lat.append(time.perf_counter() - t1)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, lat, info


QUEUE_SPIN_CYCLES = 50_000_000


def jvp_bandwidth(s, torch, n, prec, mode, reps=200, scrub=None):
    """Average duration (HIP events on the solver stream) and algorithmic GB/s of one JVP kind.

    With `scrub` (a large device tensor), the 256 MB last-level cache is
    flushed by overwriting it before every launch (cold-cache protocol); the
    events bracket the JVP kernel only.
    """
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(1)
    x = 1.0 + 0.1 * torch.randn(n, device="cuda", dtype=dt, generator=g)
    v = torch.randn(n, device="cuda", dtype=dt, generator=g)
    for _ in range(5):
        s.jvp(x, v, mode=mode)
    torch.cuda.synchronize()
    s.profile_reset()
    s.profile(True)
    # queue every launch behind a spin kernel so that they run back to back,
    # as inside a solve, instead of one at a time from an idle device
    if hasattr(torch.cuda, "_sleep"):
        torch.cuda._sleep(QUEUE_SPIN_CYCLES)
    for _ in range(reps):
        if scrub is not None:
            scrub.add_(1.0)
        s.jvp(x, v, mode=mode)
    torch.cuda.synchronize()
    st = s.profile_read()["jvp_ad" if mode == "ad" else "jvp_fd"]
    s.profile(False)
    s.profile_reset()
    avg_us = st["ms"] * 1e3 / max(1, st["launches"])
    gbs = st["bytes"] / (st["ms"] * 1e-3) / 1e9 if st["ms"] > 0 else 0.0
    return dict(avg_us=round(avg_us, 3), gbs=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4),
                bytes_per_launch=st["bytes"] / max(1, st["launches"]), launches=st["launches"])


def jvp_bandwidth_hbm(torch, spec, xp, src, prec, mode, min_bytes=1 << 30, min_reps=100):
    """The same measurement with operands the last-level cache cannot hold: R solvers (each with
    its own constant part b, read by the FD JVP) and R distinct (x, v, Jv) triples, R chosen so
    that the operands of one sweep exceed `min_bytes` (1 GiB, four times the 256 MB cache), used
    in turn, so every launch reads vectors last touched R - 1 launches (>= 1 GiB of traffic) ago.
    No scrub writes are involved: eviction is driven by the JVP reads themselves."""
    import workloads as W
    from paper_2605_13378_amd import Solver

    n = W.n_unknowns(spec)
    esz = 8 if prec == "f64" else 4
    per_call = (3 if mode == "ad" else 4) * n * esz
    R = max(2, math.ceil(min_bytes / per_call))
    dt = torch.float64 if prec == "f64" else torch.float32
    g = torch.Generator(device="cuda").manual_seed(2)
    x_prev = torch.tensor(xp, dtype=torch.float64, device="cuda")
    source = None if src is None else torch.tensor(src, dtype=torch.float64, device="cuda")
    solvers, xs, vs, outs = [], [], [], []
    for _ in range(R):
        sv = Solver(spec, prec, m=1)
        sv.set_previous(x_prev, source)
        solvers.append(sv)
        xs.append(x_prev.to(dt) + 0.1 * torch.randn(n, device="cuda", dtype=dt, generator=g))
        vs.append(torch.randn(n, device="cuda", dtype=dt, generator=g))
        outs.append(torch.empty(n, device="cuda", dtype=dt))
    reps = max(min_reps, 3 * R)
    for k in range(R):
        solvers[k].jvp(xs[k], vs[k], mode=mode, out=outs[k])
    torch.cuda.synchronize()
    for sv in solvers:
        sv.profile_reset()
        sv.profile(True)
    if hasattr(torch.cuda, "_sleep"):
        torch.cuda._sleep(QUEUE_SPIN_CYCLES)
    for i in range(reps):
        k = i % R
        solvers[k].jvp(xs[k], vs[k], mode=mode, out=outs[k])
    torch.cuda.synchronize()
    key = "jvp_ad" if mode == "ad" else "jvp_fd"
    ms = byt = 0.0
    launches = 0
    for sv in solvers:
        st = sv.profile_read()[key]
        ms += st["ms"]
        byt += st["bytes"]
        launches += st["launches"]
        sv.profile(False)
        sv.close()
    avg_us = ms * 1e3 / max(1, launches)
    gbs = byt / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return dict(avg_us=round(avg_us, 3), gbs=round(gbs, 1), frac=round(gbs / PEAK_HBM_GBS, 4),
                bytes_per_launch=byt / max(1, launches), launches=launches, operand_sets=R,
                sweep_bytes=R * per_call)


def copy_ceiling_hbm(torch, vector_bytes, min_bytes=1 << 30, reps=100):
    """Reference for the "-hbm" JVP rows: a plain device copy (torch's copy kernel, one read and one
    write stream) of one vector of `vector_bytes`, rotating over distinct (src, dst) pairs that
    total >= `min_bytes`, queued back to back; GB/s counts read + written bytes.  It is what a
    kernel with no arithmetic at all reaches for transfers of this size from HBM."""
    nel = vector_bytes // 4
    R = max(2, math.ceil(min_bytes / (2 * vector_bytes)))
    pairs = [(torch.ones(nel, dtype=torch.float32, device="cuda"), torch.empty(nel, dtype=torch.float32,
                                                                               device="cuda")) for _ in range(R)]
    for a, b in pairs:
        b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    if hasattr(torch.cuda, "_sleep"):
        torch.cuda._sleep(QUEUE_SPIN_CYCLES)
    e0.record()
    for i in range(reps):
        a, b = pairs[i % R]
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    gbs = 2 * vector_bytes / (us * 1e-6) / 1e9
    del pairs
    return dict(vector_mb=round(vector_bytes / 1e6, 1), avg_us=round(us, 3), gbs=round(gbs, 1),
                frac=round(gbs / PEAK_HBM_GBS, 4), pairs=R)


def latency_c1(torch, repeats, seeds):
    """1D Burgers N=256, one backward-Euler step, FP64, GMRES(30), tol_N 1e-10,
    tol_K 1e-12: per-solve wall time (p50/p99) of the single-workgroup engine
    and of the multi-kernel one, AD and FD (paper step), and over seeds."""
    import workloads as W

    spec, xp, _ = W.config("burgers1d", seed=0)
    s = make_solver(spec, "f64", xp, torch)
    x0 = torch.tensor(xp, dtype=torch.float64, device="cuda")
    base = dict(tol_newton=1e-10, tol_krylov=1e-12, m=30, max_newton=15)
    out = {"workload": "burgers1d_256_f64", "tol_newton": 1e-10, "tol_krylov": 1e-12}
    for engine in ("single", "multi"):
        for mode in ("ad", "fd"):
            o = dict(base, mode=mode, engine=engine)
            # FD cannot reach tol_K 1e-12 (its JVP carries ~sqrt(eps) relative
            # error), so every FD Newton step runs all restart cycles: few repeats
            if mode == "fd":
                count = 5 if engine == "single" else 2
            else:
                count = repeats if engine == "single" else max(1, repeats // 5)
            run_solves(s, x0, torch, 1 if mode == "fd" else 5, o)
            el, lat, info = run_solves(s, x0, torch, count, o)
            out[f"{engine}-{mode}"] = dict(solves=count, solves_per_s=round(count / el, 1),
                                           p50_us=round(1e6 * percentile(lat, 0.5), 1),
                                           p99_us=round(1e6 * percentile(lat, 0.99), 1),
                                           newton_iters=info["newton_iters"], krylov_iters=info["krylov_iters"],
                                           converged=info["converged"])
            log(f"[bench] C1 {engine}-{mode}: {out[f'{engine}-{mode}']}")
    # seeds 0..seeds-1 (a new previous state per solve), single workgroup, AD
    lat = []
    conv = 0
    o = dict(base, mode="ad", engine="single")
    for sd in range(seeds):
        _, xs, _ = W.config("burgers1d", seed=sd)
        xt = torch.tensor(xs, dtype=torch.float64, device="cuda")
        s.set_previous(xt)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, info = s.newton_solve(xt, **o)
        lat.append(time.perf_counter() - t1)
        conv += int(info["converged"])
    out["seeds-single-ad"] = dict(seeds=seeds, converged=conv, p50_us=round(1e6 * percentile(lat, 0.5), 1),
                                  p99_us=round(1e6 * percentile(lat, 0.99), 1))
    log(f"[bench] C1 seeds: {out['seeds-single-ad']}")
    s.close()
    return out


def completion_c3(torch, seeds, steps=10, n=2048, modes=("ad", "fd"), precisions=("f32", "f16s")):
    """2D Burgers n^2 (Crank-Nicolson, nu 1e-3, dt 5e-4), `steps` implicit steps
    from each seed's random-Fourier field; AD vs FD (paper step), FP32 and FP16S
    with FP64 Givens/update/merit.  A step fails when its final relative
    residual is non-finite or above 100 tol_N; a run fails on a non-finite step
    or when more than 20% of its steps fail.  Completion = runs not failed."""
    from paper_2605_13378_amd import Solver

    import workloads as W

    spec = W.burgers2d_spec(n)
    tol_n = 1e-4
    out = {"workload": f"burgers2d_{n}_cn_{steps}steps", "seeds": seeds, "steps": steps}
    inits = [W.burgers2d_initial(n, sd) for sd in range(seeds)]
    for prec in precisions:
        s = Solver(spec, prec, m=30)
        for mode in modes:
            ok_runs = 0
            failed_steps = 0
            solve_s = 0.0
            solves = 0
            newton = 0
            krylov = 0
            worst = 0.0
            for sd in range(seeds):
                x = torch.tensor(inits[sd], dtype=torch.float64, device="cuda")
                bad = 0
                nonfinite = False
                for _ in range(steps):
                    s.set_previous(x)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    xn, info = s.newton_solve(x, mode=mode, eps_rule="paper")
                    solve_s += time.perf_counter() - t1
                    solves += 1
                    newton += info["newton_iters"]
                    krylov += info["krylov_iters"]
                    last = info["rel_res"][-1] if info["rel_res"] else float("nan")
                    if info["status"] == "nonfinite" or not math.isfinite(last):
                        nonfinite = True
                        break
                    worst = max(worst, last)
                    if not last <= 100 * tol_n:
                        bad += 1
                    x = xn
                failed_steps += bad
                if not nonfinite and bad <= 0.2 * steps:
                    ok_runs += 1
            out[f"{prec}-{mode}"] = dict(completion=round(ok_runs / seeds, 4), runs_ok=ok_runs,
                                         failed_steps=failed_steps, solves=solves,
                                         solves_per_s=round(solves / solve_s, 2) if solve_s > 0 else None,
                                         newton_per_solve=round(newton / max(1, solves), 3),
                                         krylov_per_newton=round(krylov / max(1, newton), 2),
                                         worst_final_rel_res=worst)
            log(f"[bench] C3 {prec}-{mode}: {out[f'{prec}-{mode}']}")
        s.close()
    return out


def kerr_solver(torch, prec, chi3=0.1, eps_im=0.0, n=1024):
    from paper_2605_13378_amd import Solver

    import workloads as W

    spec = W.kerr_spec(n, chi3=chi3, eps_im=eps_im)
    src = W.kerr_gaussian_source(n)
    s = Solver(spec, prec, m=30)
    s.set_previous(None, torch.tensor(src, dtype=torch.float64, device="cuda"))
    return s, spec


def kerr_newton(torch, max_newton=50):
    """Helmholtz-Kerr 1024^2 from E = 0: Newton completion per precision
    (complex64 / complex128), chi3 and loss, AD vs FD.  Unpreconditioned
    GMRES(30) on this indefinite operator is expected to stagnate."""
    import workloads as W

    out = {}
    n_unk = 2 * 1024 * 1024
    x0 = torch.zeros(n_unk, dtype=torch.float64, device="cuda")
    for prec in ("f32", "f64"):
        for chi3 in (0.01, 0.1):
            for eps_im in (0.0, -0.05):
                s, _ = kerr_solver(torch, prec, chi3=chi3, eps_im=eps_im)
                for mode in ("ad", "fd"):
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    _, info = s.newton_solve(x0, mode=mode, eps_rule="paper", max_newton=max_newton)
                    el = time.perf_counter() - t1
                    key = f"{prec}-chi{chi3}-{'lossy' if eps_im else 'lossless'}-{mode}"
                    out[key] = dict(converged=info["converged"], status=info["status"],
                                    newton_iters=info["newton_iters"], krylov_iters=info["krylov_iters"],
                                    final_rel_res=info["rel_res"][-1] if info["rel_res"] else None,
                                    seconds=round(el, 3))
                    log(f"[bench] C4 {key}: {out[key]}")
                s.close()
    return out


def kerr_c4_rows(torch):
    """The Helmholtz-Kerr workload's physics (k0 = 2 pi / 64 cells, eps_L = 1) in the default run:
    Newton to convergence on 64^2 (chi3 0.01 and 0.1, complex64 and complex128, AD; the grid the
    parity tests compare per iterate), and the 1024^2 workload from E = 0 with a cap of 5 Newton
    steps (AD and FD, chi3 0.1): the residual reduction unpreconditioned GMRES(30) reaches there.
    Rows with a "-cslp" suffix: the same with the CSLP right preconditioner (AD)."""
    from paper_2605_13378_amd import Solver

    import workloads as W

    out = {"grid64": {}, "grid1024_cap5": {}}
    for prec in ("f32", "f64"):
        for chi3 in (0.01, 0.1):
            spec = W.kerr_spec(64, chi3=chi3, cells_per_wavelength=64.0)
            s = Solver(spec, prec, m=30)
            s.set_previous(None, torch.tensor(W.kerr_gaussian_source(64), dtype=torch.float64, device="cuda"))
            x0 = torch.zeros(2 * 64 * 64, dtype=torch.float64, device="cuda")
            for pre in ("none", "cslp"):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, info = s.newton_solve(x0, mode="ad", max_newton=50, precond=pre)
                el = time.perf_counter() - t0
                key = f"{prec}-chi{chi3}" + ("-cslp" if pre == "cslp" else "")
                out["grid64"][key] = dict(
                    converged=info["converged"], newton_iters=info["newton_iters"],
                    krylov_iters=info["krylov_iters"], lin_iters=info["lin_iters"],
                    final_rel_res=info["rel_res"][-1], seconds=round(el, 3))
                log(f"[bench] C4 64^2 {key}: {out['grid64'][key]}")
            s.close()
        s, _ = kerr_solver(torch, prec, chi3=0.1)
        x0 = torch.zeros(2 * 1024 * 1024, dtype=torch.float64, device="cuda")
        for mode, pre in (("ad", "none"), ("fd", "none"), ("ad", "cslp")):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = s.newton_solve(x0, mode=mode, eps_rule="paper", max_newton=5, precond=pre)
            el = time.perf_counter() - t0
            mode = mode + ("-cslp" if pre == "cslp" else "")
            out["grid1024_cap5"][f"{prec}-{mode}"] = dict(
                newton_iters=info["newton_iters"], krylov_iters=info["krylov_iters"],
                rel_res=[round(r, 5) for r in info["rel_res"]], seconds=round(el, 3),
                arnoldi_steps_per_s=round(info["krylov_iters"] / el, 1))
            log(f"[bench] C4 1024^2 cap 5 {prec} {mode}: {out['grid1024_cap5'][f'{prec}-{mode}']}")
        s.close()
    return out


def serving_pass(batch, reqs, inputs, rate_scale, saturate, opts=None):
    """Feed `reqs` to `batch` (Poisson arrivals scaled by 1/rate_scale, or all at
    once) and return solves/s and arrival-to-result latency percentiles."""
    import threading

    tickets = [None] * len(reqs)
    results = [None] * len(reqs)
    submitted = threading.Semaphore(0)

    def collect():
        for i in range(len(reqs)):
            submitted.acquire()
            results[i] = batch.wait(tickets[i])

    th = threading.Thread(target=collect)
    th.start()
    t0 = batch.clock()
    arrivals = []
    for i, req in enumerate(reqs):
        target = t0 if saturate else t0 + req["arrival"] / rate_scale
        if not saturate:
            while True:
                dt = target - batch.clock()
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.002) if dt > 0.0005 else 0)
        spec, xp = inputs[i]
        tickets[i] = batch.submit(spec, xp, **(opts or {}))
        arrivals.append(target)
        submitted.release()
    th.join()
    done = [r[1]["times"][2] for r in results]
    lat = [d - a for d, a in zip(done, arrivals)]
    span = max(done) - t0
    bad = sum(1 for r in results if r[1]["rc"] not in (0, 6))
    unconv = sum(1 for r in results if not r[1]["converged"])
    out = dict(solves_per_s=round(len(reqs) / span, 2), makespan_s=round(span, 3),
               p50_ms=round(1e3 * percentile(lat, 0.5), 3), p99_ms=round(1e3 * percentile(lat, 0.99), 3),
               failed=bad, not_converged=unconv)
    if bad:
        # status codes of the failed requests (jfnk_status) and which requests
        codes = {}
        for i, r in enumerate(results):
            if r[1]["rc"] not in (0, 6):
                codes.setdefault(str(r[1]["rc"]), []).append(f"{reqs[i]['kind']}:{reqs[i]['size']}")
        out["failed_status"] = codes
    return out


def serving_bench(count, slots, budget_gib, seed=0):
    """Continuous batching vs one request at a time on the serving mix (FP32, AD)."""
    from paper_2605_13378_amd import Batch

    import workloads as W

    reqs = W.serving_stream(count=count, seed=seed, rate=1.0)
    inputs = [W.serving_request_inputs(r) for r in reqs]
    budget = int(budget_gib * (1 << 30))
    single = Batch("f32", m=30, max_slots=1, budget_bytes=budget)
    multi = Batch("f32", m=30, max_slots=slots, budget_bytes=budget)
    warm = min(len(reqs), 200)
    serving_pass(single, reqs[:warm], inputs[:warm], 1.0, True)
    serving_pass(multi, reqs[:warm], inputs[:warm], 1.0, True)
    out = {"requests": count, "stream_seed": seed, "slots": slots, "budget_gib": budget_gib,
           "precision": "f32", "jvp": "ad", "mix": "1D Burgers N=2^8..2^16 / Gray-Scott side 2^6..2^10, 1:1"}
    sat1 = serving_pass(single, reqs, inputs, 1.0, True)
    satm = serving_pass(multi, reqs, inputs, 1.0, True)
    mu1 = sat1["solves_per_s"]
    out["saturation"] = {"one_at_a_time": sat1, "batched": satm}
    log(f"[bench] serving saturation: one-at-a-time {sat1} batched {satm}")
    # saturation throughput against the slot count (a process gets 4 hardware queues here,
    # so streams beyond 4 share them)
    by_slots = {"1": sat1, str(slots): satm}
    for k in (2, 4, 8, 16):
        if str(k) in by_slots:
            continue
        bk = Batch("f32", m=30, max_slots=k, budget_bytes=budget)
        serving_pass(bk, reqs[:warm], inputs[:warm], 1.0, True)
        by_slots[str(k)] = serving_pass(bk, reqs, inputs, 1.0, True)
        bk.close()
        log(f"[bench] serving saturation with {k} slots: {by_slots[str(k)]}")
    out["saturation_by_slots"] = dict(sorted(by_slots.items(), key=lambda kv: int(kv[0])))
    # every request on the multi-kernel engine with captured restart cycles (HIP graphs), against
    # the default engine choice (single-workgroup engine for the requests that fit it)
    serving_pass(multi, reqs[:warm], inputs[:warm], 1.0, True, opts=dict(engine="graph"))
    out["saturation_graph_engine"] = serving_pass(multi, reqs, inputs, 1.0, True, opts=dict(engine="graph"))
    out["saturation_multi_engine"] = serving_pass(multi, reqs, inputs, 1.0, True, opts=dict(engine="multi"))
    log(f"[bench] serving saturation, graph engine {out['saturation_graph_engine']}, "
        f"multi-kernel engine {out['saturation_multi_engine']}")
    rows = []
    for lam in (0.5, 1.0, 2.0, 4.0):
        rate = lam * mu1  # requests/s; the stream was drawn at 1 request/s
        r1 = serving_pass(single, reqs, inputs, rate, False)
        rm = serving_pass(multi, reqs, inputs, rate, False)
        rows.append({"lambda_over_mu1": lam, "rate_per_s": round(rate, 2), "one_at_a_time": r1, "batched": rm})
        log(f"[bench] serving lambda={lam} mu1: one-at-a-time {r1} batched {rm}")
    out["poisson"] = rows
    out["batched_stats"] = multi.stats()
    single.close()
    multi.close()
    return out


def _oracle_serving_request(req):
    """One serving request through the oracle (a worker process of serving_oracle)."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import NewtonOptions, Problem, newton_solve

    spec, xp = W.serving_request_inputs(req)
    with threadpool_limits(1):
        _, info = newton_solve(Problem.from_spec(spec), xp, NewtonOptions.for_precision("f32", mode="ad"))
    return info.converged


def serving_oracle(sample=32, seed=0, workers=None):
    """The serving stream's first `sample` requests through the oracle on P worker
    processes (one core each): requests per second of the whole sample."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import workloads as W

    workers = workers or min(16, os.cpu_count() or 1)
    reqs = W.serving_stream(count=2000, seed=seed, rate=1.0)[:sample]
    # spawned children: a fresh interpreter, nothing inherited from this GPU process
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        list(ex.map(_oracle_serving_request, [dict(id=0, kind="burgers1d", size=256, seed=1)] * workers))
        t0 = time.perf_counter()
        conv = list(ex.map(_oracle_serving_request, reqs))
        el = time.perf_counter() - t0
    return dict(value=round(sample / el, 3), unit="solves/s", cores=workers, kind="oracle",
                sample=f"the first {sample} requests of the serving stream (seed {seed}; FP32 tolerances, FP64 "
                       f"arithmetic), one request per worker process at a time; {sum(conv)} converged",
                seconds=round(el, 2))


def graph_engine_row(torch, spec, xp, steps, prec="f32"):
    """The headline solve on the multi-kernel engine launched directly and with each restart
    cycle replayed from a captured HIP graph (a solver on a stream of its own: the null stream
    cannot be captured)."""
    from paper_2605_13378_amd import Solver

    st = torch.cuda.Stream()
    torch.cuda.synchronize()
    out = {}
    with torch.cuda.stream(st):
        s = Solver(spec, prec, m=30, stream=st)
        x0 = torch.tensor(xp, dtype=torch.float64, device="cuda")
        s.set_previous(x0)
        o = options_for(prec, "ad")
        for eng in ("multi", "graph"):
            s.newton_solve(x0, engine=eng, **o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                _, info = s.newton_solve(x0, engine=eng, **o)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[eng] = dict(solves_per_s=round(steps / el, 2), krylov_iters=info["krylov_iters"])
        out["cycle_graphs"] = s.cycle_graphs()
        s.close()
    return out


def bicgstab_rows(torch, spec, xp, x0, steps, budget_s=8.0):
    """Newton with BiCGSTAB on the Gray-Scott workload: solves/s, iterations, per-kernel timing."""
    rows = {}
    for pr in ("f32", "f64"):
        sv = make_solver(spec, pr, xp, torch)
        for mode in ("ad", "fd"):
            o = dict(options_for(pr, mode), krylov="bicgstab")
            run_solves(sv, x0, torch, 1, o)
            cnt, t_all, lat_v, inf = 0, 0.0, [], None
            while t_all < budget_s and cnt < steps:
                el, l1, inf = run_solves(sv, x0, torch, 1, o)
                t_all += el
                lat_v += l1
                cnt += 1
            sv.profile_reset()
            sv.profile(True)
            run_solves(sv, x0, torch, 1, o)
            st = sv.profile_read()
            sv.profile(False)
            kern = {k: dict(launches=v["launches"], avg_us=round(v["ms"] * 1e3 / v["launches"], 3),
                            gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else 0.0)
                    for k, v in st.items() if v["launches"]}
            rows[f"{pr}-{mode}"] = dict(solves_per_s=round(cnt / t_all, 3), solves=cnt,
                                        p50_ms=round(1e3 * percentile(lat_v, 0.5), 3),
                                        newton_iters=inf["newton_iters"], krylov_iters=inf["krylov_iters"],
                                        lin_iters=inf["lin_iters"], converged=inf["converged"],
                                        final_rel_res=inf["rel_res"][-1], kernels=kern)
            log(f"[bench] bicgstab {pr}-{mode}: {rows[f'{pr}-{mode}']}")
        sv.close()
    return rows


def rd_rows(torch, steps, budget_s=3.0):
    """The paper's SPD problem (u^3 reaction-diffusion, 512^2, Crank-Nicolson, paper FD step):
    Newton with CG, BiCGSTAB and GMRES(30), AD and FD, FP32 and FP64."""
    import workloads as W

    spec, xp, _ = W.config("rd2d")
    x0 = torch.tensor(xp, dtype=torch.float64, device="cuda")
    rows = {}
    for pr in ("f32", "f64"):
        sv = make_solver(spec, pr, xp, torch)
        for kr in ("cg", "bicgstab", "gmres"):
            for mode in ("ad", "fd"):
                o = dict(mode=mode, eps_rule="paper", krylov=kr)
                run_solves(sv, x0, torch, 1, o)
                cnt, t_all, inf = 0, 0.0, None
                while t_all < budget_s and cnt < steps:
                    el, _, inf = run_solves(sv, x0, torch, 1, o)
                    t_all += el
                    cnt += 1
                rows[f"{pr}-{kr}-{mode}"] = dict(solves_per_s=round(cnt / t_all, 3), solves=cnt,
                                                 newton_iters=inf["newton_iters"], lin_iters=inf["lin_iters"],
                                                 converged=inf["converged"], final_rel_res=inf["rel_res"][-1])
                log(f"[bench] rd2d 512^2 {pr}-{kr}-{mode}: {rows[f'{pr}-{kr}-{mode}']}")
        sv.close()
    return rows


def suolson_rows(torch, steps, budget_s=3.0, config="suolson"):
    """The paper's Su-Olson radiation diffusion at 512^2 (affine: FD equals AD up to rounding):
    one Crank-Nicolson step with GMRES(30) and BiCGSTAB, AD and FD (paper step), FP32 and FP64.
    config: 'suolson' (rings and orbiting source, Dirichlet all round) or 'suolson1d' (the
    classic 1D profile: periodic rows, cold start, central box source)."""
    import workloads as W

    spec, xp, src = W.config(config)
    x0 = torch.tensor(xp, dtype=torch.float64, device="cuda")
    rows = {}
    for pr in ("f32", "f64"):
        from paper_2605_13378_amd import Solver

        sv = Solver(spec, pr, m=30)
        sv.set_previous(x0, torch.tensor(src, dtype=torch.float64, device="cuda"))
        for kr in ("gmres", "bicgstab"):
            for mode in ("ad", "fd"):
                o = dict(mode=mode, eps_rule="paper", krylov=kr)
                run_solves(sv, x0, torch, 1, o)
                cnt, t_all, inf = 0, 0.0, None
                while t_all < budget_s and cnt < steps:
                    el, _, inf = run_solves(sv, x0, torch, 1, o)
                    t_all += el
                    cnt += 1
                rows[f"{pr}-{kr}-{mode}"] = dict(solves_per_s=round(cnt / t_all, 3), solves=cnt,
                                                 newton_iters=inf["newton_iters"], lin_iters=inf["lin_iters"],
                                                 converged=inf["converged"], final_rel_res=inf["rel_res"][-1])
                log(f"[bench] {config} 512^2 {pr}-{kr}-{mode}: {rows[f'{pr}-{kr}-{mode}']}")
        sv.close()
    return rows


def maxwell_rows(torch, n=16, omegas=(2.0, 2.5, 3.0, 3.5, 4.0), max_newton=50):
    """Paper-form Maxwell-Kerr (2D TE): JVP bandwidth at 512^2 and a frequency sweep at n^2 with
    continuation: the first frequency starts from the Born guess (E = 0, whose first Newton step
    is the Born solve), each later one from the previous converged field; a frequency fails when
    Newton does not reach tol_Newton within max_newton iterations, and the next one then starts
    again from the Born guess; the run fails when more than 20% of the frequencies fail.  Also
    the same sweep at 256^2 with a Newton cap of 8."""
    import workloads as W
    from paper_2605_13378_amd import Solver

    out = {"jvp_512": {}, "arnoldi_jvp_512": {}}
    spec, x0, src = W.config("maxwell")
    nn = W.n_unknowns(spec)
    for pr in ("f32", "f64"):
        s = Solver(spec, pr, m=30)
        s.set_previous(None, torch.tensor(src, dtype=torch.float64, device="cuda"))
        for mode in ("ad", "fd"):
            out["jvp_512"][f"{pr}-{mode}"] = jvp_bandwidth(s, torch, nn, pr, mode)
        log(f"[bench] maxwell jvp 512^2 {pr}: {out['jvp_512']}")
        # the Arnoldi JVP (first projection fused) of one GMRES(30) cycle at a field with |E| > 0,
        # without and with the CSLP preconditioner applied to its tangent
        wd = torch.float64 if pr == "f64" else torch.float32
        xf = torch.tensor(0.3 * W.random_vector(nn, 5), dtype=wd, device="cuda")
        rhs = -s.residual(xf)
        for pc in ("none", "cslp"):
            s.set_preconditioner(pc)
            s.gmres(xf, rhs, m=30, tol=1e-30, max_restarts=1)  # warm-up
            s.profile_reset()
            s.profile(True)
            _, info = s.gmres(xf, rhs, m=30, tol=1e-30, max_restarts=1)
            st = s.profile_read()
            s.profile(False)
            j = st["jvp_ad"]
            out["arnoldi_jvp_512"][f"{pr}-{pc}"] = dict(
                launches=j["launches"], avg_us=round(j["ms"] * 1e3 / max(1, j["launches"]), 3),
                gbs=round(j["bytes"] / max(j["ms"], 1e-9) / 1e6, 1), krylov_iters=info["krylov_iters"])
        s.set_preconditioner("none")
        log(f"[bench] maxwell arnoldi jvp 512^2 {pr}: {out['arnoldi_jvp_512']}")
        s.close()
    # the continuation itself runs in the library (jfnk_frequency_sweep): at n^2 to convergence,
    # and at the paper's smallest GPU grid (256^2) with a short Newton cap
    from paper_2605_13378_amd import frequency_sweep

    for ns, cap in ((n, max_newton), (256, 8)):
        for pc in ("none", "cslp"):
            key = ("sweep" if ns == n else f"sweep_{ns}") + ("_cslp" if pc == "cslp" else "")
            specs = [W.maxwell_spec(ns, omega=om) for om in omegas]
            srcs = [W.maxwell_source(ns, omega=om) for om in omegas]
            t0 = time.perf_counter()
            _, infos, failed = frequency_sweep(specs, srcs, "f64", max_newton=cap, precond=pc)
            el = time.perf_counter() - t0
            rows, prev_ok = [], False
            for om, inf in zip(omegas, infos):
                rows.append(dict(omega=om, start="previous" if prev_ok else "born", converged=inf["converged"],
                                 newton_iters=inf["newton_iters"], krylov_iters=inf["krylov_iters"],
                                 final_rel_res=inf["rel_res"][-1]))
                prev_ok = inf["converged"]
            out[key] = dict(grid=ns, max_newton=cap, rows=rows, run_failed=failed, seconds=round(el, 3))
            log(f"[bench] maxwell sweep {ns}^2 precond {pc}: {out[key]}")
    return out


def paper_burgers_rows(torch, steps=100, n=256, budget_s=12.0):
    """The paper's JVP-cost experiment (its Table 1: 256^2 Burgers TGV, 100 time steps) and the
    double shear layer at the same size: per combination of JVP and precision, the average
    event-timed JVP duration, the JVPs' share of the solve time, iterations and completion."""
    import workloads as W
    from paper_2605_13378_amd import Solver

    rows = {}
    for case in ("tgv", "dsl"):
        spec, x0 = W.burgers2d_paper_case(case, n)
        for pr in ("f32", "f64"):
            for mode in ("ad", "fd"):
                s = Solver(spec, pr, m=30)
                x = torch.tensor(x0, dtype=torch.float64, device="cuda")
                s.profile_reset()
                s.profile(True)
                newton = krylov = ok = 0
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                done = 0
                for _ in range(steps):
                    if time.perf_counter() - t0 > budget_s:
                        break  # FD in FP32 stagnates (hundreds of thousands of Krylov iterations)
                    done += 1
                    s.set_previous(x)
                    x, info = s.newton_solve(x, mode=mode, eps_rule="paper")
                    newton += info["newton_iters"]
                    krylov += info["krylov_iters"]
                    ok += 1 if info["rel_res"][-1] <= 100 * (1e-4 if pr == "f32" else 1e-6) else 0
                torch.cuda.synchronize()
                wall_ms = 1e3 * (time.perf_counter() - t0)
                st = s.profile_read()
                s.profile(False)
                j = st["jvp_" + mode]
                rows[f"{case}-{pr}-{mode}"] = dict(
                    steps=done, completed_steps=ok, newton_iters=newton, krylov_iters=krylov,
                    jvp_launches=j["launches"], jvp_avg_us=round(j["ms"] * 1e3 / max(1, j["launches"]), 3),
                    jvp_share_of_solve=round(j["ms"] / wall_ms, 4), solve_ms_per_step=round(wall_ms / done, 3))
                log(f"[bench] burgers2d {n}^2 {case}-{pr}-{mode}: {rows[f'{case}-{pr}-{mode}']}")
                s.close()
    return rows


def cpu_baseline(spec, xp, prec):
    """The oracle, single-threaded, on one full Newton solve of the same workload."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import NewtonOptions, Problem, newton_solve

    p = Problem.from_spec(spec)
    o = NewtonOptions.for_precision(prec, mode="ad", eps_rule="normalized")
    import contextlib

    with (threadpool_limits(1) if threadpool_limits else contextlib.nullcontext()):
        t0 = time.perf_counter()
        _, info = newton_solve(p, xp, o)
        el = time.perf_counter() - t0
    # the latency workload (1D Burgers N=256, FP64, tol_N 1e-10, tol_K 1e-12) on the same core
    import workloads as W

    spec1, xp1, _ = W.config("burgers1d", seed=0)
    p1 = Problem.from_spec(spec1)
    o1 = NewtonOptions.for_precision("f64", mode="ad", tol_newton=1e-10, tol_krylov=1e-12)
    with (threadpool_limits(1) if threadpool_limits else contextlib.nullcontext()):
        newton_solve(p1, xp1, o1)
        t1 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            newton_solve(p1, xp1, o1)
        el1 = (time.perf_counter() - t1) / reps
    return dict(value=round(1.0 / el, 5), unit="Newton solves/s", cores=1, kind="oracle",
                sample=f"1 full Newton solve (AD, {prec.upper()} tolerances, FP64 arithmetic) of the "
                       f"Gray-Scott 1024^2 implicit step; {info.newton_iters} Newton / "
                       f"{info.krylov_iters} GMRES iterations in {el:.1f} s",
                latency_burgers1d_256_us=round(1e6 * el1, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "f16s"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-jvp-rows", action="store_true", help="skip the standalone JVP bandwidth rows")
    ap.add_argument("--no-serving", action="store_true", help="skip the continuous-batching serving run")
    ap.add_argument("--no-latency", action="store_true", help="skip the 1D Burgers N=256 latency rows")
    ap.add_argument("--orth", default="dcgs2", choices=["cgs2", "dcgs2"],
                    help="GMRES Gram-Schmidt form: CGS2 (three passes per Arnoldi step) or DCGS2 (two)")
    ap.add_argument("--no-bicgstab", action="store_true", help="skip the Newton-BiCGSTAB rows")
    ap.add_argument("--no-rd", action="store_true",
                    help="skip the reaction-diffusion and Su-Olson Krylov-method rows")
    ap.add_argument("--no-maxwell", action="store_true", help="skip the Maxwell-Kerr TE rows")
    ap.add_argument("--no-paper-burgers", action="store_true",
                    help="skip the 256^2 Burgers TGV/DSL rows (the paper's JVP-cost experiment)")
    ap.add_argument("--no-kerr-c4", action="store_true",
                    help="skip the Helmholtz-Kerr rows of the default run (64^2 Newton, 1024^2 capped)")
    ap.add_argument("--kerr-newton", action="store_true",
                    help="run the Helmholtz-Kerr 1024^2 Newton completion rows (minutes)")
    ap.add_argument("--completion-seeds", type=int, default=64,
                    help="seeds of the 2D Burgers 2048^2 10-step completion sweep (0: skip)")
    ap.add_argument("--latency-repeats", type=int, default=1000)
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-slots", type=int, default=8)
    ap.add_argument("--serving-budget-gib", type=float, default=16.0)
    ap.add_argument("--cycle-trace", default="", metavar="SIZES",
                    help="only run full GMRES(30) cycles (30 Arnoldi steps, no early stop) on Gray-Scott "
                         "grids of these comma-separated sides, 6 per side, in --precision, for per-step "
                         "kernel traces; prints one JSON line and exits")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="run a plain device copy of MB megabytes 3 times first (HBM counter calibration)")
    args = ap.parse_args()
    global ORTH
    ORTH = args.orth

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the JFNK hot path of this "
              f"package is single-GPU by design", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    if args.cycle_trace:
        from paper_2605_13378_amd import Solver

        wd = torch.float64 if args.precision == "f64" else torch.float32
        done = {}
        for side in (int(v) for v in args.cycle_trace.split(",")):
            spec_c, xp_c, _ = W.config("grayscott", n=side)
            sc = Solver(spec_c, args.precision, m=30)
            sc.set_previous(torch.tensor(xp_c, dtype=torch.float64, device="cuda"))
            sc.set_orthogonalization(args.orth)
            xc = torch.tensor(xp_c, dtype=wd, device="cuda")
            rc = torch.tensor(W.random_vector(len(xp_c), 5), dtype=wd, device="cuda")
            for _ in range(6):
                _, info_c = sc.gmres(xc, rc, m=30, tol=1e-300, max_restarts=1)
            torch.cuda.synchronize()
            done[side] = info_c["krylov_iters"]
            log(f"[bench] cycle trace {side}^2 {args.precision}: {done[side]} steps per cycle")
            sc.close()
        print(json.dumps({"cycle_trace": done, "precision": args.precision, "orth": args.orth}))
        return

    copy_gbs = None
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration << 20
        src_t = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            dst_t.copy_(src_t)
        e1.record()
        torch.cuda.synchronize()
        copy_gbs = round(3 * 2 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        log(f"[bench] copy calibration {args.copy_calibration} MB: {copy_gbs} GB/s (read+write)")
        del src_t, dst_t

    spec, xp, _ = W.config("grayscott", seed=0)
    n = W.n_unknowns(spec)
    prec = args.precision
    x0 = torch.tensor(xp, dtype=torch.float64, device="cuda")

    # ---- headline: AD JVP, working precision `prec` ------------------------
    s = make_solver(spec, prec, xp, torch)
    opts = options_for(prec, "ad")
    log(f"[bench] warmup {args.warmup} solves ({prec}, AD)")
    run_solves(s, x0, torch, args.warmup, opts)
    log(f"[bench] timed {args.steps} solves")
    elapsed, lat, info = run_solves(s, x0, torch, args.steps, opts)
    value = args.steps / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    log(f"[bench] {value:.2f} solves/s, {ms_per_step:.3f} ms/solve, newton {info['newton_iters']}, "
        f"krylov {info['krylov_iters']}, converged {info['converged']}")

    # ---- the same timed region again with HIP events around every kernel ----
    log("[bench] profiled pass (HIP events)")
    s.profile_reset()
    s.profile(True)
    p_el, _, _ = run_solves(s, x0, torch, args.steps, opts)
    stats = s.profile_read()
    s.profile(False)
    total_ms = sum(v["ms"] for v in stats.values())
    dom_name, dom = max(stats.items(), key=lambda kv: kv[1]["ms"])
    dom_avg_us = dom["ms"] * 1e3 / max(1, dom["launches"])
    achieved = dom["bytes"] / (dom["ms"] * 1e-3) / 1e9 if dom["ms"] > 0 else 0.0
    kernels = {k: dict(launches=v["launches"], ms=round(v["ms"], 3),
                       avg_us=round(v["ms"] * 1e3 / max(1, v["launches"]), 3),
                       gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else 0.0,
                       share=round(v["ms"] / total_ms, 4) if total_ms > 0 else 0.0)
               for k, v in stats.items() if v["launches"]}
    bpl = dom["bytes"] / max(1, dom["launches"])
    traffic = measured_traffic(dom_name, bpl, ORTH)
    roofline = dict(bound="hbm", kernel=dom_name, achieved=round(achieved, 1), peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=round(achieved / PEAK_HBM_GBS, 4), traffic=traffic, avg_us=round(dom_avg_us, 3),
                    launches=dom["launches"], bytes_per_launch_avg=bpl)

    # ---- JVP bandwidth: AD vs FD -------------------------------------------
    # "-hbm" rows rotate over >= 1 GiB of distinct operands (the HBM figures);
    # the plain rows re-use one operand set, which the 256 MB last-level cache
    # then largely serves (labelled context, not HBM bandwidth).
    jvp = {}
    for pr in (() if args.no_jvp_rows else ("f32", "f64")):
        sj = s if pr == prec else make_solver(spec, pr, xp, torch)
        for mode in ("ad", "fd"):
            jvp[f"{pr}-{mode}-hot"] = jvp_bandwidth(sj, torch, n, pr, mode)
            jvp[f"{pr}-{mode}-hbm"] = jvp_bandwidth_hbm(torch, spec, xp, None, pr, mode)
            log(f"[bench] jvp {pr}-{mode}: hbm {jvp[f'{pr}-{mode}-hbm']} hot {jvp[f'{pr}-{mode}-hot']}")
        if sj is not s:
            sj.close()

    # ---- JVP bandwidth at the 2D Burgers 2048^2 shape (100-134 MB per call)
    jvp2048 = {}
    spec_b, xp_b, _ = W.config("burgers2d", seed=0)
    n_b = W.n_unknowns(spec_b)
    for pr in (() if args.no_jvp_rows else ("f32", "f64")):
        sb = make_solver(spec_b, pr, xp_b, torch)
        for mode in ("ad", "fd"):
            jvp2048[f"{pr}-{mode}-hot"] = jvp_bandwidth(sb, torch, n_b, pr, mode, reps=100)
            jvp2048[f"{pr}-{mode}-hbm"] = jvp_bandwidth_hbm(torch, spec_b, xp_b, None, pr, mode)
            log(f"[bench] jvp 2048^2 {pr}-{mode}: hbm {jvp2048[f'{pr}-{mode}-hbm']}")
        sb.close()

    # ---- JVP bandwidth on the Helmholtz-Kerr 1024^2 grid (complex64 / complex128)
    jvpkerr = {}
    for pr in (() if args.no_jvp_rows else ("f32", "f64")):
        sk, spec_k = kerr_solver(torch, pr)
        src_k = W.kerr_gaussian_source(1024)
        for mode in ("ad", "fd"):
            jvpkerr[f"{pr}-{mode}-hot"] = jvp_bandwidth(sk, torch, W.n_unknowns(spec_k), pr, mode)
            jvpkerr[f"{pr}-{mode}-hbm"] = jvp_bandwidth_hbm(torch, spec_k, np.zeros(W.n_unknowns(spec_k)), src_k,
                                                            pr, mode)
            log(f"[bench] jvp kerr 1024^2 {pr}-{mode}: hbm {jvpkerr[f'{pr}-{mode}-hbm']}")
        sk.close()

    # ---- plain-copy reference at the vector sizes of those rows -------------
    copy_ref = {}
    for mb in (() if args.no_jvp_rows else (8, 16, 32, 64)):
        copy_ref[f"{mb}MiB"] = copy_ceiling_hbm(torch, mb << 20)
        log(f"[bench] copy reference {mb} MiB: {copy_ref[f'{mb}MiB']}")

    # ---- the same solve with captured restart cycles (HIP graph engine) ----
    graph_row = None if args.no_variants else graph_engine_row(torch, spec, xp, args.steps, prec)
    if graph_row:
        log(f"[bench] graph engine: {graph_row}")

    # ---- variants: AD vs FD, FP64 vs FP32 (solves/s, iterations) -----------
    variants = {}
    if not args.no_variants:
        for pr in ("f32", "f16s", "f64"):
            sv = s if pr == prec else make_solver(spec, pr, xp, torch)
            for mode in ("ad", "fd"):
                o = options_for(pr, mode)
                run_solves(sv, x0, torch, 1, o)
                budget = 8.0
                cnt = 0
                t_all = 0.0
                lat_v = []
                inf = None
                while t_all < budget and cnt < args.steps:
                    el, l1, inf = run_solves(sv, x0, torch, 1, o)
                    t_all += el
                    lat_v += l1
                    cnt += 1
                # one more solve with HIP events on every kernel: the Arnoldi kernels of this
                # variant (for FP16 storage, the JVP whose tangent and projection basis are FP16)
                sv.profile_reset()
                sv.profile(True)
                run_solves(sv, x0, torch, 1, o)
                kst = sv.profile_read()
                sv.profile(False)
                sv.profile_reset()
                vk = {k: dict(launches=v["launches"], avg_us=round(v["ms"] * 1e3 / max(1, v["launches"]), 3),
                              gbs=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9, 1) if v["ms"] > 0 else 0.0,
                              frac=round(v["bytes"] / (v["ms"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4) if v["ms"] > 0 else 0.0)
                      for k, v in kst.items() if v["launches"] and k in ("jvp_ad", "jvp_fd", "dcgs_update", "cgs_b",
                                                                          "cgs_c", "vy")}
                variants[f"{pr}-{mode}"] = dict(solves_per_s=round(cnt / t_all, 3), solves=cnt,
                                                p50_ms=round(1e3 * percentile(lat_v, 0.5), 3),
                                                p99_ms=round(1e3 * percentile(lat_v, 0.99), 3),
                                                newton_iters=inf["newton_iters"], krylov_iters=inf["krylov_iters"],
                                                converged=inf["converged"], final_rel_res=inf["rel_res"][-1],
                                                kernels=vk)
                log(f"[bench] variant {pr}-{mode}: {variants[f'{pr}-{mode}']}")
            if sv is not s:
                sv.close()

    bicg = None
    if not args.no_bicgstab:
        log("[bench] Newton-BiCGSTAB rows (Gray-Scott 1024^2)")
        bicg = bicgstab_rows(torch, spec, xp, x0, args.steps)

    rd = None
    if not args.no_rd:
        log("[bench] reaction-diffusion 512^2 rows (CG / BiCGSTAB / GMRES)")
        rd = rd_rows(torch, args.steps)

    mx = None
    if not args.no_maxwell:
        log("[bench] Maxwell-Kerr TE rows")
        mx = maxwell_rows(torch)

    so = so1 = None
    if not args.no_rd:
        log("[bench] Su-Olson 512^2 rows")
        so = suolson_rows(torch, args.steps)
        so1 = suolson_rows(torch, args.steps, config="suolson1d")

    pb = None
    if not args.no_paper_burgers:
        log("[bench] 256^2 Burgers TGV / DSL rows (100 Crank-Nicolson steps each)")
        pb = paper_burgers_rows(torch)

    c3 = None
    if args.completion_seeds > 0:
        log(f"[bench] completion sweep: 2D Burgers 2048^2, 10 steps, {args.completion_seeds} seeds")
        c3 = completion_c3(torch, args.completion_seeds)

    c4 = None
    if args.kerr_newton:
        log("[bench] Helmholtz-Kerr 1024^2 Newton rows")
        c4 = kerr_newton(torch)
    c4_short = None
    if not args.no_kerr_c4:
        log("[bench] Helmholtz-Kerr rows: 64^2 to convergence, 1024^2 capped at 5 Newton steps")
        c4_short = kerr_c4_rows(torch)

    c1 = None
    if not args.no_latency:
        log(f"[bench] latency rows: 1D Burgers N=256, {args.latency_repeats} repeats")
        c1 = latency_c1(torch, args.latency_repeats, seeds=1000)

    serving = None
    if not args.no_serving:
        log(f"[bench] serving: {args.serving_requests} requests, {args.serving_slots} slots")
        serving = serving_bench(args.serving_requests, args.serving_slots, args.serving_budget_gib)

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline (1 solve)")
        cpu = cpu_baseline(spec, xp, prec)
        log(f"[bench] cpu: {cpu}")
        if serving is not None:
            log("[bench] CPU oracle beside the serving stream")
            serving["cpu_oracle"] = serving_oracle()
            log(f"[bench] serving cpu oracle: {serving['cpu_oracle']}")

    out = {
        "metric": "Newton solves/sec and JVP HBM GB/s, AD vs FD, FP64/FP32/FP16; p99 latency",
        "value": round(value, 3),
        "unit": "Newton solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": CONFIG_NAME, "grid": [1024, 1024], "unknowns": n, "jvp": "ad",
                   "krylov": f"GMRES(30) {args.orth.upper()}, FP64 Givens", "tol_newton": 1e-4 if prec == "f32" else 1e-6,
                   "tol_krylov": 1e-6 if prec == "f32" else 1e-8, "seed": 0},
        "latency_ms": {"p50": round(1e3 * percentile(lat, 0.5), 3), "p99": round(1e3 * percentile(lat, 0.99), 3)},
        "newton_iters": info["newton_iters"],
        "krylov_iters": info["krylov_iters"],
        "roofline": roofline,
        "kernels": kernels,
        "profiled_pass_ms_per_step": round(1e3 * p_el / args.steps, 4),
        "jvp": jvp,
        "jvp_burgers2d_2048": jvp2048,
        "jvp_kerr_1024": jvpkerr,
        "copy_reference_hbm": copy_ref,
        "copy_calibration_gbs": copy_gbs,
        "variants": variants,
        "graph_engine": graph_row,
        "bicgstab_newton": bicg,
        "reaction_diffusion_512": rd,
        "burgers2d_256_tgv_dsl": pb,
        "suolson_512": so,
        "suolson1d_512": so1,
        "maxwell_te": mx,
        "latency_burgers1d_256": c1,
        "completion_burgers2d_2048": c3,
        "kerr_newton_1024": c4,
        "kerr_c4": c4_short,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
