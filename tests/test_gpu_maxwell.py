"""GPU parity of the paper-form 2D TE Maxwell-Kerr problem (Appendix A.4).

Element-wise residual/JVP parity runs in test_gpu_kernels (the Maxwell rows,
incl. 512^2); here: the guard (the AD JVP at E = 0 is finite and equals the
oracle's Born operator), and Newton from E = 0 (the first step is the Born
solve) per iterate against the oracle on a 16 x 16 grid.  The unpreconditioned
GMRES(30) needs hundreds of restart cycles per step on this indefinite
curl-curl operator; each Newton correction is fixed only to the Krylov
tolerance (1e-8 relative residual) times the conditioning of J, and two
implementations that sum in different orders stop at different points inside
that band.  The bounds are therefore FACTOR times the oracle's own spread
under a change of summation order alone (order_spread, pinned on the CPU);
on 4 x 4 and 6 x 6 grids, where GMRES reaches a 1e-13 tolerance in a few
dozen steps, the iterates are compared at the 1e-12 contract.  The
frequency continuation runs against the oracle's sweep the same way.
"""

import numpy as np
import pytest

import workloads as W
from gpu_cases import dev, gpu_available, host, wdtype
from oracle import NewtonOptions, Problem, jvp_ad
from test_gpu_solver import compare_newton, solver

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not gpu_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 1e-5)])
def test_maxwell_guard_born_operator(prec, tol):
    spec, x0, src = W.config("maxwell", n=96)
    p = Problem.from_spec(spec)
    v = W.random_vector(p.n, 8)
    s = solver(spec, prec, x0, src)
    jv = host(s.jvp(dev(np.zeros(p.n), wdtype(prec)), dev(v, wdtype(prec)), mode="ad"))
    _, ref = jvp_ad(p, np.zeros(p.n), v, None, src)
    assert np.all(np.isfinite(jv))
    assert np.max(np.abs(jv - ref)) <= tol * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("orth", ["dcgs2", "cgs2"])
def test_newton_maxwell_from_born(orth):
    # bounds: FACTOR times the oracle's own summation-order spread on this case
    # (order_spread "maxwell16": rho 1e-9, x 2e-8 measured, ceilings 2e-9 / 4e-8)
    import order_spread as OS

    spec, xp, src, opts, _, _, _ = OS.case("maxwell16")
    tol, tol_x = OS.gpu_bounds("maxwell16")
    info, ref = compare_newton(spec, xp, src, "f64", "ad", tol, tol_x=tol_x, orth=orth, krylov_slack=0.1, **opts)
    assert info["converged"]


@pytest.mark.parametrize("pre", ["none", "cslp"])
@pytest.mark.parametrize("n", [4, 6])
@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_newton_maxwell_tiny_grid_at_contract_bound(n, pre, prec, tol):
    """On 4 x 4 and 6 x 6 node grids GMRES reaches a 1e-13 Krylov tolerance in a few dozen
    steps and the oracle's iterates are independent of summation order to 1e-13
    (test_oracle_summation_order): every Newton iterate at the contract bound, FP64 and FP32,
    with and without the CSLP preconditioner."""
    spec = W.maxwell_spec(n, omega=2.5)
    src = W.maxwell_source(n, omega=2.5)
    kw = dict(tol_krylov=1e-13, tol_newton=1e-10) if prec == "f64" else dict(tol_krylov=1e-6)
    # at a 1e-13 Krylov tolerance the stopping step of a solve moves with summation order
    # (the oracle against itself: up to 11 steps of ~60 on 6 x 6; plain CGS2 against the
    # delayed form: 11 of 45), the iterates do not
    info, ref = compare_newton(spec, np.zeros(4 * n * n), src, prec, "ad", tol, precond=pre, orth="dcgs2",
                               max_newton=20, krylov_slack=0.3, **kw)
    assert info["converged"]


@pytest.mark.parametrize("name", ["maxwell16_sweep", "maxwell16_sweep_cslp"])
def test_frequency_sweep_matches_oracle(name):
    """jfnk_frequency_sweep against the oracle's sweep (Born start, continuation from each
    converged field, the 20% run rule): the same converged flags, Newton counts and run
    outcome, every frequency's field within FACTOR times the oracle's own summation-order
    spread (order_spread.SWEEP_CASES), Krylov counts within the same multiple of theirs."""
    import order_spread as OS
    from oracle import frequency_sweep as oracle_sweep
    from paper_2605_13378_amd import frequency_sweep

    specs, srcs, opts, _, _ = OS.sweep_case(name)
    tol_x, kslack = OS.sweep_gpu_bounds(name)
    fields, infos, failed = frequency_sweep(specs, srcs, "f64", **opts)
    probs = [Problem.from_spec(sp) for sp in specs]
    ref, ri = oracle_sweep(probs, srcs, NewtonOptions.for_precision("f64", **opts))
    assert failed == ri.failed
    assert [i["converged"] for i in infos] == ri.converged
    assert [i["newton_iters"] for i in infos] == [s.newton_iters for s in ri.steps]
    for k, (f, r) in enumerate(zip(fields, ref)):
        assert np.linalg.norm(f - r) <= tol_x * np.linalg.norm(r), (k, np.linalg.norm(f - r) / np.linalg.norm(r))
    for i, s in zip(infos, ri.steps):
        assert abs(i["krylov_iters"] - s.krylov_iters) <= kslack, (i["krylov_iters"], s.krylov_iters)


def test_frequency_sweep_failure_hand_over():
    """A Newton cap of 1 makes every frequency fail: each then starts from the Born guess, so
    every field equals that frequency's own one-step solve from E = 0, and the run fails."""
    from paper_2605_13378_amd import frequency_sweep

    specs = [W.maxwell_spec(8, omega=om) for om in (2.5, 3.0, 3.5)]
    srcs = [W.maxwell_source(8, omega=om) for om in (2.5, 3.0, 3.5)]
    fields, infos, failed = frequency_sweep(specs, srcs, "f64", max_newton=1)
    assert failed and not any(i["converged"] for i in infos)
    for k in range(3):
        alone, ia, _ = frequency_sweep(specs[k:k + 1], srcs[k:k + 1], "f64", max_newton=1)
        assert np.array_equal(alone[0], fields[k]) and ia[0]["krylov_iters"] == infos[k]["krylov_iters"]
