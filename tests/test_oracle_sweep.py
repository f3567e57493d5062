"""Pins of the oracle's frequency continuation (oracle.sweep).

The continuation is control logic around Newton (Section 3.1's outer loop,
Appendix A.4's Born start, Section 3.4's 20% rule).  Pinned here: the first
frequency's first Newton iterate is the Born field (the dense solve of the
system linearized at E = 0); the hand-over of starts and the failure rule,
exactly, with Newton replaced by a stub whose outcomes the test fixes.
"""

import numpy as np
import pytest

import oracle.sweep as SW
import workloads as W
from oracle import NewtonInfo, NewtonOptions, Problem, frequency_sweep, jvp_ad, residual


def test_first_newton_step_from_zero_is_the_born_field():
    n = 8
    spec = W.maxwell_spec(n, omega=3.0)
    p = Problem.from_spec(spec)
    src = W.maxwell_source(n, omega=3.0)
    zero = np.zeros(p.n)
    # dense Jacobian at E = 0 from the (separately pinned) AD JVP, then the Born field
    J = np.stack([jvp_ad(p, zero, e, zero, src)[1] for e in np.eye(p.n)], axis=1)
    born = np.linalg.solve(J, -residual(p, zero, zero, src))
    o = NewtonOptions.for_precision("f64", tol_krylov=1e-12, max_newton=20)
    fields, info = frequency_sweep([p], [src], o, record=True)
    assert info.starts == ["born"]
    x1 = info.steps[0].iterates[1]
    assert info.steps[0].alphas[0] == 1.0
    assert np.linalg.norm(x1 - born) <= 1e-10 * np.linalg.norm(born)
    assert info.converged == [True] and not info.failed
    assert np.linalg.norm(residual(p, fields[0], zero, src)) <= o.tol_newton * info.steps[0].f0_norm


def _stub(outcomes, calls):
    """newton_solve stand-in: records its start and returns start + 1 with the next outcome."""
    it = iter(outcomes)

    def fake(p, x_prev, opts, source=None, x0=None, record=False, perm=None):
        calls.append(x0.copy())
        ok = next(it)
        ni = NewtonInfo()
        ni.converged = ok
        return x0 + 1.0, ni

    return fake


@pytest.mark.parametrize("outcomes,starts,failed", [
    ([True] * 5, ["born", "previous", "previous", "previous", "previous"], False),
    ([True, False, True, True, True], ["born", "previous", "born", "previous", "previous"], False),  # 20%
    ([True, False, False, True, True], ["born", "previous", "born", "born", "previous"], True),  # 40%
    ([False] * 3, ["born", "born", "born"], True),
    ([False], ["born"], True),
    ([True, True, True, True, True, True, True, True, True, False], ["born"] + ["previous"] * 9, False),
])
def test_start_hand_over_and_twenty_percent_rule(monkeypatch, outcomes, starts, failed):
    calls = []
    monkeypatch.setattr(SW, "newton_solve", _stub(outcomes, calls))
    k = len(outcomes)
    spec = W.maxwell_spec(4, omega=2.0)
    probs = [Problem.from_spec(spec)] * k
    fields, info = frequency_sweep(probs, [None] * k, NewtonOptions())
    assert info.starts == starts and info.failed == failed
    assert info.converged == list(outcomes)
    for i, x0 in enumerate(calls):
        # a 'previous' start is the field frequency i-1 returned (its start + 1), a 'born' one zero
        expect = fields[i - 1] if starts[i] == "previous" else np.zeros_like(x0)
        np.testing.assert_array_equal(x0, expect)


@pytest.mark.parametrize("name", ["maxwell16_sweep", "maxwell16_sweep_cslp"])
def test_sweep_summation_order_spread_within_pinned_ceiling(name):
    """The oracle's sweep on the permuted system (summation order only changes): fields and
    Krylov counts move by no more than the ceilings the GPU bounds are derived from, and the
    converged flags and Newton counts do not move at all."""
    import order_spread as OS

    specs, srcs, opts, cx, ck = OS.sweep_case(name)
    probs = [Problem.from_spec(sp) for sp in specs]
    o = NewtonOptions.for_precision("f64", **opts)
    f1, i1 = frequency_sweep(probs, srcs, o)
    perm = np.random.default_rng(3).permutation(probs[0].n)
    f2, i2 = frequency_sweep(probs, srcs, o, perm=perm)
    assert i1.converged == i2.converged == [True] * len(probs)
    assert [s.newton_iters for s in i1.steps] == [s.newton_iters for s in i2.steps]
    for a, b in zip(f1, f2):
        assert np.linalg.norm(a - b) <= cx * np.linalg.norm(a)
    for a, b in zip(i1.steps, i2.steps):
        assert abs(a.krylov_iters - b.krylov_iters) <= ck
