"""Frequency continuation of the Maxwell-Kerr boundary-value problem (oracle).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU leg use this module.

The paper's solver has an outer continuation loop around Newton (Section 3.1):
time for the initial-boundary-value problems, the angular frequency omega for
the time-harmonic Maxwell problem.  For Maxwell the initial guess comes from
the linearized problem (Section 3.2; Appendix A.4: the Born approximation, the
wave equation linearized at E = 0 -- which is exactly the first Newton step
taken from E = 0).  A Maxwell run fails when more than 20% of its frequency
steps do not reach the requested Newton tolerance (Section 3.4).

Reading (the paper does not spell the hand-over out): each frequency starts
from the previous frequency's converged field; the first frequency, and any
frequency after one that did not converge, starts from E = 0 (the Born
guess).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .newton import NewtonInfo, NewtonOptions, newton_solve
from .problems import Problem


@dataclass
class SweepInfo:
    steps: list = field(default_factory=list)  # NewtonInfo per frequency
    starts: list = field(default_factory=list)  # 'born' or 'previous'
    converged: list = field(default_factory=list)
    failed: bool = False  # more than 20% of the frequency steps did not converge


def frequency_sweep(problems: list, sources: list, opts: NewtonOptions, record: bool = False,
                    perm: np.ndarray | None = None):
    """Solve problems[0], problems[1], ... (one per frequency, same unknown count) in
    order with the continuation above; returns (fields, SweepInfo), fields[i] the
    final field of frequency i (its last iterate when it did not converge)."""
    info = SweepInfo()
    fields = []
    prev = None  # converged field of the previous frequency
    for p, src in zip(problems, sources):
        assert isinstance(p, Problem)
        start = np.zeros(p.n) if prev is None else prev
        info.starts.append("born" if prev is None else "previous")
        x, ni = newton_solve(p, np.zeros(p.n), opts, source=src, x0=start, record=record, perm=perm)
        assert isinstance(ni, NewtonInfo)
        info.steps.append(ni)
        info.converged.append(bool(ni.converged))
        fields.append(x)
        prev = x if ni.converged else None
    bad = sum(not c for c in info.converged)
    info.failed = bad > 0.2 * len(info.converged)
    return fields, info
