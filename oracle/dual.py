"""Forward-mode dual numbers over NumPy arrays (oracle; test infrastructure).

A ``Dual`` carries a primal value and a tangent.  Running the *same* residual
function on ``Dual(x, v)`` returns ``Dual(F(x), J(x) v)``: this is the
forward-mode JVP of the paper's Section 2 (the ``jvp`` pair of the AD JVP
equation), obtained by differentiating the implemented discrete residual
operation by operation (product rule for ``*``, linearity for ``+``, ``-``,
shifts and scalar division).
"""

from __future__ import annotations

import numpy as np


class Dual:
    """Value + tangent pair; arithmetic follows the rules of differentiation."""

    __slots__ = ("val", "tan")
    # Make NumPy hand mixed ndarray/Dual operations to the Dual's reflected methods.
    __array_ufunc__ = None

    def __init__(self, val, tan):
        self.val = val
        self.tan = tan

    # sum rule
    def __add__(self, o):
        if isinstance(o, Dual):
            return Dual(self.val + o.val, self.tan + o.tan)
        return Dual(self.val + o, self.tan)

    def __radd__(self, o):
        return Dual(o + self.val, self.tan)

    def __sub__(self, o):
        if isinstance(o, Dual):
            return Dual(self.val - o.val, self.tan - o.tan)
        return Dual(self.val - o, self.tan)

    def __rsub__(self, o):
        return Dual(o - self.val, -self.tan)

    def __neg__(self):
        return Dual(-self.val, -self.tan)

    # product rule
    def __mul__(self, o):
        if isinstance(o, Dual):
            return Dual(self.val * o.val, self.val * o.tan + self.tan * o.val)
        return Dual(self.val * o, self.tan * o)

    def __rmul__(self, o):
        return Dual(o * self.val, o * self.tan)

    # quotient rule
    def __truediv__(self, o):
        if isinstance(o, Dual):
            return Dual(self.val / o.val, (self.tan * o.val - self.val * o.tan) / (o.val * o.val))
        return Dual(self.val / o, self.tan / o)

    # structural operations act on both parts alike
    def __getitem__(self, idx):
        return Dual(self.val[idx], self.tan[idx])

    def reshape(self, *shape):
        return Dual(self.val.reshape(*shape), self.tan.reshape(*shape))

    def ravel(self):
        return Dual(self.val.ravel(), self.tan.ravel())

    @property
    def shape(self):
        return self.val.shape


def roll(a, shift: int, axis: int):
    """``np.roll`` that also accepts a Dual (the shift is linear)."""
    if isinstance(a, Dual):
        return Dual(np.roll(a.val, shift, axis=axis), np.roll(a.tan, shift, axis=axis))
    return np.roll(a, shift, axis=axis)


def concatenate(parts):
    """Concatenate flat arrays or Duals."""
    if any(isinstance(p, Dual) for p in parts):
        vals = [p.val if isinstance(p, Dual) else p for p in parts]
        tans = [p.tan if isinstance(p, Dual) else np.zeros_like(p) for p in parts]
        return Dual(np.concatenate(vals), np.concatenate(tans))
    return np.concatenate(parts)


def stack_last(parts):
    """Stack along a new last axis (arrays or Duals)."""
    if any(isinstance(p, Dual) for p in parts):
        vals = [p.val if isinstance(p, Dual) else p for p in parts]
        tans = [p.tan if isinstance(p, Dual) else np.zeros_like(p) for p in parts]
        return Dual(np.stack(vals, axis=-1), np.stack(tans, axis=-1))
    return np.stack(parts, axis=-1)
