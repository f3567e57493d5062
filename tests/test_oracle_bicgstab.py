"""Pins of the oracle's BiCGSTAB against what mathematics and an independent
implementation fix (no GPU).

* dense solves: the converged iterate's true residual meets the tolerance and
  the iterate matches A^{-1} b within the conditioning bound;
* SciPy's bicgstab (an independent implementation of the same iteration, run
  with the same relative tolerance and no absolute one): same iteration
  count, same iterate to rounding;
* closed forms: J = a I converges at the first half step to b / a;
* a planted breakdown ((r0, J r0) = 0) is reported, not hidden;
* Newton with BiCGSTAB reaches the same root as Newton with GMRES.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import NewtonOptions, Problem, bicgstab_solve, newton_solve


def well_conditioned(n, seed):
    rng = np.random.default_rng(seed)
    return np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)


@pytest.mark.parametrize("n,seed", [(20, 1), (60, 2), (150, 3)])
def test_dense_solve(n, seed):
    A = well_conditioned(n, seed)
    b = np.random.default_rng(seed + 10).standard_normal(n)
    tol = 1e-10
    x, info = bicgstab_solve(lambda v: A @ v, b, tol=tol, maxiter=200)
    assert info.converged and not info.breakdown
    assert np.linalg.norm(b - A @ x) <= 1.0001 * tol * np.linalg.norm(b)
    x_ref = np.linalg.solve(A, b)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - x_ref) <= 2 * cond * tol * np.linalg.norm(x_ref)


@pytest.mark.parametrize("n,seed,tol", [(40, 4, 1e-8), (120, 5, 1e-11)])
def test_matches_scipy_bicgstab(n, seed, tol):
    A = well_conditioned(n, seed)
    b = np.random.default_rng(seed + 20).standard_normal(n)
    count = [0]

    def cb(_x):
        count[0] += 1

    x_sp, flag = spla.bicgstab(A, b, rtol=tol, atol=0.0, maxiter=500, callback=cb)
    assert flag == 0
    x, info = bicgstab_solve(lambda v: A @ v, b, tol=tol, maxiter=500)
    assert info.converged
    # SciPy's callback runs after full iterations only; a half-step stop ends
    # its last iteration without one
    assert info.iters in (count[0], count[0] + 1)
    assert np.linalg.norm(x - x_sp) <= 1e-9 * np.linalg.norm(x_sp)


@pytest.mark.parametrize("a", [2.0, -0.5, 7.25])
def test_scaled_identity_closed_form(a):
    b = np.random.default_rng(7).standard_normal(30)
    x, info = bicgstab_solve(lambda v: a * v, b, tol=1e-12)
    assert info.converged and info.iters == 1
    assert np.allclose(x, b / a, rtol=1e-15, atol=0.0)


def test_breakdown_is_reported():
    A = np.array([[0.0, 1.0], [-1.0, 0.0]])  # skew: (r0, A r0) = 0
    x, info = bicgstab_solve(lambda v: A @ v, np.array([1.0, 0.0]), tol=1e-12)
    assert info.breakdown and not info.converged
    assert not x.any()


def test_zero_rhs_and_cap():
    A = well_conditioned(30, 8)
    x, info = bicgstab_solve(lambda v: A @ v, np.zeros(30))
    assert info.converged and info.iters == 0 and not x.any()
    b = np.ones(30)
    x, info = bicgstab_solve(lambda v: A @ v, b, tol=1e-30, maxiter=3)
    assert not info.converged and info.iters == 3


def test_newton_bicgstab_reaches_gmres_root():
    spec = dict(W.grayscott_spec(24), ny=20)
    xp = W.grayscott_initial(24, 0, ny=20, side_frac=1 / 8, patches=6)
    p = Problem.from_spec(spec)
    og = NewtonOptions.for_precision("f64", tol_newton=1e-10, tol_krylov=1e-12)
    ob = NewtonOptions.for_precision("f64", tol_newton=1e-10, tol_krylov=1e-12, krylov="bicgstab")
    xg, ig = newton_solve(p, xp, og)
    xb, ib = newton_solve(p, xp, ob)
    assert ig.converged and ib.converged
    # ||J^-1|| <= 1 for this diffusive implicit step: both within 1e-10 ||F0|| of the root
    assert np.linalg.norm(xg - xb) <= 2e-10 * ig.f0_norm
    assert ib.lin_iters and all(k >= 1 for k in ib.lin_iters)
