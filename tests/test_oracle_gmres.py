"""Pins of the oracle's restarted GMRES (paper Section 2: minimal residual over
the Krylov space, restarted; CGS2 Arnoldi; Givens least squares).

Checked against numpy.linalg.solve on dense systems, against
scipy.sparse.linalg.gmres (the paper's own CPU routine) on the same system,
against exact termination in d steps for an operator with d distinct
eigenvalues, and against the structural identities of the Arnoldi process
(orthonormal basis, A V_k = V_{k+1} Hbar_k, Givens estimate = true residual).
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import gmres_solve
from oracle.gmres import back_substitute, givens


def dense_system(n, seed, shift=4.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    b = rng.standard_normal(n)
    return A, b


@pytest.mark.parametrize("m", [60, 7])
def test_matches_dense_solve(m):
    A, b = dense_system(50, 0, shift=3.0)
    x, info = gmres_solve(lambda v: A @ v, b, m=m, tol=1e-12, max_restarts=200)
    assert info.converged
    xs = np.linalg.solve(A, b)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 1e-12 * cond * 10
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b) * 1.0001


def test_agrees_with_scipy_gmres():
    A, b = dense_system(80, 1, shift=2.0)
    x, info = gmres_solve(lambda v: A @ v, b, m=10, tol=1e-10, max_restarts=500)
    xr, flag = spla.gmres(A, b, rtol=1e-10, restart=10, maxiter=500, atol=0.0)
    assert info.converged and flag == 0
    xs = np.linalg.solve(A, b)
    cond = np.linalg.cond(A)
    for sol in (x, xr):
        assert np.linalg.norm(sol - xs) / np.linalg.norm(xs) <= 1e-10 * cond * 10
    assert np.linalg.norm(x - xr) / np.linalg.norm(xs) <= 2e-10 * cond * 10


def test_orthonormal_basis_and_arnoldi_relation():
    A, b = dense_system(40, 2, shift=1.5)
    x, info = gmres_solve(lambda v: A @ v, b, m=25, tol=1e-14, max_restarts=1, record=True)
    k = info.last_k
    V = np.stack(info.last_V[: k + 1], axis=1)
    Vk = V[:, :k]
    np.testing.assert_allclose(V.T @ V, np.eye(k + 1), atol=1e-13)
    np.testing.assert_allclose(A @ Vk, V @ info.last_H, atol=1e-12)


def test_exact_termination_with_few_distinct_eigenvalues():
    rng = np.random.default_rng(3)
    n, d = 60, 4
    S = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n)  # well conditioned, non-normal A
    lam = np.repeat([1.0, 2.5, -3.0, 7.0], n // d)
    A = S @ np.diag(lam) @ np.linalg.inv(S)
    b = rng.standard_normal(n)
    x, info = gmres_solve(lambda v: A @ v, b, m=30, tol=1e-10, max_restarts=2)
    assert info.converged
    assert info.iters <= d
    np.testing.assert_allclose(A @ x, b, atol=1e-8 * np.linalg.norm(b))


def test_givens_estimate_equals_true_residual():
    A, b = dense_system(70, 4, shift=1.2)
    x, info = gmres_solve(lambda v: A @ v, b, m=8, tol=1e-11, max_restarts=300)
    assert info.converged
    # every restart's true residual equals the estimate the previous cycle ended with
    ends = []
    it = 0
    for c in range(info.cycles):
        it += min(8, len(info.est_res) - it)
        ends.append(info.est_res[it - 1])
    for est, true in zip(ends, info.true_res[1:]):
        assert abs(est - true) <= 1e-9 * true + 1e-13 * np.linalg.norm(b)


def test_zero_rhs_and_nonfinite():
    A, b = dense_system(10, 5)
    x, info = gmres_solve(lambda v: A @ v, np.zeros(10))
    assert info.converged and info.iters == 0 and not x.any()
    b[3] = np.nan
    x, info = gmres_solve(lambda v: A @ v, b)
    assert info.nonfinite and not info.converged


def test_restart_cap_reports_not_converged():
    A, b = dense_system(30, 6, shift=0.5)
    x, info = gmres_solve(lambda v: A @ v, b, m=1, tol=1e-12, max_restarts=1)
    assert not info.converged and info.iters == 1 and info.cycles == 1


def test_givens_and_back_substitution_primitives():
    for a, bb in ((3.0, 4.0), (-1.0, 2.0), (0.0, 5.0), (2.0, 0.0)):
        c, s = givens(a, bb)
        r = c * a + s * bb
        assert abs(-s * a + c * bb) <= 1e-15 * (abs(a) + abs(bb))
        assert abs(abs(r) - np.hypot(a, bb)) <= 1e-15 * np.hypot(a, bb)
        assert abs(c * c + s * s - 1.0) <= 1e-15
    rng = np.random.default_rng(7)
    R = np.triu(rng.standard_normal((6, 6))) + 4 * np.eye(6)
    g = rng.standard_normal(6)
    np.testing.assert_allclose(R @ back_substitute(R, g), g, atol=1e-14)


def test_happy_breakdown_on_invariant_subspace():
    # rhs in a 3-dimensional invariant subspace of a diagonal operator: with a
    # zero tolerance only the breakdown test can end the first cycle, at step 3
    n = 20
    lam = np.linspace(1, 3, n)
    b = np.zeros(n)
    b[[2, 7, 11]] = [1.0, -2.0, 0.5]
    x, info = gmres_solve(lambda v: lam * v, b, m=10, tol=0.0, max_restarts=1)
    assert info.iters == 3 and info.breakdowns == 1
    np.testing.assert_allclose(lam * x, b, atol=1e-14)


def test_pde_operator_solution_matches_dense():
    # GMRES on a JVP operator assembled densely from the oracle's AD JVP
    from oracle import Problem, jvp_ad

    spec = W.grayscott_spec(6, D=4e-3, Dv=2e-3, dt=1.0, h=0.06)
    p = Problem.from_spec(spec)
    x = W.grayscott_initial(6, seed=3, side_frac=1 / 3, patches=2)
    J = np.stack([jvp_ad(p, x, e, x)[1] for e in np.eye(p.n)], axis=1)
    rhs = W.random_vector(p.n, 8)
    sol, info = gmres_solve(lambda v: jvp_ad(p, x, v, x)[1], rhs, m=30, tol=1e-13)
    assert info.converged
    np.testing.assert_allclose(sol, np.linalg.solve(J, rhs), rtol=0, atol=1e-11 * np.abs(sol).max())
