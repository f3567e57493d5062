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


# ---------------------------------------------------------------------------
# Arnoldi with the second Gram-Schmidt pass delayed by one step ('dcgs2'):
# the same basis and Hessenberg matrix as CGS2 in exact arithmetic.
# ---------------------------------------------------------------------------


@pytest.mark.parametrize("m,seed", [(25, 2), (8, 9)])
def test_dcgs2_single_cycle_equals_cgs2(m, seed):
    A, b = dense_system(40, seed, shift=1.5)
    _, i1 = gmres_solve(lambda v: A @ v, b, m=m, tol=1e-30, max_restarts=1, record=True)
    _, i2 = gmres_solve(lambda v: A @ v, b, m=m, tol=1e-30, max_restarts=1, record=True, orth="dcgs2")
    assert i1.last_k == i2.last_k == m
    np.testing.assert_allclose(i2.last_H, i1.last_H, rtol=0, atol=1e-13 * np.abs(i1.last_H).max())
    V1 = np.stack(i1.last_V, axis=1)
    V2 = np.stack(i2.last_V, axis=1)
    assert V2.shape == V1.shape == (40, m + 1)
    np.testing.assert_allclose(V2, V1, rtol=0, atol=1e-13)
    np.testing.assert_allclose(V2.T @ V2, np.eye(m + 1), atol=1e-13)
    np.testing.assert_allclose(A @ V2[:, :m], V2 @ i2.last_H, atol=1e-12)


@pytest.mark.parametrize("m", [60, 7])
def test_dcgs2_matches_dense_solve_and_cgs2_counts(m):
    A, b = dense_system(50, 0, shift=3.0)
    x1, i1 = gmres_solve(lambda v: A @ v, b, m=m, tol=1e-12, max_restarts=200)
    x2, i2 = gmres_solve(lambda v: A @ v, b, m=m, tol=1e-12, max_restarts=200, orth="dcgs2")
    assert i2.converged and i2.iters == i1.iters and i2.cycles == i1.cycles
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x2 - xs) / np.linalg.norm(xs) <= 1e-12 * np.linalg.cond(A) * 10
    assert np.linalg.norm(b - A @ x2) <= 1e-12 * np.linalg.norm(b) * 1.0001


def test_dcgs2_agrees_with_scipy_gmres():
    A, b = dense_system(80, 1, shift=2.0)
    x, info = gmres_solve(lambda v: A @ v, b, m=10, tol=1e-10, max_restarts=500, orth="dcgs2")
    xr, flag = spla.gmres(A, b, rtol=1e-10, restart=10, maxiter=500, atol=0.0)
    assert info.converged and flag == 0
    cond = np.linalg.cond(A)
    assert np.linalg.norm(x - xr) / np.linalg.norm(xr) <= 2e-10 * cond * 10


def test_dcgs2_happy_breakdown_and_exact_termination():
    n = 20
    lam = np.linspace(1, 3, n)
    b = np.zeros(n)
    b[[2, 7, 11]] = [1.0, -2.0, 0.5]
    x, info = gmres_solve(lambda v: lam * v, b, m=10, tol=0.0, max_restarts=1, orth="dcgs2")
    # the third column ends the cycle: the reorthogonalized norm is 0 to rounding, so the
    # estimate is exactly 0 (a tolerance stop at tol = 0) or the breakdown test fires
    assert info.iters == 3 and (info.breakdowns == 1 or info.est_res[-1] == 0.0)
    np.testing.assert_allclose(lam * x, b, atol=1e-14)


def test_dcgs2_keeps_orthogonality_where_one_pass_loses_it():
    # clustered spectrum: after five steps the Krylov space holds the clusters and each new
    # product is nearly in its span, so a single Gram-Schmidt pass loses orthogonality at the
    # 1e-9 level; the delayed second pass must restore it to rounding
    n, m = 200, 12
    rng = np.random.default_rng(4)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([1.0, 2.0, 3.0, 5.0, 8.0], n // 5) + 1e-7 * rng.standard_normal(n)
    A = (Q * lam) @ Q.T
    b = rng.standard_normal(n)
    _, info = gmres_solve(lambda v: A @ v, b, m=m, tol=0.0, max_restarts=1, record=True, orth="dcgs2")
    k = info.last_k
    assert k == m and len(info.last_V) == m + 1
    V = np.stack(info.last_V, axis=1)
    assert np.abs(V.T @ V - np.eye(m + 1)).max() <= 1e-13
    assert np.abs(A @ V[:, :m] - V @ info.last_H).max() <= 1e-13 * lam.max()
    # one pass alone (the first projection only) does lose it here
    W1 = [b / np.linalg.norm(b)]
    for j in range(m):
        w = A @ W1[j]
        w = w - sum(np.dot(q, w) * q for q in W1)
        W1.append(w / np.linalg.norm(w))
    W1 = np.stack(W1, axis=1)
    assert np.abs(W1.T @ W1 - np.eye(m + 1)).max() > 1e-11


def test_dcgs2_zero_rhs_nonfinite_and_cap():
    A, b = dense_system(10, 5)
    x, info = gmres_solve(lambda v: A @ v, np.zeros(10), orth="dcgs2")
    assert info.converged and info.iters == 0 and not x.any()
    A2, b2 = dense_system(30, 6, shift=0.5)
    x, info = gmres_solve(lambda v: A2 @ v, b2, m=1, tol=1e-12, max_restarts=1, orth="dcgs2")
    assert not info.converged and info.iters == 1 and info.cycles == 1
    x1, _ = gmres_solve(lambda v: A2 @ v, b2, m=1, tol=1e-12, max_restarts=1)
    np.testing.assert_allclose(x, x1, rtol=1e-14)
    b[3] = np.nan
    x, info = gmres_solve(lambda v: A @ v, b, orth="dcgs2")
    assert info.nonfinite and not info.converged


def test_dcgs2_pde_operator_matches_cgs2():
    from oracle import Problem, jvp_ad

    spec = W.grayscott_spec(12, D=4e-3, Dv=2e-3, dt=1.0, h=0.06)
    p = Problem.from_spec(spec)
    x = W.grayscott_initial(12, seed=3, side_frac=1 / 3, patches=2)
    rhs = W.random_vector(p.n, 8)
    mv = lambda v: jvp_ad(p, x, v, x)[1]  # noqa: E731
    s1, i1 = gmres_solve(mv, rhs, m=10, tol=1e-12, max_restarts=50)
    s2, i2 = gmres_solve(mv, rhs, m=10, tol=1e-12, max_restarts=50, orth="dcgs2")
    assert i1.converged and i2.converged and i1.iters == i2.iters
    assert np.linalg.norm(s1 - s2) <= 1e-11 * np.linalg.norm(s1)
