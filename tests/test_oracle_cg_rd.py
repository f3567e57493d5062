"""Pins of the oracle's conjugate gradients and of the scalar reaction-diffusion
residual against what mathematics and independent implementations fix (no GPU).

Reaction-diffusion (u_t = D Lap u - u^3, homogeneous Dirichlet, theta scheme):
* closed form: grid sine modes vanish on the boundary nodes and are
  eigenvectors of the discrete Dirichlet Laplacian with eigenvalue
  -(4/h^2) sin^2(a pi h / 2) per direction, so F is known elementwise;
* boundary nodes are identity rows (F = u there);
* the AD Jacobian equals the hand-derived I + theta dt (-D L + 3 diag(u^2)) on
  the interior rows, and its interior block is symmetric positive definite.

CG:
* dense SPD solves; SciPy's cg (independent implementation, same rtol and no
  atol): same iteration count, same iterate to rounding;
* closed forms: J = a I converges in one iteration to b / a; a matrix with k
  distinct eigenvalues converges in exactly k iterations;
* the J-norm of the error decreases monotonically (CG's optimality);
* (p, J p) <= 0 (indefinite J) is reported as a breakdown;
* Newton with CG reaches the same reaction-diffusion root as Newton with GMRES.
"""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import NewtonOptions, Problem, cg_solve, jvp_ad, newton_solve, residual


def rd_grid(nx, ny):
    spec = W.rd2d_spec(nx, D=0.01, ny=ny)
    return spec, Problem.from_spec(spec)


def sine_mode(nx, ny, a, b, amp):
    x = np.linspace(0.0, 1.0, nx)[None, :]
    y = np.linspace(0.0, 1.0, ny)[:, None]
    return (amp * np.sin(a * np.pi * x) * np.sin(b * np.pi * y)).ravel()


def dirichlet_eig(a, b, hx, hy):
    return -(4.0 / hx ** 2) * np.sin(a * np.pi * hx / 2) ** 2 - (4.0 / hy ** 2) * np.sin(b * np.pi * hy / 2) ** 2


@pytest.mark.parametrize("nx,ny,theta", [(17, 13, 0.5), (32, 32, 1.0), (9, 21, 0.5)])
def test_rd_residual_sine_modes_closed_form(nx, ny, theta):
    spec, _ = rd_grid(nx, ny)
    spec["theta"] = theta
    p = Problem.from_spec(spec)
    u = sine_mode(nx, ny, 2, 3, 0.8)
    un = sine_mode(nx, ny, 1, 1, 1.3)
    lu = dirichlet_eig(2, 3, p.hx, p.hy)
    ln = dirichlet_eig(1, 1, p.hx, p.hy)
    N_u = -p.D * lu * u + u ** 3
    N_n = -p.D * ln * un + un ** 3
    expect = u - un + p.dt * (theta * N_u + (1 - theta) * N_n)
    m = np.zeros((ny, nx))
    m[1:-1, 1:-1] = 1.0
    m = m.ravel()
    expect = m * expect  # the modes vanish on the boundary nodes
    got = residual(p, u, un)
    assert np.max(np.abs(got - expect)) <= 1e-13 * max(1.0, np.max(np.abs(expect)))


def test_rd_boundary_rows_are_identity():
    spec, p = rd_grid(12, 10)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(p.n)
    un = rng.standard_normal(p.n)
    F = residual(p, u, un).reshape(p.ny, p.nx)
    U = u.reshape(p.ny, p.nx)
    for edge in (np.s_[0, :], np.s_[-1, :], np.s_[:, 0], np.s_[:, -1]):
        assert np.array_equal(F[edge], U[edge])


def hand_jacobian(p, u):
    n = p.n
    J = np.eye(n)
    c = p.theta * p.dt
    for j in range(1, p.ny - 1):
        for i in range(1, p.nx - 1):
            k = j * p.nx + i
            J[k, k] = 1.0 + c * (p.D * (2 / p.hx ** 2 + 2 / p.hy ** 2) + 3 * u[k] ** 2)
            J[k, k - 1] = J[k, k + 1] = -c * p.D / p.hx ** 2
            J[k, k - p.nx] = J[k, k + p.nx] = -c * p.D / p.hy ** 2
    return J


def test_rd_ad_jacobian_is_the_hand_derived_spd_matrix():
    spec, p = rd_grid(7, 6)
    u = np.random.default_rng(9).uniform(-1.5, 1.5, p.n)
    un = W.random_vector(p.n, 4)
    J = np.column_stack([jvp_ad(p, u, e, un)[1] for e in np.eye(p.n)])
    H = hand_jacobian(p, u)
    assert np.max(np.abs(J - H)) <= 1e-14 * np.max(np.abs(H))
    inner = np.zeros((p.ny, p.nx), bool)
    inner[1:-1, 1:-1] = True
    idx = np.flatnonzero(inner.ravel())
    B = J[np.ix_(idx, idx)]
    assert np.array_equal(B, B.T)
    assert np.linalg.eigvalsh(B).min() > 0.0


def spd(n, seed, lo=0.5, hi=20.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * rng.uniform(lo, hi, n)) @ Q.T


@pytest.mark.parametrize("n,seed", [(20, 1), (80, 2), (200, 3)])
def test_cg_dense_spd_solve(n, seed):
    A = spd(n, seed)
    b = np.random.default_rng(seed + 10).standard_normal(n)
    tol = 1e-10
    x, info = cg_solve(lambda v: A @ v, b, tol=tol, maxiter=500)
    assert info.converged and not info.breakdown
    assert np.linalg.norm(b - A @ x) <= 1.0001 * tol * np.linalg.norm(b) + 1e-14 * np.linalg.norm(b)
    x_ref = np.linalg.solve(A, b)
    assert np.linalg.norm(x - x_ref) <= 2 * np.linalg.cond(A) * tol * np.linalg.norm(x_ref)


@pytest.mark.parametrize("n,seed,tol", [(60, 4, 1e-8), (150, 5, 1e-11)])
def test_cg_matches_scipy(n, seed, tol):
    A = spd(n, seed)
    b = np.random.default_rng(seed + 20).standard_normal(n)
    count = [0]

    def cb(_x):
        count[0] += 1

    x_sp, flag = spla.cg(A, b, rtol=tol, atol=0.0, maxiter=1000, callback=cb)
    assert flag == 0
    x, info = cg_solve(lambda v: A @ v, b, tol=tol, maxiter=1000)
    assert info.converged and info.iters == count[0]
    assert np.linalg.norm(x - x_sp) <= 1e-10 * np.linalg.norm(x_sp)


@pytest.mark.parametrize("a", [3.0, 0.25])
def test_cg_scaled_identity(a):
    b = np.random.default_rng(6).standard_normal(25)
    x, info = cg_solve(lambda v: a * v, b, tol=1e-12)
    assert info.converged and info.iters == 1
    assert np.allclose(x, b / a, rtol=1e-15, atol=0.0)


def test_cg_terminates_in_as_many_iterations_as_distinct_eigenvalues():
    d = np.repeat([1.0, 2.0, 5.0], [10, 7, 13])
    b = np.random.default_rng(7).standard_normal(d.size)
    x, info = cg_solve(lambda v: d * v, b, tol=1e-12, maxiter=50)
    assert info.converged and info.iters == 3
    assert info.res[1] > 1e-3 * np.linalg.norm(b)  # not before the third
    assert np.allclose(x, b / d, rtol=1e-12)


def test_cg_error_energy_norm_decreases():
    A = spd(60, 11, lo=0.1, hi=50.0)
    b = np.random.default_rng(12).standard_normal(60)
    xs = np.linalg.solve(A, b)
    errs = []
    for k in range(1, 25):
        x, _ = cg_solve(lambda v: A @ v, b, tol=0.0, maxiter=k)
        e = x - xs
        errs.append(float(e @ A @ e))
    assert all(b2 < a2 for a2, b2 in zip(errs, errs[1:]))


def test_cg_reports_indefinite_breakdown():
    x, info = cg_solve(lambda v: np.array([1.0, -1.0]) * v, np.array([1.0, 1.0]), tol=1e-12)
    assert info.breakdown and not info.converged and not x.any()
    x, info = cg_solve(lambda v: np.array([1.0, -2.0]) * v, np.array([1.0, 1.0]), tol=1e-12)
    assert info.breakdown and not info.converged


def test_cg_zero_rhs_and_cap():
    A = spd(30, 13)
    x, info = cg_solve(lambda v: A @ v, np.zeros(30))
    assert info.converged and info.iters == 0 and not x.any()
    x, info = cg_solve(lambda v: A @ v, np.ones(30), tol=1e-30, maxiter=4)
    assert not info.converged and info.iters == 4


def test_newton_cg_reaches_gmres_root_on_reaction_diffusion():
    spec = W.rd2d_spec(24, ny=20)
    xp = W.rd2d_initial(24, 0, ny=20)
    p = Problem.from_spec(spec)
    og = NewtonOptions.for_precision("f64", tol_newton=1e-10, tol_krylov=1e-12)
    oc = NewtonOptions.for_precision("f64", tol_newton=1e-10, tol_krylov=1e-12, krylov="cg")
    xg, ig = newton_solve(p, xp, og)
    xc, ic = newton_solve(p, xp, oc)
    assert ig.converged and ic.converged
    # SPD with eigenvalues >= 1 (||J^-1|| <= 1): both within 1e-10 ||F0|| of the root
    assert np.linalg.norm(xg - xc) <= 2e-10 * ig.f0_norm
    assert ic.lin_iters and all(k >= 1 for k in ic.lin_iters)
