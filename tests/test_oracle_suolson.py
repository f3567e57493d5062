"""Pins of the oracle's Su-Olson residual (Appendix A.2) against closed forms (no GPU).

* grid sine modes (eigenvectors of the discrete Dirichlet Laplacian) on both
  fields give F elementwise, with and without the source;
* boundary nodes of both fields are identity rows;
* the AD Jacobian is the hand-derived constant matrix
  I + theta dt [[-(1/3) L + I, -I], [-xi I, xi I]] on the interior rows,
  whatever the state (the system is affine);
* the FD difference quotient equals the AD product up to rounding (affine
  residual: no truncation term);
* Newton converges in one iteration (up to the Krylov tolerance).
"""

import numpy as np
import pytest

import workloads as W
from oracle import EPS_MACH, NewtonOptions, Problem, fd_step, jvp_ad, jvp_fd, newton_solve, residual


def grid(nx, ny, xi=0.1, theta=0.5):
    spec = W.suolson_spec(nx, xi=xi, theta=theta, ny=ny)
    return spec, Problem.from_spec(spec)


def mode(p, a, b, amp):
    x = np.linspace(0.0, 1.0, p.nx)[None, :]
    y = np.linspace(0.0, 1.0, p.ny)[:, None]
    return (amp * np.sin(a * np.pi * x) * np.sin(b * np.pi * y)).ravel()


def eig(p, a, b):
    # the grid spans L = hx (nx - 1); modes sin(a pi x'), x' = x / L, vanish on the boundary nodes
    tx = a * np.pi / (p.nx - 1)
    ty = b * np.pi / (p.ny - 1)
    return -(4.0 / p.hx ** 2) * np.sin(tx / 2) ** 2 - (4.0 / p.hy ** 2) * np.sin(ty / 2) ** 2


def inner(p):
    m = np.zeros((p.ny, p.nx))
    m[1:-1, 1:-1] = 1.0
    return np.tile(m.ravel(), 2)


@pytest.mark.parametrize("nx,ny,theta,with_source", [(17, 13, 0.5, False), (24, 24, 1.0, True), (9, 21, 0.5, True)])
def test_suolson_sine_modes_closed_form(nx, ny, theta, with_source):
    spec, p = grid(nx, ny, xi=0.3, theta=theta)
    lu = eig(p, 2, 3)
    ln = eig(p, 1, 2)
    U, V = mode(p, 2, 3, 0.8), mode(p, 2, 3, -0.4)
    Un, Vn = mode(p, 1, 2, 1.1), mode(p, 1, 2, 0.6)
    x = np.concatenate([U, V])
    xn = np.concatenate([Un, Vn])
    N = np.concatenate([-(lu / 3.0) * U + (U - V), -p.xi * (U - V)])
    Nn = np.concatenate([-(ln / 3.0) * Un + (Un - Vn), -p.xi * (Un - Vn)])
    src = None
    expect = x - xn + p.dt * (theta * N + (1 - theta) * Nn)
    if with_source:
        Q = mode(p, 1, 1, 2.0)
        src = np.concatenate([Q, np.zeros_like(Q)])
        expect = expect - p.dt * src
    expect = inner(p) * expect  # every field vanishes on the boundary nodes
    got = residual(p, x, xn, src)
    assert np.max(np.abs(got - expect)) <= 1e-13 * max(1.0, np.abs(expect).max())


def test_suolson_boundary_rows_are_identity():
    spec, p = grid(11, 9)
    rng = np.random.default_rng(2)
    x, xn, s = rng.standard_normal((3, p.n))
    F = residual(p, x, xn, s)
    m = inner(p)
    assert np.array_equal(F[m == 0], x[m == 0])


def test_suolson_jacobian_is_the_constant_hand_derived_matrix():
    spec, p = grid(6, 5, xi=0.25)
    n1 = p.nx * p.ny
    c = p.theta * p.dt
    H = np.eye(p.n)
    for j in range(1, p.ny - 1):
        for i in range(1, p.nx - 1):
            k = j * p.nx + i
            H[k, k] = 1.0 + c * ((2 / p.hx ** 2 + 2 / p.hy ** 2) / 3.0 + 1.0)
            H[k, k - 1] = H[k, k + 1] = -c / (3.0 * p.hx ** 2)
            H[k, k - p.nx] = H[k, k + p.nx] = -c / (3.0 * p.hy ** 2)
            H[k, n1 + k] = -c
            H[n1 + k, k] = -c * p.xi
            H[n1 + k, n1 + k] = 1.0 + c * p.xi
    for seed in (0, 1):
        x = W.random_vector(p.n, 10 + seed, 3.0)
        J = np.column_stack([jvp_ad(p, x, e, x)[1] for e in np.eye(p.n)])
        assert np.max(np.abs(J - H)) <= 1e-14 * np.abs(H).max()


@pytest.mark.parametrize("rule", ["paper", "normalized"])
def test_suolson_fd_equals_ad_up_to_rounding(rule):
    spec, x0, src = W.config("suolson", n=40)
    p = Problem.from_spec(spec)
    v = W.random_vector(p.n, 4)
    eps = fd_step(rule, EPS_MACH["f64"], x0, v)
    F, ja = jvp_ad(p, x0, v, x0, src)
    jf = jvp_fd(p, x0, v, eps, x0, src)
    S = max(1.0, np.abs(F).max(), np.abs(x0).max())
    assert np.abs(jf - ja).max() <= 32 * EPS_MACH["f64"] / 2 * S / eps * (1 + np.abs(v).max())


def test_suolson_newton_one_step():
    spec, x0, src = W.config("suolson", n=32)
    p = Problem.from_spec(spec)
    o = NewtonOptions.for_precision("f64", tol_krylov=1e-11, tol_newton=1e-9)
    x, info = newton_solve(p, x0, o, source=src)
    assert info.converged and info.newton_iters == 1
    assert info.rel_res[1] <= 1e-10


# The classic 1D-profile configuration: rows periodic (hy = L / ny), the first
# and last columns Dirichlet nodes.


def grid_py(nx, ny, xi=0.1, theta=0.5):
    spec = W.suolson_spec(nx, xi=xi, theta=theta, ny=ny, periodic_y=True)
    return spec, Problem.from_spec(spec)


def mode_py(p, a, b, amp, phase=0.3):
    # Dirichlet sine in x times a periodic Fourier mode in y
    x = np.linspace(0.0, 1.0, p.nx)[None, :]
    jy = np.arange(p.ny)[:, None]
    return (amp * np.sin(a * np.pi * x) * np.cos(2.0 * np.pi * b * jy / p.ny + phase)).ravel()


def eig_py(p, a, b):
    tx = a * np.pi / (p.nx - 1)
    ty = 2.0 * np.pi * b / p.ny
    return -(4.0 / p.hx ** 2) * np.sin(tx / 2) ** 2 - (4.0 / p.hy ** 2) * np.sin(ty / 2) ** 2


def inner_py(p):
    m = np.zeros((p.ny, p.nx))
    m[:, 1:-1] = 1.0
    return np.tile(m.ravel(), 2)


@pytest.mark.parametrize("nx,ny,theta", [(17, 12, 0.5), (24, 7, 1.0), (9, 16, 0.5)])
def test_suolson_periodic_rows_fourier_modes_closed_form(nx, ny, theta):
    """Periodic Fourier modes in y are eigenvectors of the wrapped second difference (a
    wrong wrap, or a y boundary held, breaks the first and last rows)."""
    spec, p = grid_py(nx, ny, xi=0.3, theta=theta)
    lu = eig_py(p, 2, 1)
    ln = eig_py(p, 1, 2)
    U, V = mode_py(p, 2, 1, 0.8), mode_py(p, 2, 1, -0.4)
    Un, Vn = mode_py(p, 1, 2, 1.1, 0.9), mode_py(p, 1, 2, 0.6, 0.9)
    x = np.concatenate([U, V])
    xn = np.concatenate([Un, Vn])
    N = np.concatenate([-(lu / 3.0) * U + (U - V), -p.xi * (U - V)])
    Nn = np.concatenate([-(ln / 3.0) * Un + (Un - Vn), -p.xi * (Un - Vn)])
    Q = mode_py(p, 1, 0, 2.0)
    src = np.concatenate([Q, np.zeros_like(Q)])
    expect = inner_py(p) * (x - xn + p.dt * (theta * N + (1 - theta) * Nn) - p.dt * src)
    got = residual(p, x, xn, src)
    assert np.max(np.abs(got - expect)) <= 1e-13 * max(1.0, np.abs(expect).max())


def test_suolson_periodic_rows_boundary_columns_only():
    spec, p = grid_py(11, 6)
    rng = np.random.default_rng(4)
    x, xn, s = rng.standard_normal((3, p.n))
    F = residual(p, x, xn, s)
    m = inner_py(p)
    assert np.array_equal(F[m == 0], x[m == 0])
    assert not np.allclose(F[m == 1], x[m == 1])
    # the first and last rows are interior rows here
    assert m.reshape(2, p.ny, p.nx)[:, 0, 1:-1].all() and m.reshape(2, p.ny, p.nx)[:, -1, 1:-1].all()


def test_suolson_periodic_rows_reduce_to_the_1d_profile():
    """With the box source and a cold start every row of the solution is the same 1D profile:
    one Newton step of the 2D problem equals the dense solve of the 1D (x only) system."""
    spec, p = grid_py(41, 6, xi=0.1)
    x0, src = W.suolson_box_initial(41, 6)
    o = NewtonOptions(m=30, tol_newton=1e-12, tol_krylov=1e-13, max_newton=3)
    x, info = newton_solve(p, x0, o, source=src)
    assert info.converged
    U = x[: p.n // 2].reshape(p.ny, p.nx)
    V = x[p.n // 2:].reshape(p.ny, p.nx)
    assert np.max(np.abs(U - U[0])) <= 1e-13 and np.max(np.abs(V - V[0])) <= 1e-13
    # 1D Crank-Nicolson system along x, Dirichlet ends, from U = V = 0
    nx, c = p.nx, p.theta * p.dt
    q = src[: nx]
    L1 = np.zeros((nx, nx))
    for i in range(1, nx - 1):
        L1[i, i - 1] = L1[i, i + 1] = 1.0 / p.hx ** 2
        L1[i, i] = -2.0 / p.hx ** 2
    I = np.eye(nx)
    E = np.eye(nx)
    E[0, 0] = E[-1, -1] = 0.0  # interior rows
    A = np.block([[I + c * E @ (-(1.0 / 3.0) * L1 + I), -c * E], [-c * p.xi * E, I + c * p.xi * E]])
    rhs = np.concatenate([p.dt * q, np.zeros(nx)])
    ref = np.linalg.solve(A, rhs)
    assert np.max(np.abs(U[0] - ref[:nx])) <= 1e-10 * np.abs(ref).max()
    assert np.max(np.abs(V[0] - ref[nx:])) <= 1e-10 * np.abs(ref).max()
    assert U[0, nx // 2] > 0 and U[0, 0] == 0.0
