"""Pins of the oracle's CSLP preconditioner for the Maxwell-Kerr problem
(Appendix A.4) and of right-preconditioned GMRES / Newton (no GPU).

* undamped, the preconditioner is the diagonal of the Jacobian wherever the
  Kerr tangent term does not reach that diagonal: at E = 0 (the Born
  operator), and at a node whose other component is zero (there the
  tangent of |E| along the component's own direction vanishes), probed by
  unit vectors through the AD JVP of the residual (an independent route
  through the curl-curl stencil, the loss sign, |E| and chi); hx != hy, so
  a swap of the two 2/h^2 terms fails;
* the complex structure: the Jacobian at E = 0 is complex-linear on each
  component, so its Re and Im unit columns hold d and i d, and M acts as
  that complex number;
* the damping multiplies the permittivity term only;
* boundary nodes: M = 1;
* right-preconditioned GMRES solves the unpreconditioned system: the update
  M^{-1} z equals the dense solve of J dx = rhs, with and without restarts;
* Newton with the preconditioner converges to the same field as without.

The scalar Helmholtz-Kerr form (M = 2/hx^2 + 2/hy^2 - k0^2 eps(E)(1 - 0.5 i)):
the Born Jacobian diagonal and its complex structure; M(E) E equal to the
source-free residual at a node whose neighbours are zero (fixes the |E|^2
law, chi3, the loss sign and both 2/h^2 terms); damping, boundary identity
and inverse; right-preconditioned GMRES against a dense solve; Newton to the
same field with and without it.
"""

import numpy as np
import pytest

import workloads as W
from oracle import NewtonOptions, Problem, cslp_diagonal, cslp_solve, gmres_solve, jvp_ad, newton_solve, residual


def grid(nx, ny, omega=3.3, chi=0.4, loss=0.05):
    spec = W.maxwell_spec(nx, omega=omega, chi=chi, loss=loss, ny=ny)
    return spec, Problem.from_spec(spec)


def unit(p, plane, j, i):
    e = np.zeros(p.n)
    e[plane * p.nx * p.ny + j * p.nx + i] = 1.0
    return e


def column_diag(p, x, plane, j, i):
    """Complex diagonal entry of J(x) for the component whose Re part is `plane` (0: Ex, 2: Ey)."""
    col = jvp_ad(p, x, unit(p, plane, j, i), x, None)[1]
    k = j * p.nx + i
    N = p.nx * p.ny
    return col[plane * N + k] + 1j * col[(plane + 1) * N + k]


@pytest.mark.parametrize("nx,ny", [(9, 7), (6, 11)])
def test_undamped_cslp_is_the_born_jacobian_diagonal(nx, ny):
    spec, p = grid(nx, ny)
    assert abs(p.hx - p.hy) > 0.01
    x = np.zeros(p.n)
    mxx, myy = cslp_diagonal(p, x, damping=0.0)
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            dx = column_diag(p, x, 0, j, i)
            dy = column_diag(p, x, 2, j, i)
            assert abs(mxx[j, i] - dx) <= 1e-12 * abs(dx), (j, i, mxx[j, i], dx)
            assert abs(myy[j, i] - dy) <= 1e-12 * abs(dy), (j, i, myy[j, i], dy)


def test_complex_structure_of_the_born_diagonal():
    spec, p = grid(8, 6)
    x = np.zeros(p.n)
    N = p.nx * p.ny
    j, i = 2, 3
    k = j * p.nx + i
    d = column_diag(p, x, 0, j, i)
    col_im = jvp_ad(p, x, unit(p, 1, j, i), x, None)[1]  # direction i e_k on Ex
    assert abs(col_im[k] - (-d.imag)) <= 1e-12 * abs(d)
    assert abs(col_im[N + k] - d.real) <= 1e-12 * abs(d)
    # M^{-1} (M v) = v with M acting as complex multiplication on each component
    mxx, myy = cslp_diagonal(p, x)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(p.n)
    vx = v[:N] + 1j * v[N:2 * N]
    vy = v[2 * N:3 * N] + 1j * v[3 * N:]
    mv = np.concatenate([(mxx.ravel() * vx).real, (mxx.ravel() * vx).imag, (myy.ravel() * vy).real,
                         (myy.ravel() * vy).imag])
    assert np.allclose(cslp_solve(p, x, mv), v, rtol=0, atol=1e-13)


@pytest.mark.parametrize("which", [0, 2])
def test_undamped_cslp_follows_the_local_field(which):
    """At a node where the other component is zero the Kerr tangent term is off this diagonal."""
    spec, p = grid(9, 8)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(p.n) * 0.8
    N = p.nx * p.ny
    other = 2 if which == 0 else 0
    nodes = [(j, i) for j in range(1, p.ny - 1) for i in range(1, p.nx - 1)]
    for j, i in nodes:
        k = j * p.nx + i
        x[which * N + k] = 0.0          # this component zero at the node...
        x[(which + 1) * N + k] = 0.0
        assert x[other * N + k] != 0.0  # ...the other one not
    mxx, myy = cslp_diagonal(p, x, damping=0.0)
    M = mxx if which == 0 else myy
    for j, i in nodes:
        d = column_diag(p, x, which, j, i)
        assert abs(M[j, i] - d) <= 1e-12 * abs(d), (which, j, i, M[j, i], d)
    # and the field matters: the Born diagonal differs by omega^2 chi |E| (1 - loss i)
    mb = cslp_diagonal(p, np.zeros(p.n), damping=0.0)[0 if which == 0 else 1]
    assert np.max(np.abs(M - mb)[1:-1, 1:-1]) > 0.1


def test_damping_scales_the_permittivity_term_only():
    spec, p = grid(7, 9)
    x = np.random.default_rng(5).standard_normal(p.n)
    m0x, m0y = cslp_diagonal(p, x, damping=0.0)
    mdx, mdy = cslp_diagonal(p, x, damping=0.5)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose((mdx - 2 / p.hy ** 2)[inner], ((1 - 0.5j) * (m0x - 2 / p.hy ** 2))[inner], rtol=1e-14)
    assert np.allclose((mdy - 2 / p.hx ** 2)[inner], ((1 - 0.5j) * (m0y - 2 / p.hx ** 2))[inner], rtol=1e-14)
    # the default is the paper's damping
    dx, dy = cslp_diagonal(p, x)
    assert np.array_equal(dx, mdx) and np.array_equal(dy, mdy)


def test_boundary_nodes_are_identity():
    spec, p = grid(8, 7)
    rng = np.random.default_rng(2)
    x, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    mv = cslp_solve(p, x, v).reshape(4, p.ny, p.nx)
    vv = v.reshape(4, p.ny, p.nx)
    bnd = np.ones((p.ny, p.nx), bool)
    bnd[1:-1, 1:-1] = False
    assert np.array_equal(mv[:, bnd], vv[:, bnd])
    assert not np.allclose(mv[:, ~bnd], vv[:, ~bnd])


def test_cslp_rejects_other_problems():  # Gray-Scott: no CSLP
    p = Problem.from_spec(W.grayscott_spec(8))
    with pytest.raises(ValueError):
        cslp_diagonal(p, np.zeros(p.n))


def dense_jacobian(p, x):
    return np.stack([jvp_ad(p, x, e, x, None)[1] for e in np.eye(p.n)], axis=1)


@pytest.mark.parametrize("m,restarts", [(200, 3), (60, 60)])
def test_right_preconditioned_gmres_solves_the_original_system(m, restarts):
    spec, p = grid(7, 6, omega=2.2, chi=0.3)
    rng = np.random.default_rng(7)
    x = 0.5 * rng.standard_normal(p.n)
    rhs = rng.standard_normal(p.n)
    ref = np.linalg.solve(dense_jacobian(p, x), rhs)
    mv = lambda v: jvp_ad(p, x, v, x, None)[1]  # noqa: E731
    z, info = gmres_solve(lambda v: mv(cslp_solve(p, x, v)), rhs, m=m, tol=1e-11, max_restarts=restarts)
    assert info.converged, info
    dx = cslp_solve(p, x, z)
    assert np.linalg.norm(dx - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.linalg.norm(z - ref) > 1e-3 * np.linalg.norm(ref)  # z itself is not the update


def test_newton_with_cslp_reaches_the_same_field():
    spec = W.maxwell_spec(12, omega=2.5, ny=10)
    src = W.maxwell_source(12, omega=2.5, ny=10)
    p = Problem.from_spec(spec)
    x0 = np.zeros(p.n)
    outs = {}
    for pc in ("none", "cslp"):
        o = NewtonOptions(m=30, tol_newton=1e-9, tol_krylov=1e-10, max_newton=8, max_restarts=20, precond=pc)
        x, info = newton_solve(p, x0, o, source=src)
        assert info.converged, (pc, info.rel_res)
        outs[pc] = x
    assert np.linalg.norm(outs["cslp"] - outs["none"]) <= 1e-9 * np.linalg.norm(outs["none"])
    assert np.linalg.norm(residual(p, outs["cslp"], x0, src)) <= 1e-10 * np.linalg.norm(residual(p, x0, x0, src))
    with pytest.raises(ValueError):
        newton_solve(p, x0, NewtonOptions(krylov="bicgstab", precond="cslp"), source=src)


# ---------------------------------------------------------------------------
# Helmholtz-Kerr: the same construction on the scalar operator
# -Lap E - k0^2 (eps_L + chi3 |E|^2) E (one complex component per node)
# ---------------------------------------------------------------------------


def kerr_grid(nx, ny, chi=0.3, eps_im=-0.05, cpw=8.0):
    """hx != hy and a lossy eps_L, so that a swapped 2/h^2 term or a dropped loss sign fails."""
    return Problem(kind="kerr", nx=nx, ny=ny, hx=1.0, hy=0.8, k0=2.0 * np.pi / cpw, eps_re=1.0, eps_im=eps_im,
                   chi3=chi)


def kerr_unit(p, j, i, f):
    e = np.zeros(p.n)
    e[2 * (j * p.nx + i) + f] = 1.0
    return e


@pytest.mark.parametrize("nx,ny", [(9, 7), (6, 11)])
def test_kerr_undamped_cslp_is_the_born_jacobian_diagonal(nx, ny):
    p = kerr_grid(nx, ny)
    x = np.zeros(p.n)
    (m,) = cslp_diagonal(p, x, damping=0.0)
    for j in range(1, ny - 1):
        for i in range(1, nx - 1):
            k = j * nx + i
            col = jvp_ad(p, x, kerr_unit(p, j, i, 0), x, None)[1]
            d = col[2 * k] + 1j * col[2 * k + 1]
            assert abs(m[j, i] - d) <= 1e-12 * abs(d), (j, i, m[j, i], d)
            # the Im unit column holds i d: the Jacobian at E = 0 is complex-linear
            col_im = jvp_ad(p, x, kerr_unit(p, j, i, 1), x, None)[1]
            assert abs(col_im[2 * k] + d.imag) <= 1e-12 * abs(d) and abs(col_im[2 * k + 1] - d.real) <= 1e-12 * abs(d)


def test_kerr_undamped_cslp_times_an_isolated_field_is_the_residual():
    """Where E vanishes at every neighbour of a node, the source-free residual there is M(E) E
    (complex product): a route through the residual itself that fixes the |E|^2 law, chi3, the
    loss sign and both 2/h^2 terms of the field-dependent diagonal, node by node."""
    p = kerr_grid(8, 7, chi=0.7)
    rng = np.random.default_rng(21)
    checked = 0
    for j in range(1, p.ny - 1):
        for i in range(1, p.nx - 1):
            x = np.zeros(p.n)
            k = j * p.nx + i
            e = complex(*rng.standard_normal(2))
            x[2 * k], x[2 * k + 1] = e.real, e.imag
            (m,) = cslp_diagonal(p, x, damping=0.0)
            F = residual(p, x, None, None)
            f = F[2 * k] + 1j * F[2 * k + 1]
            assert abs(m[j, i] * e - f) <= 1e-12 * abs(f), (j, i, m[j, i] * e, f)
            checked += 1
    assert checked == 6 * 5
    # and the field matters: |E|^2 enters with chi3
    x = W.random_vector(p.n, 4)
    (m,) = cslp_diagonal(p, x, damping=0.0)
    (mb,) = cslp_diagonal(p, np.zeros(p.n), damping=0.0)
    re, im = x[0::2].reshape(p.ny, p.nx), x[1::2].reshape(p.ny, p.nx)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose((mb - m)[inner], (p.k0 ** 2 * p.chi3 * (re * re + im * im))[inner], rtol=1e-13, atol=0)


def test_kerr_damping_boundary_and_inverse():
    p = kerr_grid(7, 9)
    rng = np.random.default_rng(5)
    x, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    (m0,) = cslp_diagonal(p, x, damping=0.0)
    (md,) = cslp_diagonal(p, x)
    diag = 2.0 / p.hx ** 2 + 2.0 / p.hy ** 2
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose((md - diag)[inner], ((1 - 0.5j) * (m0 - diag))[inner], rtol=1e-14)
    # boundary nodes: identity
    mv = cslp_solve(p, x, v).reshape(p.ny, p.nx, 2)
    vv = v.reshape(p.ny, p.nx, 2)
    bnd = np.ones((p.ny, p.nx), bool)
    bnd[1:-1, 1:-1] = False
    assert np.array_equal(mv[bnd], vv[bnd]) and not np.allclose(mv[~bnd], vv[~bnd])
    # M acts as a complex multiplication: M^{-1} (M v) = v
    c = v[0::2] + 1j * v[1::2]
    mc = md.ravel() * c
    back = cslp_solve(p, x, np.stack([mc.real, mc.imag], axis=-1).ravel())
    assert np.allclose(back, v, rtol=0, atol=1e-13)


def test_kerr_right_preconditioned_gmres_and_newton():
    p = kerr_grid(7, 6, chi=0.3)
    rng = np.random.default_rng(7)
    x = 0.5 * rng.standard_normal(p.n)
    rhs = rng.standard_normal(p.n)
    ref = np.linalg.solve(dense_jacobian(p, x), rhs)
    mv = lambda v: jvp_ad(p, x, v, x, None)[1]  # noqa: E731
    z, info = gmres_solve(lambda v: mv(cslp_solve(p, x, v)), rhs, m=100, tol=1e-12, max_restarts=3)
    assert info.converged, info
    dx = cslp_solve(p, x, z)
    assert np.linalg.norm(dx - ref) <= 1e-9 * np.linalg.norm(ref)
    assert np.linalg.norm(z - ref) > 1e-3 * np.linalg.norm(ref)
    # Newton with and without the preconditioner: the same field
    src = np.zeros(p.n)
    src.reshape(p.ny, p.nx, 2)[1:-1, 1:-1, 0] = 0.3 * rng.standard_normal((p.ny - 2, p.nx - 2))
    x0 = np.zeros(p.n)
    outs = {}
    for pc in ("none", "cslp"):
        o = NewtonOptions(m=30, tol_newton=1e-10, tol_krylov=1e-11, max_newton=10, max_restarts=20, precond=pc)
        xs, ni = newton_solve(p, x0, o, source=src)
        assert ni.converged, (pc, ni.rel_res)
        outs[pc] = xs
    assert np.linalg.norm(outs["cslp"] - outs["none"]) <= 1e-9 * np.linalg.norm(outs["none"])
