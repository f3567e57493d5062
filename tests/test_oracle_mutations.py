"""Planted mistakes in the oracle must fail its pins.

Each case patches one plausible mistake into the oracle (a sign, a dropped
term, a transposed operand, a wrong index) and runs the pin that should catch
it; the pin must raise.  This shows the pins constrain every part they claim.
"""

import numpy as np
import pytest

import oracle.dual as odual
import oracle.gmres as ogm
import oracle.jvp as ojvp
import oracle.problems as oprob
import test_oracle_gmres as tg
import test_oracle_jvp as tj
import test_oracle_newton as tn
import test_oracle_residual as tr


def _expect_failure(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_sign_of_first_difference(monkeypatch):
    monkeypatch.setattr(oprob, "d1", lambda f, h, axis: (oprob.roll(f, 1, axis) - oprob.roll(f, -1, axis)) / (2 * h))
    _expect_failure(tr.test_burgers1d_fourier_mode, 1.0)
    _expect_failure(tr.test_burgers2d_taylor_green_crank_nicolson)


def test_dropped_factor_in_second_difference(monkeypatch):
    monkeypatch.setattr(oprob, "d2", lambda f, h, axis: (oprob.roll(f, -1, axis) - f + oprob.roll(f, 1, axis)) / (h * h))
    _expect_failure(tr.test_grayscott_mode_and_pointwise_terms)
    _expect_failure(tj.test_ad_columns_equal_analytic_jacobian, tj.tiny_cases()[2])


def test_laplacian_missing_a_direction(monkeypatch):
    monkeypatch.setattr(oprob, "lap", lambda f, p: oprob.d2(f, p.hx, 1) + oprob.d2(f, p.hx, 0))  # hy -> hx
    spec = tj.tiny_cases()[2]  # hx != hy? make it so
    spec = dict(spec, hy=spec["hx"] * 1.7)
    _expect_failure(tj.test_ad_columns_equal_analytic_jacobian, spec)


def test_product_rule_missing_a_term(monkeypatch):
    def bad_mul(self, o):
        if isinstance(o, odual.Dual):
            return odual.Dual(self.val * o.val, self.tan * o.val)
        return odual.Dual(self.val * o, self.tan * o)
    monkeypatch.setattr(odual.Dual, "__mul__", bad_mul)
    for spec in tj.tiny_cases():
        _expect_failure(tj.test_ad_equals_complex_step, spec)


def test_fd_quotient_scaled_wrong(monkeypatch):
    orig = ojvp.jvp_fd
    monkeypatch.setattr(ojvp, "jvp_fd", lambda *a, **k: 0.5 * orig(*a, **k))
    monkeypatch.setattr(tj, "jvp_fd", ojvp.jvp_fd)
    _expect_failure(tj.test_fd_minus_ad_truncation_closed_form, tj.tiny_cases()[0])


def test_givens_sign(monkeypatch):
    orig = ogm.givens
    monkeypatch.setattr(ogm, "givens", lambda a, b: (orig(a, b)[0], -orig(a, b)[1]))
    # restarts from the true residual still reach the answer; the estimate pin catches it
    _expect_failure(tg.test_givens_estimate_equals_true_residual)
    _expect_failure(tg.test_exact_termination_with_few_distinct_eigenvalues)


def test_back_substitution_transposed(monkeypatch):
    orig = ogm.back_substitute
    monkeypatch.setattr(ogm, "back_substitute", lambda R, g: orig(np.ascontiguousarray(R.T), g))
    _expect_failure(tg.test_givens_estimate_equals_true_residual)
    _expect_failure(tg.test_exact_termination_with_few_distinct_eigenvalues)


def test_single_gram_schmidt_pass_loses_orthogonality(monkeypatch):
    # replace the second CGS pass by nothing: dot products against a perturbed basis
    calls = {"n": 0}
    orig_dot = np.dot

    def noisy_dot(a, b):
        calls["n"] += 1
        return orig_dot(a, b) * (1 + 1e-6)
    monkeypatch.setattr(ogm.np, "dot", noisy_dot)
    _expect_failure(tg.test_orthonormal_basis_and_arnoldi_relation)


def test_kerr_boundary_mask_wrong(monkeypatch):
    def bad_mask(p):
        m = np.zeros((p.ny, p.nx))
        m[1:, 1:-1] = 1.0  # forgets the top boundary row
        return m
    monkeypatch.setattr(oprob, "interior_mask", bad_mask)
    _expect_failure(tr.test_kerr_boundary_rows_hold_the_field)


def test_wrong_time_level_in_theta_scheme(monkeypatch):
    orig = oprob.N_apply
    # evaluate the old-level operator at the new level: x_prev ignored
    monkeypatch.setattr(oprob, "N_apply", lambda p, x: orig(p, x) * 1.0 if x is not None else None)
    orig_res = oprob.residual

    def bad_residual(p, x, x_prev, source=None):
        return orig_res(p, x, x, source) + (x - x_prev) * 0 + (x - x_prev)
    monkeypatch.setattr(tr, "residual", bad_residual)
    _expect_failure(tr.test_burgers2d_taylor_green_crank_nicolson)


def test_line_search_that_accepts_every_step(monkeypatch):
    # a sufficient-decrease constant that accepts any step never backtracks
    import dataclasses
    from oracle import newton as onewton

    def opts(**kw):
        return dataclasses.replace(onewton.NewtonOptions(**kw), ls_c=-1e30)
    monkeypatch.setattr(tn, "NewtonOptions", opts)
    _expect_failure(tn.test_line_search_armijo_and_halving)


# --- BiCGSTAB: mistakes planted by rewriting one line of the oracle's source --
import inspect  # noqa: E402

import oracle.bicgstab as obicg  # noqa: E402
import test_oracle_bicgstab as tb  # noqa: E402


def _bicgstab_mutant(old: str, new: str):
    src = inspect.getsource(obicg)
    assert old in src
    ns: dict = {}
    exec(compile(src.replace(old, new, 1), "bicgstab_mutant", "exec"), ns)
    return ns["bicgstab"]


@pytest.mark.parametrize("old,new", [
    ("omega = ts / tt", "omega = -ts / tt"),                            # sign of the stabilizing step
    ("beta = (rho / rho_prev) * (alpha / omega)", "beta = (rho / rho_prev) * (omega / alpha)"),  # swapped ratio
    ("s = r - alpha * v", "s = r + alpha * v"),                          # sign of the half step
    ("r = s - omega * t", "r = s - omega * s"),                          # wrong operand
    ("p = r + beta * (p - omega * v)", "p = r + beta * p"),              # dropped correction term
])
def test_bicgstab_mutations_fail_a_pin(monkeypatch, old, new):
    monkeypatch.setattr(tb, "bicgstab_solve", _bicgstab_mutant(old, new))
    failed = 0
    for fn, args in ((tb.test_dense_solve, (60, 2)), (tb.test_matches_scipy_bicgstab, (40, 4, 1e-8))):
        try:
            fn(*args)
        except AssertionError:
            failed += 1
    assert failed >= 1


import oracle.cg as ocg  # noqa: E402
import test_oracle_cg_rd as tc  # noqa: E402


def _cg_mutant(old: str, new: str):
    src = inspect.getsource(ocg)
    assert old in src
    ns: dict = {}
    exec(compile(src.replace(old, new, 1), "cg_mutant", "exec"), ns)
    return ns["cg"]


@pytest.mark.parametrize("old,new", [
    ("alpha = rr / pJp", "alpha = pJp / rr"),                      # inverted step length
    ("r = r - alpha * Jp", "r = r + alpha * Jp"),                  # sign of the residual update
    ("p = r + (rr_new / rr) * p", "p = r + (rr / rr_new) * p"),    # inverted beta
    ("p = r + (rr_new / rr) * p", "p = r"),                        # steepest descent (dropped conjugation)
    ("if pJp <= 0.0:", "if pJp < 0.0:"),                           # zero curvature not caught
])
def test_cg_mutations_fail_a_pin(monkeypatch, old, new):
    monkeypatch.setattr(tc, "cg_solve", _cg_mutant(old, new))
    failed = 0
    for fn, args in ((tc.test_cg_dense_spd_solve, (80, 2)), (tc.test_cg_matches_scipy, (60, 4, 1e-8)),
                     (tc.test_cg_reports_indefinite_breakdown, ())):
        try:
            fn(*args)
        except (AssertionError, ZeroDivisionError, FloatingPointError):
            failed += 1
    assert failed >= 1


def test_rd_sink_sign_wrong(monkeypatch):
    monkeypatch.setitem(oprob.SPATIAL, "rd2d", lambda p, f: [-p.D * oprob.lap(f[0], p) - f[0] * f[0] * f[0]])
    _expect_failure(tc.test_rd_residual_sine_modes_closed_form, 17, 13, 0.5)
    _expect_failure(tc.test_rd_ad_jacobian_is_the_hand_derived_spd_matrix)


def test_rd_boundary_not_held(monkeypatch):
    orig = oprob.interior_mask
    monkeypatch.setattr(oprob, "interior_mask", lambda p: np.ones_like(orig(p)))
    _expect_failure(tc.test_rd_boundary_rows_are_identity)


def _dcgs2_mutant(monkeypatch, old: str, new: str):
    src = inspect.getsource(ogm)
    assert old in src
    ns: dict = {}
    exec(compile(src.replace(old, new, 1), "gmres_mutant", "exec"), ns)
    monkeypatch.setattr(tg, "gmres_solve", ns["gmres"])


@pytest.mark.parametrize("old,new", [
    ("vj = vj - ah[i] * V[i]", "vj = vj + ah[i] * V[i]"),          # sign of the reorthogonalization
    ("h[:j] = b - Ha[:j]", "h[:j] = b"),                            # Arnoldi-relation term dropped
    ("u = w - gamma * uh", "u = w + gamma * uh"),                   # sign of the projection on u^
    ("a = np.array([np.dot(V[i], u) for i in range(col + 1)])",
     "a = np.array([np.dot(V[i], u) for i in range(col)] + [0.0])"),  # second pass misses the newest vector
    ("Hraw[: j + 1, j] = h", "Hraw[: j + 1, j] = -h"),              # sign of the stored column
    ("u = u - (Ha[i] + h[i] - gamma * ah[i]) * V[i]", "u = u - (h[i] - gamma * ah[i]) * V[i]"),  # dropped term
])
def test_dcgs2_mutations_fail_a_pin(monkeypatch, old, new):
    # (the second-pass coefficients a vanish in exact arithmetic, so mistakes confined to
    # how they enter H or beta change results only at rounding level and no pin can see them)
    _dcgs2_mutant(monkeypatch, old, new)
    failed = 0
    for fn, args in ((tg.test_dcgs2_single_cycle_equals_cgs2, (25, 2)),
                     (tg.test_dcgs2_keeps_orthogonality_where_one_pass_loses_it, ())):
        try:
            fn(*args)
        except (AssertionError, ValueError, ZeroDivisionError):
            failed += 1
    assert failed >= 1


import test_oracle_suolson as tso  # noqa: E402


@pytest.mark.parametrize("bad", [
    lambda p, f: [-(1.0 / 3.0) * oprob.lap(f[0], p) + (f[1] - f[0]), -p.xi * (f[0] - f[1])],  # coupling sign
    lambda p, f: [-(1.0 / 3.0) * oprob.lap(f[0], p) + (f[0] - f[1]), -(f[0] - f[1])],         # xi dropped
    lambda p, f: [-oprob.lap(f[0], p) + (f[0] - f[1]), -p.xi * (f[0] - f[1])],                # 1/3 dropped
])
def test_suolson_mistakes_fail_a_pin(monkeypatch, bad):
    monkeypatch.setitem(oprob.SPATIAL, "suolson", bad)
    _expect_failure(tso.test_suolson_sine_modes_closed_form, 17, 13, 0.5, False)
    _expect_failure(tso.test_suolson_jacobian_is_the_constant_hand_derived_matrix)


import test_oracle_maxwell as tmx  # noqa: E402


def test_maxwell_guard_removed(monkeypatch):
    from oracle.dual import Dual

    def unguarded(s):
        if isinstance(s, Dual):
            v = np.sqrt(s.val)
            with np.errstate(divide="ignore", invalid="ignore"):
                return Dual(v, s.tan / (2.0 * v))
        return np.sqrt(s)

    monkeypatch.setattr(oprob, "guarded_norm", unguarded)
    _expect_failure(tmx.test_maxwell_guard_gives_the_born_operator_at_zero)


@pytest.mark.parametrize("old,new", [
    ("nxr = dxdy(eyr) - d2(exr, p.hy, 0)", "nxr = -dxdy(eyr) - d2(exr, p.hy, 0)"),      # mixed-derivative sign
    ("(m * (exi - loss * exr))", "(m * (exi + loss * exr))"),                           # sign of the loss
    ("nyr = dxdy(exr) - d2(eyr, p.hx, 1)", "nyr = dxdy(exr) - d2(eyr, p.hy, 0)"),      # wrong direction
])
def test_maxwell_mistakes_fail_a_pin(monkeypatch, old, new):
    src = inspect.getsource(oprob.maxwell_residual)
    assert old in src
    ns = dict(vars(oprob))
    exec(compile(src.replace(old, new, 1), "maxwell_mutant", "exec"), ns)
    monkeypatch.setattr(oprob, "maxwell_residual", ns["maxwell_residual"])
    _expect_failure(tmx.test_maxwell_sine_modes_closed_form, 17, 13, 0.05)


import oracle.newton as onewton  # noqa: E402
import oracle.precond as oprec  # noqa: E402
import test_oracle_cslp as tcs  # noqa: E402


@pytest.mark.parametrize("old,new,pin", [
    ("2.0 / (p.hy * p.hy) - w2 * eps_p", "2.0 / (p.hx * p.hx) - w2 * eps_p", "born"),         # hx / hy swapped
    ("(1.0 - 1j * p.eps_im)", "(1.0 + 1j * p.eps_im)", "born"),                                # sign of the loss
    ("(1.0 + p.chi3 * absE)", "(1.0 + p.chi3 * absE * absE)", "field"),                       # |E|^2 for |E|
    ("eps_p = eps * (1.0 - 1j * damping)", "eps_p = eps", "damping"),                         # damping dropped
    ("np.where(inner, 2.0 / (p.hx * p.hx) - w2 * eps_p, 1.0 + 0j)",
     "2.0 / (p.hx * p.hx) - w2 * eps_p", "boundary"),                                          # boundary not identity
])
def test_cslp_mistakes_fail_a_pin(monkeypatch, old, new, pin):
    src = inspect.getsource(oprec.cslp_diagonal)
    assert old in src
    ns = dict(vars(oprec))
    exec(compile(src.replace(old, new, 1), "cslp_mutant", "exec"), ns)
    monkeypatch.setattr(oprec, "cslp_diagonal", ns["cslp_diagonal"])
    monkeypatch.setattr(tcs, "cslp_diagonal", ns["cslp_diagonal"])
    if pin == "born":
        _expect_failure(tcs.test_undamped_cslp_is_the_born_jacobian_diagonal, 9, 7)
    elif pin == "field":
        _expect_failure(tcs.test_undamped_cslp_follows_the_local_field, 0)
    elif pin == "damping":
        _expect_failure(tcs.test_damping_scales_the_permittivity_term_only)
    else:
        _expect_failure(tcs.test_boundary_nodes_are_identity)


def test_cslp_update_left_in_the_preconditioned_space(monkeypatch):
    src = inspect.getsource(onewton.newton_solve)
    assert "dx = minv(bwd(z))" in src
    ns = dict(vars(onewton))
    exec(compile(src.replace("dx = minv(bwd(z))", "dx = bwd(z)", 1), "newton_mutant", "exec"), ns)
    monkeypatch.setattr(tcs, "newton_solve", ns["newton_solve"])
    _expect_failure(tcs.test_newton_with_cslp_reaches_the_same_field)


def test_suolson_periodic_rows_held_as_boundary(monkeypatch):
    def all_round(p):
        m = np.zeros((p.ny, p.nx))
        m[1:-1, 1:-1] = 1.0
        return m

    monkeypatch.setattr(oprob, "interior_mask", all_round)
    _expect_failure(tso.test_suolson_periodic_rows_fourier_modes_closed_form, 17, 12, 0.5)
    _expect_failure(tso.test_suolson_periodic_rows_reduce_to_the_1d_profile)
