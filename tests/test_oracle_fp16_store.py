"""Pins of the oracle's FP16 basis store (GMRES with store='fp16').

The store rounds every vector written to the Krylov basis to binary16 after a
power-of-two scaling.  Pinned against an independent rounding (the
significand cut to 11 bits, ties to even, by integer arithmetic on the FP64
bit pattern), against binary16's exact representability of every stored
basis vector, and against the effect the rounding must have on the Arnoldi
process: a relation residual and a loss of orthogonality of the order of the
binary16 unit roundoff u = 2^-11, not of FP64's, while the restarted solve
still meets its tolerance and the two Gram-Schmidt forms stay within O(u) of
each other.
"""

import math

import numpy as np
import pytest

from oracle import gmres_solve
from oracle.gmres import store_fp16

U16 = 2.0 ** -11


def round_to_11_bits(v):
    """Nearest value with an 11-bit significand (ties to even), by integer
    arithmetic on the FP64 bits: binary16 rounding without its exponent range."""
    b = v.astype(np.float64).view(np.uint64)
    drop = np.uint64(52 - 10)  # FP64 keeps 52 fraction bits, binary16 10
    low = b & ((np.uint64(1) << drop) - np.uint64(1))
    half = np.uint64(1) << (drop - np.uint64(1))
    keep = b >> drop
    up = (low > half) | ((low == half) & ((keep & np.uint64(1)) == np.uint64(1)))
    r = (keep + up.astype(np.uint64)) << drop
    return r.view(np.float64)


def dense_system(n, seed, shift=3.0):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + shift * np.eye(n)
    return A, rng.standard_normal(n)


def test_store_matches_independent_rounding():
    rng = np.random.default_rng(0)
    for scale in (1e-3, 1.0, 37.0, 1e4):
        v = scale * rng.standard_normal(4096)
        s = store_fp16(v)
        # entries the scaled binary16 holds in its normal range: same as the 11-bit rounding
        sig = 2.0 ** -round(math.log2(np.linalg.norm(v) / math.sqrt(v.size)))
        normal = np.abs(v * sig) >= 2.0 ** -14
        assert normal.mean() > 0.99
        np.testing.assert_array_equal(s[normal], round_to_11_bits(v[normal]))
        assert np.all(np.abs(s[normal] - v[normal]) <= U16 * np.abs(v[normal]))
        # every stored value times the scale is a binary16 number; storing again changes nothing
        assert np.array_equal((s * sig).astype(np.float16).astype(np.float64), s * sig)
        np.testing.assert_array_equal(store_fp16(s), s)
    # a tie rounds to even: 1 + 2^-11 sits halfway between 1 and 1 + 2^-10
    v = np.ones(4)
    v[1] = 1.0 + 2.0 ** -11
    v[2] = 1.0 + 3 * 2.0 ** -11
    s = store_fp16(v)
    assert s[1] == 1.0 and s[2] == 1.0 + 2 * 2.0 ** -10
    assert not store_fp16(np.zeros(5)).any()


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
def test_fp16_store_effect_on_arnoldi(orth):
    A, b = dense_system(300, 1)
    m = 20
    _, i64 = gmres_solve(lambda v: A @ v, b, m=m, tol=0.0, max_restarts=1, record=True, orth=orth)
    _, i16 = gmres_solve(lambda v: A @ v, b, m=m, tol=0.0, max_restarts=1, record=True, orth=orth, store="fp16")
    for info, lo, hi in ((i64, 0.0, 1e-13), (i16, 1e-3 * U16, 4 * U16)):
        V = np.stack(info.last_V[: m + 1], axis=1)
        rel = np.abs(A @ V[:, :m] - V @ info.last_H).max() / np.abs(A).max()
        orth_loss = np.abs(V.T @ V - np.eye(m + 1)).max()
        assert lo <= rel <= hi, (orth, rel)
        assert lo <= orth_loss <= hi * 2, (orth, orth_loss)
    # same Hessenberg to O(u)
    d = np.abs(i16.last_H - i64.last_H).max() / np.abs(i64.last_H).max()
    assert 1e-2 * U16 <= d <= 8 * U16, d
    if orth == "dcgs2":
        # the completed v_j are written to the store: binary16 up to their power-of-two scale
        for v in i16.last_V[1:m]:
            sig = 2.0 ** -round(math.log2(np.linalg.norm(v) / math.sqrt(v.size)))
            assert np.array_equal((v * sig).astype(np.float16).astype(np.float64), v * sig)


@pytest.mark.parametrize("orth", ["cgs2", "dcgs2"])
def test_fp16_store_restarted_solve_meets_tolerance(orth):
    A, b = dense_system(200, 2, shift=2.0)
    x, info = gmres_solve(lambda v: A @ v, b, m=15, tol=1e-10, max_restarts=50, orth=orth, store="fp16")
    assert info.converged
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    _, i64 = gmres_solve(lambda v: A @ v, b, m=15, tol=1e-10, max_restarts=50, orth=orth)
    # the store limits what one cycle achieves: the true residual after the first cycle stays
    # near u ||b|| although the Givens estimate went further, so more steps are needed
    bn = np.linalg.norm(b)
    assert info.true_res[1] >= 0.1 * U16 * bn and info.true_res[1] >= 5 * i64.true_res[1]
    assert info.iters > i64.iters
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.cond(A) * 10 * np.linalg.norm(xs)


def test_dcgs2_and_cgs2_agree_under_fp16_store():
    A, b = dense_system(250, 3)
    m = 16
    _, a = gmres_solve(lambda v: A @ v, b, m=m, tol=0.0, max_restarts=1, record=True, orth="cgs2", store="fp16")
    _, c = gmres_solve(lambda v: A @ v, b, m=m, tol=0.0, max_restarts=1, record=True, orth="dcgs2", store="fp16")
    d = np.abs(a.last_H - c.last_H).max() / np.abs(a.last_H).max()
    assert d <= 8 * U16, d
