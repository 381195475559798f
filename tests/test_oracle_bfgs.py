"""Pins for the oracle's BFGS matrices (eq. 3, eq. 2, Alg. 2) — CPU only.

Each check compares the oracle with something it does not compute itself:
hand-derived fractions, algebraic identities the paper states or implies,
numpy's matrix inverse, and brute-force exact arithmetic.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import dense, recursion, bfgs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq3_hand.json")


def _frac(x):
    return Fraction(x[0], x[1])


def spd(n, cond=10.0, seed=0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def secant_pairs(n, k, seed=0, h0=None, damping=1.0):
    A = spd(n, 20.0, seed)
    b = np.random.default_rng(seed + 1).standard_normal(n)
    S, Y, h, _, _ = bfgs.bfgs_quadratic(A, b, k, h0=h0, damping=damping)
    return A, S, Y, h


# --- hand-derived golden matrices (eq. 3) ----------------------------------------------
@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_golden_exact(case):
    h0 = [_frac(v) for v in case["h0"]]
    S = [[_frac(v) for v in s] for s in case["S"]]
    Y = [[_frac(v) for v in y] for y in case["Y"]]
    want = [[_frac(v) for v in row] for row in case["B"]]
    got = dense.inverse_hessian_exact(h0, S, Y)
    assert got == want
    # the dense float64 update and the block recursion agree with the same hand values
    f = lambda M: np.array([[float(v) for v in row] for row in M])
    Bf = dense.inverse_hessian([float(v) for v in h0], f(S), f(Y))
    np.testing.assert_allclose(Bf, f(want), rtol=1e-15, atol=1e-15)
    cols = recursion.apply_hk([float(v) for v in h0], f(S), f(Y), np.eye(len(h0)))
    np.testing.assert_allclose(cols, f(want), rtol=1e-15, atol=1e-15)


# --- brute force in exact rationals (n, k <= 6) ----------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_exact_rationals_small_integers(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 7))
    k = int(rng.integers(1, 7))
    A = rng.integers(-3, 4, (n, n))
    A = A @ A.T + n * np.eye(n, dtype=np.int64)          # integer SPD
    S = rng.integers(-4, 5, (k, n))
    S[np.all(S == 0, axis=1), 0] = 1
    Y = S @ A                                            # y = A s, s^T y > 0
    h0 = rng.integers(1, 5, n)
    exact = dense.inverse_hessian_exact(h0.tolist(), S.tolist(), Y.tolist())
    exact_f = np.array([[float(v) for v in row] for row in exact])
    B = dense.inverse_hessian(h0, S, Y)
    scale = np.abs(exact_f).max()
    assert np.abs(B - exact_f).max() <= 1e-12 * scale
    cols = recursion.apply_hk(h0, S, Y, np.eye(n))
    assert np.abs(cols - exact_f).max() <= 1e-12 * scale
    # the secant condition of the last pair holds exactly in rationals
    s, y = S[-1].tolist(), Y[-1].tolist()
    for i in range(n):
        assert sum(exact[i][j] * y[j] for j in range(n)) == s[i]


# --- secant, symmetry, positive definiteness ----------------------------------------------
@pytest.mark.parametrize("damping", [1.0, 0.7])
def test_secant_symmetry_pd(damping):
    n, k = 40, 12
    A, S, Y, h = secant_pairs(n, k, seed=3, damping=damping)
    B = dense.inverse_hessian(h, S, Y)
    np.testing.assert_allclose(B @ Y[-1], S[-1], rtol=0, atol=1e-13 * np.abs(S[-1]).max())
    assert np.abs(B - B.T).max() <= 1e-14 * np.abs(B).max()
    assert np.linalg.eigvalsh(B).min() > 0
    # block recursion: symmetric bilinear form and secant
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, n))
    Bu = recursion.apply_hk(h, S, Y, u)
    Bv = recursion.apply_hk(h, S, Y, v)
    assert abs(u @ Bv - v @ Bu) <= 1e-13 * abs(u @ Bv)
    assert v @ Bv > 0
    np.testing.assert_allclose(recursion.apply_hk(h, S, Y, Y[-1]), S[-1], atol=1e-13 * np.abs(S[-1]).max())


def test_hereditary_exact_line_search():
    """Exact line search on a quadratic keeps every earlier secant condition (conjugate steps)."""
    n, k = 60, 20
    A, S, Y, h = secant_pairs(n, k, seed=5)
    HY = recursion.apply_hk(h, S, Y, Y)
    rel = np.abs(HY - S).max() / np.abs(S).max()
    assert rel < 1e-6


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_quadratic_termination(n):
    """n exact-line-search BFGS steps on an SPD quadratic recover A^-1 (numpy's inverse)."""
    A = spd(n, 10.0, seed=n)
    b = np.random.default_rng(n).standard_normal(n)
    S, Y, h, _, _ = bfgs.bfgs_quadratic(A, b, n)
    assert S.shape[0] == n
    B = dense.inverse_hessian(h, S, Y)
    Ainv = np.linalg.inv(A)
    assert np.abs(B - Ainv).max() <= 1e-10 * np.abs(Ainv).max()
    # diagonal B_0 as well
    h0 = np.random.default_rng(1).uniform(0.5, 2.0, n)
    S, Y, h, _, _ = bfgs.bfgs_quadratic(A, b, n, h0=h0)
    B = dense.inverse_hessian(h, S, Y)
    assert np.abs(B - Ainv).max() <= 1e-10 * np.abs(Ainv).max()


def test_eq2_inverse_is_eq3():
    """Eq. (3) is the Sherman-Morrison inverse of the eq. (2) Hessian update."""
    n, k = 12, 7
    A, S, Y, h = secant_pairs(n, k, seed=9, damping=0.7)
    h0 = np.random.default_rng(2).uniform(0.5, 2.0, n)
    H = dense.hessian_eq2(h0, S, Y)
    B = dense.inverse_hessian(h0, S, Y)
    assert np.abs(np.linalg.inv(H) - B).max() <= 1e-10 * np.abs(B).max()


def test_block_recursion_is_dense_matrix():
    n, k = 80, 25
    A, S, Y, h = secant_pairs(n, k, seed=11, damping=0.7)
    h0 = np.random.default_rng(3).uniform(0.2, 3.0, n)
    B = dense.inverse_hessian(h0, S, Y)
    V = np.random.default_rng(4).standard_normal((7, n))
    out = recursion.apply_hk(h0, S, Y, V)
    np.testing.assert_allclose(out, V @ B, rtol=0, atol=1e-12 * np.abs(V @ B).max())
    E = recursion.apply_hk(h0, S, Y, V, subtract_b0=True)
    np.testing.assert_allclose(E, V @ (B - np.diag(h0)), rtol=0, atol=1e-12 * np.abs(V @ B).max())


def test_scale_invariance():
    n, k = 30, 10
    A, S, Y, h = secant_pairs(n, k, seed=13, damping=0.7)
    B1 = dense.inverse_hessian(h, S, Y)
    alpha = np.geomspace(1e-3, 1e3, k)[:, None]
    B2 = dense.inverse_hessian(h, alpha * S, alpha * Y)
    assert np.abs(B1 - B2).max() <= 1e-12 * np.abs(B1).max()


def test_gamma_bounds():
    """gamma = s^T y / y^T y = s^T A s / s^T A^2 s lies in [1/lmax, 1/lmin]."""
    n = 50
    A = spd(n, 30.0, seed=17)
    ev = np.linalg.eigvalsh(A)
    b = np.random.default_rng(5).standard_normal(n)
    S, Y, h, _, _ = bfgs.bfgs_quadratic(A, b, 3)
    gamma = h[0]
    assert 1 / ev.max() <= gamma <= 1 / ev.min()
    assert gamma == pytest.approx(S[0] @ Y[0] / (Y[0] @ Y[0]), rel=1e-15)


def test_zero_pairs_is_b0():
    h0 = np.array([1.0, 2.0, 3.0])
    V = np.arange(6.0).reshape(2, 3)
    np.testing.assert_array_equal(recursion.apply_hk(h0, np.zeros((0, 3)), np.zeros((0, 3)), V), V * h0)


# --- the limited-memory form (L-BFGS with a fixed B_0) ----------------------------------
def test_limited_memory_one_pair_is_a_single_update():
    """memory = 1: every direction is -B g with B the single eq. (3) update of B_0 by
    the last pair, written out here as a dense matrix, (I - r s y^T) B_0 (I - r y s^T)
    + r s s^T.  Damped steps keep the iterates away from full BFGS."""
    n, k = 9, 6
    A = spd(n, 30.0, 5)
    b = np.random.default_rng(6).standard_normal(n)
    h0 = np.linspace(0.5, 2.0, n)
    S, Y, _, _, _ = bfgs.bfgs_quadratic(A, b, k, h0=h0, damping=0.6, memory=1)
    g = -b.copy()
    for i in range(k):
        if i == 0:
            B = np.diag(h0)
        else:
            s, y = S[i - 1], Y[i - 1]
            r = 1.0 / (y @ s)
            I = np.eye(n)
            B = (I - r * np.outer(s, y)) @ np.diag(h0) @ (I - r * np.outer(y, s)) + r * np.outer(s, s)
        p = -B @ g
        alpha = 0.6 * (-(g @ p) / (p @ A @ p))
        np.testing.assert_allclose(S[i], alpha * p, rtol=1e-12, atol=1e-14)
        g = g + A @ S[i]
    S_full, _, _, _, _ = bfgs.bfgs_quadratic(A, b, k, h0=h0, damping=0.6)
    assert np.abs(S_full[2:] - S[2:]).max() > 1e-3 * np.abs(S).max()   # the memory matters here


@pytest.mark.parametrize("memory", [1, 3])
def test_limited_memory_exact_line_search_is_full_bfgs(memory):
    """With exact line searches on a quadratic and a fixed B_0, limited-memory BFGS
    takes the steps of full-memory BFGS (both are conjugate gradients preconditioned by
    B_0: the directions depend only on the last pair once the earlier ones are
    conjugate), so the two agree to rounding over a few iterations."""
    n, k = 12, 6
    A = spd(n, 15.0, 8)
    b = np.random.default_rng(9).standard_normal(n)
    h0 = np.linspace(0.7, 1.3, n)
    S_l, _, _, m_l, _ = bfgs.bfgs_quadratic(A, b, k, h0=h0, memory=memory)
    S_f, _, _, m_f, _ = bfgs.bfgs_quadratic(A, b, k, h0=h0)
    assert np.abs(S_l - S_f).max() <= 1e-10 * np.abs(S_f).max()
    assert np.abs(m_l - m_f).max() <= 1e-10 * np.abs(m_f).max()


def test_limited_memory_covering_all_pairs_is_full_bfgs():
    n, k = 8, 5
    A = spd(n, 10.0, 2)
    b = np.random.default_rng(3).standard_normal(n)
    S_l, _, _, _, _ = bfgs.bfgs_quadratic(A, b, k, damping=0.5, memory=k)
    S_f, _, _, _, _ = bfgs.bfgs_quadratic(A, b, k, damping=0.5)
    assert np.array_equal(S_l, S_f)
