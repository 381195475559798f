"""The pins are strong enough: plausible mistakes planted in a CPU copy of the
two-loop recursion (Alg. 2) each fail at least one pin.  CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import bfgs, twoloop

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq3_hand.json")


def two_loop_variant(h0, S, Y, v, mistake=None):
    k = len(S)
    r = [1.0 / (Y[i] @ S[i]) for i in range(k)]
    q = v.astype(np.float64).copy()
    a = np.zeros(k)
    order1 = range(k) if mistake == "first_loop_ascending" else range(k - 1, -1, -1)
    for i in order1:
        s_, y_ = (Y[i], S[i]) if mistake == "swap_s_y" else (S[i], Y[i])
        a[i] = r[i] * (s_ @ q)
        q = q - a[i] * y_
    z = q / h0 if mistake == "inverse_b0" else h0 * q
    for i in range(k):
        b = (Y[i] @ z) if mistake == "drop_rho" else r[i] * (Y[i] @ z)
        z = z + S[i] * ((b - a[i]) if mistake == "flip_sign" else (a[i] - b))
    return z


def pins_pass(fn):
    # golden hand cases
    for case in json.load(open(GOLDEN))["cases"]:
        f = lambda M: np.array([[a / b for a, b in row] for row in M], dtype=np.float64)
        h0 = np.array([a / b for a, b in case["h0"]])
        S, Y, B = f(case["S"]), f(case["Y"]), f(case["B"])
        got = np.array([fn(h0, S, Y, e) for e in np.eye(len(h0))])
        if np.abs(got - B).max() > 1e-12:
            return False
    # secant + symmetry on a random problem
    rng = np.random.default_rng(0)
    n = 20
    M = rng.standard_normal((n, n))
    A = M @ M.T + n * np.eye(n)
    S = rng.standard_normal((6, n))
    Y = S @ A
    h0 = rng.uniform(0.5, 2, n)
    if np.abs(fn(h0, S, Y, Y[-1]) - S[-1]).max() > 1e-10 * np.abs(S[-1]).max():
        return False
    u, v = rng.standard_normal((2, n))
    if abs(u @ fn(h0, S, Y, v) - v @ fn(h0, S, Y, u)) > 1e-10 * abs(u @ fn(h0, S, Y, v)):
        return False
    # quadratic termination
    S, Y, h, _, _ = bfgs.bfgs_quadratic(A, rng.standard_normal(n), n)
    B = np.array([fn(h, S, Y, e) for e in np.eye(n)])
    return np.abs(B - np.linalg.inv(A)).max() <= 1e-9 * np.abs(np.linalg.inv(A)).max()


def test_unmutated_copy_passes_and_matches_oracle():
    assert pins_pass(lambda h0, S, Y, v: two_loop_variant(h0, S, Y, v))
    assert pins_pass(lambda h0, S, Y, v: twoloop.two_loop(h0, S, Y, v))


@pytest.mark.parametrize("mistake", ["first_loop_ascending", "swap_s_y", "inverse_b0",
                                     "drop_rho", "flip_sign"])
def test_planted_mistake_is_caught(mistake):
    assert not pins_pass(lambda h0, S, Y, v: two_loop_variant(h0, S, Y, v, mistake))
