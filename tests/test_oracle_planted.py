"""The pins are strong enough: plausible mistakes planted in a CPU copy of the
eq. (3) recursion each fail at least one pin.  CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import bfgs, recursion

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq3_hand.json")


def recursion_variant(h0, S, Y, v, mistake=None):
    """B_k v by eq. (3) as a recursion on the pair index, with an optional mistake."""
    k = len(S)
    order = list(range(k))[::-1] if mistake == "reversed_pairs" else list(range(k))

    def level(m, v):
        if m == 0:
            return v / h0 if mistake == "inverse_b0" else h0 * v
        i = order[m - 1]
        s, y = (Y[i], S[i]) if mistake == "swap_s_y" else (S[i], Y[i])
        r = 1.0 if mistake == "drop_rho" else 1.0 / (y @ s)
        t = s @ v
        w = v - r * (y @ v) * s if mistake == "transpose_right" else v - r * t * y
        z = level(m - 1, w)
        u = y @ z
        if mistake == "drop_ss_term":
            return z - r * u * s
        return z + r * ((u - t) if mistake == "flip_sign" else (t - u)) * s

    return level(k, np.asarray(v, np.float64))


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
    assert pins_pass(lambda h0, S, Y, v: recursion_variant(h0, S, Y, v))
    assert pins_pass(lambda h0, S, Y, v: recursion.apply_hk(h0, S, Y, v))


@pytest.mark.parametrize("mistake", ["reversed_pairs", "swap_s_y", "inverse_b0", "drop_rho",
                                     "transpose_right", "drop_ss_term", "flip_sign"])
def test_planted_mistake_is_caught(mistake):
    assert not pins_pass(lambda h0, S, Y, v: recursion_variant(h0, S, Y, v, mistake))
