"""Dense BFGS matrices (oracle, test infrastructure only).

inverse_hessian        eq. (3): B_{k+1} = (I - r s y^T) B_k (I - r y s^T) + r s s^T,
                       r = 1 / (y^T s), from B_0 = diag(h0), pairs in push order.
inverse_hessian_exact  the same recursion in exact rational arithmetic.
hessian_eq2            eq. (2): H_{k+1} = H_k + y y^T / (y^T s) - H_k s s^T H_k^T / (s^T H_k s),
                       from H_0 = diag(1/h0) (the Hessian whose inverse is B_0).

Pinned by: hand-derived golden matrices (tests/golden), the secant condition,
symmetry/positive definiteness, quadratic termination against numpy's inverse,
and the eq. (2) <-> eq. (3) inverse relation (Sherman-Morrison).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def inverse_hessian(h0, S, Y) -> np.ndarray:
    """Eq. (3) applied once per pair.  h0: (n,), S, Y: (k, n) (row i = s_i / y_i)."""
    h0 = np.asarray(h0, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n = h0.shape[0]
    B = np.diag(h0)
    I = np.eye(n)
    for s, y in zip(S, Y):
        r = 1.0 / float(y @ s)
        left = I - r * np.outer(s, y)
        right = I - r * np.outer(y, s)
        B = left @ B @ right + r * np.outer(s, s)
    return B


def inverse_hessian_exact(h0, S, Y):
    """Eq. (3) in exact rationals; inputs convertible to Fraction.  Returns a list of lists."""
    n = len(h0)
    F = lambda v: Fraction(v)
    B = [[F(h0[i]) if i == j else Fraction(0) for j in range(n)] for i in range(n)]
    for s, y in zip(S, Y):
        s = [F(v) for v in s]
        y = [F(v) for v in y]
        r = 1 / sum(a * b for a, b in zip(y, s))
        left = [[(1 if i == j else 0) - r * s[i] * y[j] for j in range(n)] for i in range(n)]
        right = [[(1 if i == j else 0) - r * y[i] * s[j] for j in range(n)] for i in range(n)]
        tmp = [[sum(left[i][m] * B[m][j] for m in range(n)) for j in range(n)] for i in range(n)]
        B = [[sum(tmp[i][m] * right[m][j] for m in range(n)) + r * s[i] * s[j] for j in range(n)]
             for i in range(n)]
    return B


def hessian_eq2(h0, S, Y) -> np.ndarray:
    """Eq. (2) Hessian recursion from H_0 = diag(1/h0)."""
    H = np.diag(1.0 / np.asarray(h0, dtype=np.float64))
    for s, y in zip(np.asarray(S, np.float64), np.asarray(Y, np.float64)):
        Hs = H @ s
        H = H + np.outer(y, y) / float(y @ s) - np.outer(Hs, H.T @ s) / float(s @ Hs)
    return H
