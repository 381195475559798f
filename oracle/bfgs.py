"""Full-history BFGS with an exact line search on a quadratic (oracle, test
infrastructure only).

The search direction is Alg. 1's p = -B_k g computed by the eq. (3) recursion
with every pair kept and a fixed initial inverse Hessian B_0 (full-memory
L-BFGS is BFGS, and B_0 then no longer changes with the iteration).  With no
B_0 supplied, the first step is p = -g and B_0 = gamma I with
gamma = s_0^T y_0 / y_0^T y_0 from the first pair, then frozen.

The step length minimises the quadratic exactly along p (times `damping`, which
keeps the Wolfe conditions for damping in (0, 1] and leaves S^T Y far from
diagonal).  s = alpha p, y = A s, g <- g + y.

`memory` > 0 is the limited-memory form the paper compares with full-memory BFGS
(L-BFGS, the 2-D Marmousi section): the recursion runs over the last `memory`
pairs only, with the same fixed B_0.

Used only to pin the input generator (its conjugate-gradient pairs are BFGS
pairs) and the oracle itself (quadratic termination, hereditary secant
conditions).  Never feeds the GPU library.
"""
from __future__ import annotations

import numpy as np

from .recursion import apply_hk


def bfgs_quadratic(A, b, k: int, h0=None, damping: float = 1.0, memory: int = 0):
    A = np.asarray(A, np.float64)
    b = np.asarray(b, np.float64)
    n = b.shape[0]
    m = np.zeros(n)
    g = -b.copy()
    S, Y = [], []
    h = None if h0 is None else np.asarray(h0, np.float64)
    gnorm = [float(np.linalg.norm(g))]
    for _ in range(k):
        if not S and h is None:
            p = -g
        else:
            keep = slice(-memory, None) if memory > 0 else slice(None)
            p = -apply_hk(h, np.array(S[keep]), np.array(Y[keep]), g)
        Ap = A @ p
        alpha = damping * (-(g @ p) / (p @ Ap))
        s = alpha * p
        y = A @ s
        m = m + s
        g = g + y
        S.append(s)
        Y.append(y)
        if h is None:
            h = np.full(n, float(s @ y) / float(y @ y))
        gnorm.append(float(np.linalg.norm(g)))
        if gnorm[-1] == 0.0:
            break
    return np.array(S), np.array(Y), h, m, gnorm
