"""Alg. 3 single-pass randomized SVD and the posterior variance (oracle, test
infrastructure only).

rsvd(h0, S, Y, X, rank) follows Alg. 3 step by step on the operator
B_k - B_0 (the difference probed by Alg. 2, whose low-rank part enters
eq. (10)):
  1. E = (B_k - B_0) X                     Alg. 2 with its final subtraction
  2. Q R = E                               Householder QR (LAPACK), R_ii >= 0
  3. Omega (Q^T X) = Q^T E                 LU with partial pivoting on (Q^T X)^T,
                                           then Omega <- (Omega + Omega^T) / 2
  4. U_s Lambda U_s^T = Omega              symmetric eigendecomposition with signed
                                           eigenvalues, ordered by |lambda| descending
                                           (ties: signed value descending, then index);
                                           each eigenvector's largest-magnitude entry
                                           made positive (lowest index on ties)
  5. V = Q U_s, keeping the first `rank` columns; Sigma = the first `rank` eigenvalues
posterior_diag: diag(V Lambda V^T + B_0) (eq. (10)), the variance of eq. (14) with
C_m = I.

Readings (the paper leaves them open): the solve in step 3 is square and is done by
LU; Omega is symmetrised because step 4 writes its factorisation as U Lambda U^T;
B_k - B_0 is indefinite in general, so Lambda keeps signs; oversampling columns are
dropped after ordering.

Pinned by: exactness when rank + oversampling exceeds rank(B_k - B_0) (against a
dense eigendecomposition of the eq. (3) matrix), the Nystrom identity
Q Omega Q^T = E (X^T E)^-1 E^T, and diag(B_k) by unit-pulse probing (Alg. 2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .twoloop import two_loop


def order_and_sign(lam: np.ndarray, Us: np.ndarray):
    c = lam.shape[0]
    order = sorted(range(c), key=lambda i: (-abs(lam[i]), -lam[i], i))
    lam = lam[order].copy()
    Us = Us[:, order].copy()
    for i in range(c):
        col = Us[:, i]
        j = int(np.argmax(np.abs(col)))          # first maximum = lowest index on ties
        if col[j] < 0:
            Us[:, i] = -col
    return lam, Us


def rsvd(h0, S, Y, X, rank: int, E=None):
    """X: (c, n) probes (already rounded to storage).  Returns a dict of every step."""
    h0 = np.asarray(h0, np.float64)
    X = np.asarray(X, np.float64)
    c, n = X.shape
    assert rank <= c <= n
    if E is None:
        E = two_loop(h0, S, Y, X, subtract_b0=True)            # step 1, (c, n)
    Em = E.T                                                     # n x c
    Xm = X.T
    Q, R = np.linalg.qr(Em, mode="reduced")                      # step 2
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    Q = Q * d
    R = d[:, None] * R
    T = Q.T @ Xm                                                 # step 3
    F = Q.T @ Em
    lu, piv = scipy.linalg.lu_factor(T.T)
    Omega = scipy.linalg.lu_solve((lu, piv), F.T).T
    Omega = 0.5 * (Omega + Omega.T)
    lam, Us = np.linalg.eigh(Omega)                              # step 4
    lam, Us = order_and_sign(lam, Us)
    V = Q @ Us[:, :rank]                                         # step 5
    return dict(E=E, Q=Q, R=R, T=T, F=F, Omega=Omega, lam=lam, Us=Us,
                U=V.T.copy(), Sigma=lam[:rank].copy())


def posterior_diag(h0, U, Sigma) -> np.ndarray:
    """diag(U^T diag(Sigma) U) + h0 with U of shape (rank, n)."""
    U = np.asarray(U, np.float64)
    return np.asarray(h0, np.float64) + (np.asarray(Sigma, np.float64)[:, None] * U * U).sum(axis=0)


def low_rank_apply(U, Sigma, W) -> np.ndarray:
    """(U^T diag(Sigma) U) W for W of shape (m, n); basis-independent comparison helper."""
    U = np.asarray(U, np.float64)
    return ((np.asarray(W, np.float64) @ U.T) * np.asarray(Sigma)) @ U
