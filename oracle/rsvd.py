"""Single-pass randomized SVD of B_k - B_0 and the posterior variance (oracle,
test infrastructure only).

Alg. 3 sketches the operator A = B_k - B_0 (the difference Alg. 2 probes, whose
low-rank part enters eq. (10)) with a block of random vectors X and recovers a
symmetric low-rank factorisation from that single sketch.  rsvd() takes the
algorithm's steps in the paper's order:  the sketch E = A X; an orthonormal basis
Q of its range from the QR factorisation E = Q R; the small matrix Omega that
satisfies Omega (Q^T X) = Q^T E; its factorisation Omega = U_s Lambda U_s^T; and
the basis U = Q U_s of the leading `rank` directions.  posterior_diag() forms
diag(U Lambda U^T + B_0) of eq. (10), the variance of eq. (14) with C_m = I.

Readings where the paper leaves the method open:
  * Q R = E is LAPACK's Householder QR with the signs chosen so that R_ii >= 0;
  * Omega (Q^T X) = Q^T E is square and is solved by LU with partial pivoting,
    then symmetrised, (Omega + Omega^T) / 2, since the next step factors it as
    U_s Lambda U_s^T;
  * A is indefinite in general, so Lambda keeps its signs: eigenvalues ordered by
    |lambda| descending (ties: signed value descending, then index), each
    eigenvector's largest-magnitude entry made positive (lowest index on ties);
  * the oversampling columns are dropped after ordering.

Pinned by: exactness when rank + oversampling exceeds rank(B_k - B_0) (against a
dense eigendecomposition of the eq. (3) matrix), the Nystrom identity
Q Omega Q^T = E (X^T E)^-1 E^T, and diag(B_k) by unit-pulse probing.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .recursion import apply_hk


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
        E = apply_hk(h0, S, Y, X, subtract_b0=True)            # the sketch, (c, n)
    Em = E.T                                                     # n x c
    Xm = X.T
    Q, R = np.linalg.qr(Em, mode="reduced")                      # range basis
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    Q = Q * d
    R = d[:, None] * R
    T = Q.T @ Xm                                                 # Omega (Q^T X) = Q^T E
    F = Q.T @ Em
    lu, piv = scipy.linalg.lu_factor(T.T)
    Omega = scipy.linalg.lu_solve((lu, piv), F.T).T
    Omega = 0.5 * (Omega + Omega.T)
    lam, Us = np.linalg.eigh(Omega)                              # Omega = U_s Lambda U_s^T
    lam, Us = order_and_sign(lam, Us)
    V = Q @ Us[:, :rank]                                         # leading directions
    return dict(E=E, Q=Q, R=R, T=T, F=F, Omega=Omega, lam=lam, Us=Us,
                U=V.T.copy(), Sigma=lam[:rank].copy())


def rsvd_precond(h0, S, Y, X, rank: int, E=None):
    """Alg. 3 on the B_0-whitened difference A_w = B_0^-1/2 (B_k - B_0) B_0^-1/2, whose
    eigenvalues are those of B_k B_0^-1 - I (similar matrices): the view in which the
    retrieved operator "starts from the identity".  With V = X the probes the library
    stores, the whitened sketch is E_w = A_w X_w for X_w = B_0^1/2 X, computed as
    B_0^-1/2 ((B_k - B_0) X); then Q R = E_w, Omega (Q^T X_w) = Q^T E_w, and U, Sigma
    as in rsvd().  U is the whitened basis: B_k = B_0 + B_0^1/2 U diag(Sigma) U^T B_0^1/2."""
    h0 = np.asarray(h0, np.float64)
    X = np.asarray(X, np.float64)
    c, n = X.shape
    assert rank <= c <= n
    if E is None:
        E = apply_hk(h0, S, Y, X, subtract_b0=True)
    Ew = (E / np.sqrt(h0)).T
    Xw = (X * np.sqrt(h0)).T
    Q, R = np.linalg.qr(Ew, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    Q = Q * d
    R = d[:, None] * R
    T = Q.T @ Xw
    F = Q.T @ Ew
    lu, piv = scipy.linalg.lu_factor(T.T)
    Omega = scipy.linalg.lu_solve((lu, piv), F.T).T
    Omega = 0.5 * (Omega + Omega.T)
    lam, Us = np.linalg.eigh(Omega)
    lam, Us = order_and_sign(lam, Us)
    V = Q @ Us[:, :rank]
    return dict(E=E, Q=Q, T=T, Omega=Omega, lam=lam, U=V.T.copy(), Sigma=lam[:rank].copy())


def rsvd_two_pass(h0, S, Y, X, rank: int, precond: bool = False):
    """The two-pass variant (Halko et al.'s Q^T A Q): Q from the sketch as in rsvd()
    (or rsvd_precond()), then a second application of the operator to Q itself and
    Omega = Q^T (A Q), symmetrised, in place of the solve with Q^T X."""
    h0 = np.asarray(h0, np.float64)
    X = np.asarray(X, np.float64)
    c, n = X.shape
    E = apply_hk(h0, S, Y, X, subtract_b0=True)
    w = 1.0 / np.sqrt(h0) if precond else np.ones(n)
    Q, R = np.linalg.qr((E * w).T, mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    Q = Q * d
    AQ = (apply_hk(h0, S, Y, (Q * w[:, None]).T, subtract_b0=True) * w).T
    Omega = Q.T @ AQ
    Omega = 0.5 * (Omega + Omega.T)
    lam, Us = np.linalg.eigh(Omega)
    lam, Us = order_and_sign(lam, Us)
    V = Q @ Us[:, :rank]
    return dict(Q=Q, Omega=Omega, lam=lam, U=V.T.copy(), Sigma=lam[:rank].copy())


def posterior_diag_precond(h0, U, Sigma) -> np.ndarray:
    """diag(B_0 + B_0^1/2 U^T diag(Sigma) U B_0^1/2) with the whitened basis U (rank, n)."""
    h0 = np.asarray(h0, np.float64)
    U = np.asarray(U, np.float64)
    return h0 + h0 * (np.asarray(Sigma, np.float64)[:, None] * U * U).sum(axis=0)


def posterior_diag(h0, U, Sigma) -> np.ndarray:
    """diag(U^T diag(Sigma) U) + h0 with U of shape (rank, n)."""
    U = np.asarray(U, np.float64)
    return np.asarray(h0, np.float64) + (np.asarray(Sigma, np.float64)[:, None] * U * U).sum(axis=0)


def low_rank_apply(U, Sigma, W) -> np.ndarray:
    """(U^T diag(Sigma) U) W for W of shape (m, n); basis-independent comparison helper."""
    U = np.asarray(U, np.float64)
    return ((np.asarray(W, np.float64) @ U.T) * np.asarray(Sigma)) @ U
