"""Pins for the oracle's randomized SVD (Alg. 3), posterior variance (eq. 10/14)
and probe generator — CPU only."""
import numpy as np
import pytest
import scipy.stats

from oracle import dense, recursion, rsvd, probes, bfgs
from workloads import quadratic as wq
import torch


def cg_problem(n_grid=(12, 8), k=10, seed=0, precond=False):
    prob = wq.make_grid(n_grid[0], n_grid[1], seed)
    M = prob.D.reciprocal() if precond else None
    S, Y, _ = wq.cg_pairs(prob, k, precond=M)
    S, Y = S.numpy(), Y.numpy()
    if precond:
        h0 = M.numpy()
    else:
        h0 = np.full(prob.n, S[0] @ Y[0] / (Y[0] @ Y[0]))
    return prob, S, Y, h0


@pytest.mark.parametrize("precond", [False, True])
def test_rsvd_exact_when_oversampled(precond):
    """rank(B_k - B_0) <= k + 1 on a quadratic with fixed B_0, so rank k, p >= 2 is exact:
    U Sigma U^T equals the dense eq. (3) difference and Sigma its top eigenvalues."""
    prob, S, Y, h0 = cg_problem(k=10, precond=precond)
    n, k = prob.n, S.shape[0]
    Bdiff = dense.inverse_hessian(h0, S, Y) - np.diag(h0)
    ev = np.linalg.eigvalsh(Bdiff)
    ev = ev[np.argsort(-np.abs(ev))]
    assert np.abs(ev[k + 1:]).max() <= 1e-12 * np.abs(ev[0])      # the rank bound itself
    X = probes.normal_block(n, k + 5, seed=3)
    out = rsvd.rsvd(h0, S, Y, X, rank=k + 1)
    rec = (out["U"].T * out["Sigma"]) @ out["U"]
    assert np.abs(rec - Bdiff).max() <= 1e-11 * np.abs(Bdiff).max()
    np.testing.assert_allclose(out["Sigma"], ev[:k + 1], rtol=0, atol=1e-11 * abs(ev[0]))
    # orthonormal basis
    np.testing.assert_allclose(out["U"] @ out["U"].T, np.eye(k + 1), atol=1e-12)
    # posterior diagonal = diag(B_k) when exact, also by unit-pulse probing (Alg. 2)
    d = rsvd.posterior_diag(h0, out["U"], out["Sigma"])
    Bk = Bdiff + np.diag(h0)
    np.testing.assert_allclose(d, np.diag(Bk), rtol=1e-11)
    idx = np.random.default_rng(0).choice(n, 16, replace=False)
    pulses = np.eye(n)[idx]
    col = recursion.apply_hk(h0, S, Y, pulses)
    np.testing.assert_allclose(d[idx], col[np.arange(16), idx], rtol=1e-11)


def test_nystrom_identity():
    """Q Omega Q^T = E (X^T E)^-1 E^T when Q^T X is invertible (algebra of Alg. 3)."""
    prob = wq.make_grid(10, 6, 1)
    S, Y = wq.random_secant_pairs(prob, 8, seed=2)            # rank(B - B0) = 16
    S, Y = S.numpy(), Y.numpy()
    h0 = np.full(prob.n, 0.7)
    X = probes.normal_block(prob.n, 12, seed=5)
    out = rsvd.rsvd(h0, S, Y, X, rank=12)
    E = out["E"].T
    Xm = X.T
    lhs = out["Q"] @ out["Omega"] @ out["Q"].T
    rhs = E @ np.linalg.solve(Xm.T @ E, E.T)
    assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(rhs).max()
    # before symmetrisation Omega was already symmetric up to rounding (X^T E symmetric)
    assert np.abs(out["Omega"] - out["Omega"].T).max() == 0.0


def test_ordering_and_sign_rule():
    lam = np.array([0.5, -2.0, 2.0, 1e-3])
    Us = np.array([[0.0, -0.6, 0.8, 0.0], [1.0, 0.8, 0.6, 0.0], [0.0, 0.0, 0.0, -1.0]])
    l2, U2 = rsvd.order_and_sign(lam, Us)
    np.testing.assert_array_equal(l2, [2.0, -2.0, 0.5, 1e-3])
    np.testing.assert_array_equal(U2[:, 0], [0.8, 0.6, 0.0])
    np.testing.assert_array_equal(U2[:, 1], [-0.6, 0.8, 0.0])
    np.testing.assert_array_equal(U2[:, 3], [0.0, 0.0, 1.0])


def test_rank_truncation_error_bounded():
    """With rank + p < rank(B - B0) the result is an approximation; its error must stay
    below the first dropped eigenvalue times a modest factor (sanity bound)."""
    prob = wq.make_grid(10, 6, 1)
    S, Y = wq.random_secant_pairs(prob, 10, seed=4)
    S, Y = S.numpy(), Y.numpy()
    h0 = np.full(prob.n, 0.5)
    Bdiff = dense.inverse_hessian(h0, S, Y) - np.diag(h0)
    ev = np.linalg.eigvalsh(Bdiff)
    ev = ev[np.argsort(-np.abs(ev))]
    X = probes.normal_block(prob.n, 18, seed=1)
    out = rsvd.rsvd(h0, S, Y, X, rank=8)
    rec = (out["U"].T * out["Sigma"]) @ out["U"]
    err = np.linalg.norm(rec - Bdiff, 2)
    assert err <= 50 * abs(ev[8])


# --- probes ------------------------------------------------------------------------------
def test_philox_matches_numpy_philox():
    """numpy.random.Philox is Philox4x64-10; it pre-increments its counter, so its first
    block is ours at counter (1, 0, 0, 0)."""
    for key in [0, 1, 12345, 2**63 + 17]:
        bg = np.random.Philox(key=key)
        raw = bg.random_raw(8)
        k = np.array([key & (2**64 - 1), 0], dtype=np.uint64)
        np.testing.assert_array_equal(probes.philox4x64_10([1, 0, 0, 0], k), raw[:4])
        np.testing.assert_array_equal(probes.philox4x64_10([2, 0, 0, 0], k), raw[4:])
    bg = np.random.Philox(counter=[5, 7, 0, 0], key=[9, 3])
    np.testing.assert_array_equal(probes.philox4x64_10([6, 7, 0, 0], [9, 3]), bg.random_raw(4))


def test_normals_distribution_and_addressing():
    X = probes.normal_block(4099, 16, seed=42)
    flat = X.ravel()
    assert abs(flat.mean()) < 0.01
    assert abs(flat.var() - 1) < 0.01
    assert scipy.stats.kstest(flat, "norm").pvalue > 1e-3
    c = np.corrcoef(X)
    assert np.abs(c - np.eye(16)).max() < 0.06
    for (r, j) in [(0, 0), (1, 0), (2, 5), (3, 15), (4098, 9)]:
        assert probes.normal_entry(42, r, j) == X[j, r]
    assert not np.array_equal(probes.normal_block(64, 2, 1), probes.normal_block(64, 2, 2))


def test_round_to_storage():
    x = np.array([1.0 + 2.0**-9, 1.0 + 3 * 2.0**-9, 1.0 + 2.0**-30, -3.0e38 * 1.5])
    np.testing.assert_array_equal(probes.round_to(x[:3], "bf16"), [1.0, 1.0 + 2.0**-7, 1.0])
    assert np.isinf(probes.round_to(x[3:], "f32")[0])
    assert probes.round_to([1.0 + 2.0**-30], "f32")[0] == 1.0


def test_box_muller_pairs_against_numpy_philox():
    """Each counter block gives two Box-Muller pairs: rows 4q, 4q+1 from (u_0, u_1) and
    rows 4q+2, 4q+3 from (u_2, u_3).  Against numpy's Philox (a library generator):
    the pair's squared radius is -2 ln u_0 (resp. u_2) and its angle 2 pi u_1 (resp.
    u_3), with u = ((x >> 11) + 1) 2^-53 of the raw 64-bit outputs."""
    seed = 77
    X = probes.normal_block(64, 3, seed)
    M = 2**64 - 1
    for col in range(3):
        for q in range(16):
            # numpy's Philox increments its 256-bit counter before each block: start one below
            before = [q - 1, col, 0, 0] if q > 0 else ([M, col - 1, 0, 0] if col > 0 else [M, M, M, M])
            bg = np.random.Philox(counter=np.array(before, np.uint64), key=np.array([seed, 0], np.uint64))
            raw = bg.random_raw(4)
            u = ((raw >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
            for h in range(2):
                z0, z1 = X[col, 4 * q + 2 * h], X[col, 4 * q + 2 * h + 1]
                assert z0 * z0 + z1 * z1 == pytest.approx(-2.0 * np.log(u[2 * h]), rel=1e-13)
                ang = np.arctan2(z1, z0) % (2 * np.pi)
                assert abs(ang - 2 * np.pi * u[2 * h + 1]) <= 1e-12 or abs(abs(ang - 2 * np.pi * u[2 * h + 1]) - 2 * np.pi) <= 1e-12


def test_box_muller_pair_members_independent():
    """Within a column, the two members of a pair (rows 4q, 4q+1) and neighbouring
    pairs are uncorrelated, and so are their squares (the cos/sin members of one
    Box-Muller pair are independent normals)."""
    X = probes.normal_block(400_000, 2, seed=9)
    for col in range(2):
        x = X[col]
        for a, b in [(0, 1), (2, 3), (1, 2), (0, 2)]:
            u, v = x[a::4], x[b::4]
            assert abs(np.corrcoef(u, v)[0, 1]) < 0.015
            assert abs(np.corrcoef(u * u, v * v)[0, 1]) < 0.015


# --- preconditioned and two-pass variants ---------------------------------------------------
def _small_history(n=60, k=8, seed=3):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((n, n))
    A = M @ M.T / n + np.eye(n)
    S = rng.standard_normal((k, n))
    Y = S @ A
    h0 = rng.uniform(0.3, 3.0, n)
    return h0, S, Y


def test_precond_sigma_is_spectrum_of_bk_b0inv_minus_identity():
    """The whitened difference's eigenvalues are those of B_k B_0^-1 - I (the operator the
    paper says starts from the identity), and when rank + p >= rank(B_k - B_0) the
    factorisation is exact: B_0 + B_0^1/2 U Sigma U^T B_0^1/2 = B_k."""
    h0, S, Y = _small_history()
    n, k = h0.shape[0], S.shape[0]
    Bk = dense.inverse_hessian(h0, S, Y)
    ev = np.linalg.eigvals(Bk @ np.diag(1.0 / h0) - np.eye(n)).real
    ev = ev[np.argsort(-np.abs(ev))]
    X = probes.normal_block(n, 2 * k + 6, 5)
    out = rsvd.rsvd_precond(h0, S, Y, X, 2 * k)
    np.testing.assert_allclose(np.sort(out["Sigma"]), np.sort(ev[:2 * k]), rtol=0, atol=1e-10 * abs(ev[0]))
    W = np.sqrt(h0)[:, None] * out["U"].T
    rec = np.diag(h0) + (W * out["Sigma"]) @ W.T
    assert np.abs(rec - Bk).max() <= 1e-10 * np.abs(Bk).max()
    np.testing.assert_allclose(rsvd.posterior_diag_precond(h0, out["U"], out["Sigma"]), np.diag(Bk), rtol=1e-10)


@pytest.mark.parametrize("precond", [False, True])
def test_two_pass_is_exact_and_symmetric(precond):
    h0, S, Y = _small_history(seed=7)
    n, k = h0.shape[0], S.shape[0]
    Bk = dense.inverse_hessian(h0, S, Y)
    X = probes.normal_block(n, 2 * k + 4, 9)
    out = rsvd.rsvd_two_pass(h0, S, Y, X, 2 * k, precond=precond)
    if precond:
        W = np.sqrt(h0)[:, None] * out["U"].T
        rec = np.diag(h0) + (W * out["Sigma"]) @ W.T
    else:
        rec = np.diag(h0) + (out["U"].T * out["Sigma"]) @ out["U"]
    assert np.abs(rec - Bk).max() <= 1e-10 * np.abs(Bk).max()
    single = (rsvd.rsvd_precond if precond else rsvd.rsvd)(h0, S, Y, X, 2 * k)
    np.testing.assert_allclose(np.sort(out["Sigma"]), np.sort(single["Sigma"]), atol=1e-10 * abs(single["Sigma"][0]))
