"""Pins for the seeded input generators (CPU only)."""
import numpy as np
import pytest
import torch

from oracle import bfgs
from workloads import quadratic as wq


def dense_of(prob):
    n = prob.n
    return prob.matvec(torch.eye(n, dtype=torch.float64)).numpy()


def test_grid_operator_spd_and_structure():
    prob = wq.make_grid(30, 12, seed=0)
    A = dense_of(prob)
    assert np.abs(A - A.T).max() <= 1e-15
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0
    np.testing.assert_allclose(np.diag(A), prob.diag().numpy(), rtol=1e-14)
    # cross-parameter coupling 0.1 between co-located points of different fields
    m = prob.nz * prob.nx
    g_centre = wq.gaussian_taps()[wq.SMOOTH_HALF] ** 2
    assert A[5, m + 5] == pytest.approx(0.1 * g_centre, rel=1e-13)
    # the smoother is local: +-20 cells
    assert A[0, 21] == 0.0 and A[0, 20] != 0.0


def test_batched_matvec_matches_single():
    prob = wq.make_grid(17, 9, seed=3)
    X = torch.randn(4, prob.n, dtype=torch.float64)
    AX = prob.matvec(X)
    for j in range(4):
        torch.testing.assert_close(AX[j], prob.matvec(X[j]), rtol=0, atol=1e-14)


def test_dense_problem_recipe():
    prob = wq.make_problem("tiny")
    rng = np.random.default_rng(0)
    D = np.exp(rng.standard_normal(300))
    U = rng.standard_normal((300, 8)) * np.sqrt(1 / 8)
    np.testing.assert_array_equal(prob.A.numpy(), np.diag(D) + U @ U.T)


@pytest.mark.parametrize("precond", [False, True])
def test_cg_pairs_are_bfgs_pairs(precond):
    """Conjugate-gradient steps equal the steps of full-history BFGS with exact line search
    (oracle driver, Alg. 1 directions) started from the same B_0."""
    prob = wq.make_grid(8, 6, seed=2)
    A = dense_of(prob)
    h0 = (1.0 / prob.diag()).numpy() if precond else None
    S, Y, _ = wq.cg_pairs(prob, 15, precond=None if h0 is None else torch.as_tensor(h0))
    So, Yo, _, _, _ = bfgs.bfgs_quadratic(A, prob.b.numpy(), 15, h0=h0)
    np.testing.assert_allclose(S.numpy(), So, rtol=0, atol=1e-10 * np.abs(So).max())
    np.testing.assert_allclose(Y.numpy(), Yo, rtol=0, atol=1e-10 * np.abs(Yo).max())


def test_cg_pairs_conjugacy():
    prob = wq.make_grid(20, 10, seed=4)
    S, Y, gn = wq.cg_pairs(prob, 30)
    G = (S @ Y.T).numpy()
    d = np.abs(np.diag(G))
    off = np.abs(G - np.diag(np.diag(G))) / np.sqrt(np.outer(d, d))
    assert off.max() < 1e-6
    assert gn[-1] < gn[0]
    assert (np.diag(G) > 0).all()


def test_random_secant_pairs():
    prob = wq.make_grid(9, 5, seed=1)
    S, Y = wq.random_secant_pairs(prob, 6, seed=3)
    torch.testing.assert_close(Y, prob.matvec(S))
    G = (S @ Y.T).numpy()
    assert (np.diag(G) > 0).all()
    d = np.sqrt(np.outer(np.diag(G), np.diag(G)))
    assert (np.abs(G) / d - np.eye(6)).max() > 0.05           # not conjugate


def test_batch_shapes():
    shapes = wq.batch_shapes()
    assert len(shapes) == 64
    for s in shapes:
        assert 20 <= s["k"] <= 150
        assert s["n"] == 3 * s["nx"] * s["nz"]
        assert 4.0e4 < s["n"] < 1.1e6
        assert 1.5 < s["nx"] / s["nz"] < 6.5
    assert shapes == wq.batch_shapes()
