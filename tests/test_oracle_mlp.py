"""Pins for the learned-preconditioner oracle (CPU only)."""
import numpy as np
import pytest

from oracle import mlp


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(3) + 0.01 * rng.standard_normal(mlp.NPARAM)
    X = rng.standard_normal((37, 8))
    t = rng.standard_normal(37)
    loss, g = mlp.loss_and_grad(p, X, t)
    idx = rng.choice(mlp.NPARAM, 60, replace=False)
    idx = np.concatenate([idx, [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4799, 4800]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss_and_grad(p + e, X, t)[0] - mlp.loss_and_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_gelu_values_and_derivative():
    x = np.array([-3.0, -1.0, 0.0, 0.5, 2.0])
    # x Phi(x) with Phi the standard normal CDF (closed values at 0 and symmetric identity)
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    np.testing.assert_allclose(mlp.gelu(x) - mlp.gelu(-x), x, rtol=1e-15, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(x), (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h), rtol=1e-8)
    assert mlp.gelu_grad(np.array([0.0]))[0] == pytest.approx(0.5)


def test_adam_first_step_is_lr_sign():
    p = np.array([1.0, -2.0, 3.0])
    g = np.array([0.3, -5.0, 1e-3])
    opt = mlp.Adam(3, lr=0.01)
    p1 = opt.step(p, g)
    # bias correction makes m_hat = g and v_hat = g^2 at step 1: the step is lr g / (|g| + eps)
    np.testing.assert_allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=0, atol=1e-6)


def test_features_layout():
    nx, nz = 4, 3
    logD = np.arange(3 * nz * nx, dtype=float)
    gabs = 100 + np.arange(3 * nz * nx, dtype=float)
    F = mlp.features(logD, gabs, nx, nz, 1.0)
    assert F.shape == (3 * nz * nx, 8)
    # point (param 1, iz 2, ix 3): index (1 * nz + 2) * nx + 3 = 23
    i = (1 * nz + 2) * nx + 3
    m = nz * nx
    np.testing.assert_array_equal(F[i], [logD[i], logD[i + m], logD[i - m], gabs[i], gabs[i + m], gabs[i - m], 1.0, 1.0])


def test_training_reduces_loss():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((512, 8))
    t = np.log(1.0 / (np.exp(X[:, 0]) + 0.5))     # a smooth function of the first feature
    p = mlp.init_params(0)
    opt = mlp.Adam(mlp.NPARAM, lr=3e-3)
    l0 = mlp.loss_and_grad(p, X, t)[0]
    for _ in range(200):
        loss, g = mlp.loss_and_grad(p, X, t)
        p = opt.step(p, g)
    assert loss < 0.1 * l0


def test_forward_hand_value():
    """Forward pass on a sparse parameter set written out by hand: biases before the
    activation, GELU on both hidden layers, W2 read as (output unit, input unit) with
    W2[0, 1] != W2[1, 0].  Phi comes from scipy.stats.norm, not from the oracle's erf."""
    from scipy.stats import norm

    def g(x):
        return x * norm.cdf(x)

    W1, b1, W2, b2, w3, b3 = (np.zeros(s) for s in mlp.SIZES)
    W1[0, 0], W1[1, 1] = 1.0, 0.5
    b1[0], b1[1], b1[2] = 0.25, -0.5, 1.0
    W2[0, 1], W2[1, 0], W2[1, 2] = 2.0, -1.0, 0.5
    b2[0], b2[1], b2[3] = 0.1, -0.2, 0.7
    w3[0], w3[1], w3[3] = 1.0, 3.0, -2.0
    b3[0] = 0.05
    p = mlp.flatten([W1, b1, W2, b2, w3, b3])
    X = np.zeros((3, 8))
    X[0, 0] = 1.0
    X[1, 1] = 2.0
    X[2, :] = [-0.7, 1.3, 5.0, 5.0, 5.0, 5.0, 5.0, 5.0]   # features 2..7 have no weights
    want = []
    for x in X:
        h0_, h1_, h2_ = g(x[0] + 0.25), g(0.5 * x[1] - 0.5), g(1.0)
        z0 = 2.0 * h1_ + 0.1
        z1 = -1.0 * h0_ + 0.5 * h2_ - 0.2
        want.append(g(z0) + 3.0 * g(z1) - 2.0 * g(0.7) + 0.05)
    np.testing.assert_allclose(mlp.forward(p, X), want, rtol=1e-14, atol=1e-15)
