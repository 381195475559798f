"""Learned diagonal preconditioner network (oracle, test infrastructure only).

The paper builds its initial inverse Hessian B_0 from diagonal Hessian
estimates computed from wavefields (preconditioners P1-P4, eqs. 4-8).  The
learned analogue predicts log h0 per (grid point, parameter) with an MLP
8 -> 64 -> 64 -> 1 with GELU (x Phi(x), exact erf) activations; h0 = exp(output).

Parameters, flattened in this order (4801 values):
    W1 (64 x 8, row-major), b1 (64), W2 (64 x 64, row-major), b2 (64), w3 (64), b3 (1)
Loss: mean squared error on log targets.  Optimiser: Adam (Kingma & Ba, 2015).

Features of point (param p, iz, ix), "own" parameter first:
    [logD_p, logD_{p+1}, logD_{p+2}, |g0|_p, |g0|_{p+1}, |g0|_{p+2}, iz / (nz - 1), sigma_scale]
(indices mod 3), i.e. the diagonal of the model operator, the initial gradient
magnitude, the depth and the smoothing scale at that point.

Pinned by: central finite differences of the loss (float64), Adam's closed-form
first step (lr * sign(g)), and a hand-checked feature layout.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

SIZES = [(64, 8), (64,), (64, 64), (64,), (64,), (1,)]
NPARAM = 4801
SQRT2 = math.sqrt(2.0)
INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def unflatten(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (NPARAM,)
    out, o = [], 0
    for shp in SIZES:
        sz = int(np.prod(shp))
        out.append(p[o:o + sz].reshape(shp))
        o += sz
    return out


def flatten(parts):
    return np.concatenate([np.asarray(a, np.float64).ravel() for a in parts])


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases, float64."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((64, 8)) * math.sqrt(2.0 / 8)
    W2 = rng.standard_normal((64, 64)) * math.sqrt(2.0 / 64)
    w3 = rng.standard_normal(64) * math.sqrt(2.0 / 64)
    return flatten([W1, np.zeros(64), W2, np.zeros(64), w3, np.zeros(1)])


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * INV_SQRT_2PI * np.exp(-0.5 * x * x)


def forward(p, X, keep=False):
    W1, b1, W2, b2, w3, b3 = unflatten(p)
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = gelu(z1)
    z2 = h1 @ W2.T + b2
    h2 = gelu(z2)
    out = h2 @ w3 + b3[0]
    if keep:
        return out, (X, z1, h1, z2, h2)
    return out


def loss_and_grad(p, X, t):
    """Mean squared error and its gradient with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unflatten(p)
    out, (X, z1, h1, z2, h2) = forward(p, X, keep=True)
    t = np.asarray(t, np.float64)
    N = out.shape[0]
    r = out - t
    loss = float(np.mean(r * r))
    dout = 2.0 * r / N
    gw3 = h2.T @ dout
    gb3 = np.array([dout.sum()])
    dz2 = np.outer(dout, w3) * gelu_grad(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * gelu_grad(z1)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(axis=0)
    return loss, flatten([gW1, gb1, gW2, gb2, gw3, gb3])


class Adam:
    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, p, g, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mhat = self.m / (1 - self.b1 ** self.t)
        vhat = self.v / (1 - self.b2 ** self.t)
        return p - lr * mhat / (np.sqrt(vhat) + self.eps)


def features(logD, gabs, nx: int, nz: int, sigma_scale: float) -> np.ndarray:
    """logD, gabs: field-major (3 * nz * nx,) arrays -> (n, 8) features."""
    L = np.asarray(logD, np.float64).reshape(3, nz, nx)
    G = np.asarray(gabs, np.float64).reshape(3, nz, nx)
    depth = np.broadcast_to((np.arange(nz) / max(nz - 1, 1))[:, None], (nz, nx))
    rows = []
    for p in range(3):
        q, r = (p + 1) % 3, (p + 2) % 3
        f = np.stack([L[p], L[q], L[r], G[p], G[q], G[r], depth, np.full((nz, nx), sigma_scale)], axis=-1)
        rows.append(f.reshape(-1, 8))
    return np.concatenate(rows, axis=0)


def round_bf16(p) -> np.ndarray:
    """The bfloat16 copy of float32 master weights the forward pass uses, as float64."""
    import torch
    return torch.from_numpy(np.asarray(p, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
