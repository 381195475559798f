"""Learned diagonal initial inverse Hessian.

The paper replaces the scalar B_0 by diagonal preconditioners built from
wavefields (eqs. 4-8) and shows fewer iterations with them.  Here the diagonal
is predicted per (grid point, parameter) by a small network (8 -> 64 -> 64 -> 1,
GELU) trained on posterior variances that the method itself produces: the
diagonal of eq. (14) from a rank-r randomized SVD of H_k with the scalar
gamma I start.  Every step (features, forward, backward, Adam, exp) runs in the
library's kernels; this module only arranges the data.

Inputs of a model vector follow the field-major layout (param * nz + iz) * nx + ix.
"""
from __future__ import annotations

import math

import torch

from ._lib import Bfgs, Mlp, MLP_NPARAM


def init_params(seed: int = 0) -> torch.Tensor:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases: a float32 CPU vector."""
    g = torch.Generator().manual_seed(seed)
    parts = [torch.randn(64 * 8, generator=g, dtype=torch.float64) * math.sqrt(2.0 / 8), torch.zeros(64),
             torch.randn(64 * 64, generator=g, dtype=torch.float64) * math.sqrt(2.0 / 64), torch.zeros(64),
             torch.randn(64, generator=g, dtype=torch.float64) * math.sqrt(2.0 / 64), torch.zeros(1)]
    p = torch.cat([t.to(torch.float64) for t in parts]).float()
    assert p.numel() == MLP_NPARAM
    return p


def posterior_log_diag(S: torch.Tensor, Y: torch.Tensor, rank: int, oversample: int, seed: int,
                       storage: str = "f32", h0: torch.Tensor | None = None) -> torch.Tensor:
    """log of the posterior variance (eq. 14) of the history (S, Y) ((k, n) each):
    BFGS with h0 (gamma I when None), rank-`rank` randomized SVD of H_k - H_0."""
    n = S.shape[1]
    dt = torch.float64 if storage == "f64" else torch.float32
    H = Bfgs(n, S.shape[0], None if h0 is None else h0.to("cuda", dt), storage)
    for s, y in zip(S, Y):
        H.push_pair(s.to("cuda", dt), y.to("cuda", dt))
    H.rsvd(min(rank, H.k), oversample, seed)
    d = H.posterior_diag()
    out = torch.log(d.float())
    H.close()
    return out


def features(logD: torch.Tensor, gabs: torch.Tensor, nx: int, nz: int, sigma_scale: float) -> torch.Tensor:
    return Mlp.features(logD, gabs, nx, nz, sigma_scale)


def train(X: torch.Tensor, T: torch.Tensor, steps: int = 2000, batch: int = 65536, lr: float = 3e-3,
          seed: int = 0, params: torch.Tensor | None = None, log_every: int = 0):
    """Minibatch Adam on the mean squared error of log targets.  Returns (net, losses)."""
    X = X.to("cuda", torch.float32).contiguous()
    T = T.to("cuda", torch.float32).contiguous()
    N = X.shape[0]
    net = Mlp(init_params(seed) if params is None else params)
    g = torch.Generator(device="cuda").manual_seed(seed)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    b = min(batch, N)
    for step in range(steps):
        if b < N:
            idx = torch.randint(0, N, (b,), generator=g, device="cuda")
            xb, tb = X.index_select(0, idx), T.index_select(0, idx)
        else:
            xb, tb = X, T
        net.train_step(xb, tb, lr, loss)
        if log_every and (step % log_every == 0 or step == steps - 1):
            losses.append((step, float(loss.item())))
    return net, losses


def predict_h0(net: Mlp, logD: torch.Tensor, gabs: torch.Tensor, nx: int, nz: int,
               sigma_scale: float) -> torch.Tensor:
    """h0 = exp(network(features)) for every entry of the model vector (float32, device)."""
    return net.forward(features(logD, gabs, nx, nz, sigma_scale), exp_out=True)
