"""Smoothed, median-damped diagonal B_0 of eq. (4) (oracle, test infrastructure only).

The paper builds its initial inverse Hessian as B_0 = (H_0 + lambda I)^-1 from a
diagonal Hessian estimate H_0, smoothed the way the gradient is smoothed and
stabilised with the median of the smoothed estimate.  Readings used here (the
paper gives neither the smoother nor the exact damping rule):
  * the smoother is separable Gaussian per parameter field, weights
    exp(-t^2 / (2 sigma^2)) for |t| <= half, each 1-D pass divided by the weights
    that fall inside the grid (so a constant field stays constant);
  * lambda = damping * median(smoothed H_0), the median of the float32-rounded
    smoothed values (the mean of the two middle values when n is even);
  * h0 = 1 / (smoothed H_0 + lambda).

Pinned by: a constant field is left unchanged; a unit impulse away from the edges
becomes the outer product of the normalised weights; the median of a hand-written
list; the closed form 1 / ((1 + damping) c) for a constant field.
"""
from __future__ import annotations

import numpy as np


def gaussian_weights(sigma: float, half: int) -> np.ndarray:
    t = np.arange(-half, half + 1, dtype=np.float64)
    return np.exp(-0.5 * (t / sigma) ** 2)


def smooth_axis(f: np.ndarray, axis: int, w: np.ndarray) -> np.ndarray:
    """One renormalised Gaussian pass along `axis` (zero outside the grid)."""
    half = (w.shape[0] - 1) // 2
    m = f.shape[axis]
    out = np.zeros_like(f, dtype=np.float64)
    norm = np.zeros(m)
    for t in range(-half, half + 1):
        wt = w[t + half]
        lo, hi = max(0, -t), min(m, m - t)          # output indices j with j + t inside the grid
        if lo >= hi:
            continue
        src = [slice(None)] * f.ndim
        dst = [slice(None)] * f.ndim
        src[axis] = slice(lo + t, hi + t)
        dst[axis] = slice(lo, hi)
        out[tuple(dst)] += wt * f[tuple(src)]
        norm[lo:hi] += wt
    shape = [1] * f.ndim
    shape[axis] = m
    return out / norm.reshape(shape)


def smooth(h, nx: int, nz: int, nparam: int, sigma: float, half: int) -> np.ndarray:
    """x pass then z pass of each field; float64."""
    f = np.asarray(h, np.float64).reshape(nparam, nz, nx)
    w = gaussian_weights(sigma, half)
    return smooth_axis(smooth_axis(f, 2, w), 1, w).reshape(-1)


def precond_diag(h, nx: int, nz: int, nparam: int, sigma: float, half: int, damping: float = 1.0):
    """Returns (h0, hs, lambda): hs the smoothed estimate rounded to float32 (as stored),
    lambda = damping * median(hs), h0 = 1 / (hs + lambda) rounded to float32."""
    hs = smooth(h, nx, nz, nparam, sigma, half).astype(np.float32).astype(np.float64)
    lam = damping * float(np.median(hs))
    h0 = (1.0 / (hs + lam)).astype(np.float32).astype(np.float64)
    return h0, hs, lam
