"""Shared test helpers: seeded inputs on both sides and error metrics."""
from __future__ import annotations

import numpy as np
import torch

from oracle.probes import round_to
from workloads import quadratic as wq

TOL = {"f64": 1e-12, "f32": 1e-6, "bf16": 1e-3}


def rel_f(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def col_max_rel(a, b) -> float:
    """Element-wise error per column: max over columns of max_i |a - b| / max_i |b|
    (rows of the (ncols, n) arrays are columns of the block)."""
    a = np.atleast_2d(np.asarray(a, np.float64))
    b = np.atleast_2d(np.asarray(b, np.float64))
    num = np.abs(a - b).max(axis=1)
    den = np.maximum(np.abs(b).max(axis=1), 1e-300)
    return float((num / den).max())


def sigma_err(got, ref) -> float:
    """max_i |got_i - ref_i| / |ref_0| after sorting both by signed value.  The ordering
    by |lambda| is not unique where two eigenvalues of opposite sign have nearly equal
    magnitude (rounding decides which comes first), so the spectra are compared as
    sets; sigma_order_ok checks the ordering itself."""
    got = np.sort(np.asarray(got, np.float64))
    ref = np.asarray(ref, np.float64)
    return float(np.abs(got - np.sort(ref)).max() / abs(ref[0]))


def sigma_order_ok(got, tol) -> bool:
    """|Sigma| is non-increasing, up to tol |Sigma_0| for near ties."""
    a = np.abs(np.asarray(got, np.float64))
    return bool((np.diff(a) <= tol * a[0]).all())


def gpu_input(x64: torch.Tensor, storage: str) -> torch.Tensor:
    """What the binding is handed: float64 for float64 storage, float32 otherwise."""
    return x64.to("cuda", torch.float64 if storage == "f64" else torch.float32)


def oracle_input(x64, storage: str) -> np.ndarray:
    """The stored values the GPU will compute with, rounded on the CPU."""
    x = x64.cpu().numpy() if isinstance(x64, torch.Tensor) else np.asarray(x64)
    return round_to(x, storage)


def h0_storage(h0_64, storage):
    x = h0_64.cpu().numpy() if isinstance(h0_64, torch.Tensor) else np.asarray(h0_64)
    return x.copy() if storage == "f64" else x.astype(np.float32).astype(np.float64)


def make_pairs(kind: str, nx: int, nz: int, k: int, seed: int = 0, precond: bool = False):
    """(problem, S, Y, h0_or_None) float64 on the CPU."""
    prob = wq.make_grid(nx, nz, seed)
    h0 = (1.0 / prob.diag()) if precond else None
    if kind == "cg":
        # stop once the gradient is at rounding level: later steps underflow float32
        S, Y, _ = wq.cg_pairs(prob, k, precond=h0, rel_tol=1e-12)
    else:
        S, Y = wq.random_secant_pairs(prob, k, seed=seed + 7)
    return prob, S, Y, h0


def gamma_of(S_q: np.ndarray, Y_q: np.ndarray) -> float:
    return float(S_q[0] @ Y_q[0]) / float(Y_q[0] @ Y_q[0])
