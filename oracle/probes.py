"""Probe vectors for Alg. 3 (oracle, test infrastructure only).

The paper samples the operator with independent random vectors; the reading
used throughout is i.i.d. N(0, 1) entries from Philox4x64-10 keyed by the seed
with counter (row / 4, column), turned into normals by Box-Muller in float64
(see ``philox.c`` for the exact mapping), then rounded to the storage type:
float64 kept, float32 by round-to-nearest-even, bfloat16 by rounding that
float32 value to nearest-even.

Pinned by: the raw Philox stream against numpy.random.Philox (a library
implementation of the same generator), and moments / independence checks of
the normals.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from .recursion import lib


def philox4x64_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.empty(4, dtype=np.uint64)
    lib().oracle_philox4x64_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def normal_entry(seed: int, row: int, col: int) -> float:
    return float(lib().oracle_normal_entry(ctypes.c_uint64(seed), row, col))


def normal_block(n: int, ncols: int, seed: int) -> np.ndarray:
    """(ncols, n) float64: row j is probe column j."""
    out = np.empty((ncols, n), dtype=np.float64)
    lib().oracle_normal_block(n, ncols, ctypes.c_uint64(seed), out.ctypes.data)
    return out


def round_to(x, storage: str) -> np.ndarray:
    """Round float64 values to the storage type and return them as float64."""
    x = np.asarray(x, dtype=np.float64)
    if storage == "f64":
        return x.copy()
    x32 = x.astype(np.float32)
    if storage == "f32":
        return x32.astype(np.float64)
    if storage == "bf16":
        return torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    raise ValueError(storage)
