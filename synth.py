"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random numbers; it holds none of the transform's or the
checksums' arithmetic.  Every generator is numpy PCG64 seeded explicitly, so the
GPU path and the CPU oracle see the same arrays.

Workload recipes (the paper measures on random synthetic signals only):
  * uniform   : re, im i.i.d. U[-1, 1)
  * normal    : re, im i.i.d. N(0, 1)   (the paper's ROC study uses normal signals)
  * weights   : U[0, 1) real weights for the sum(w * |FFT(x)|^2) loss
  * ragged    : sizes drawn uniformly from {2^k, 3*2^k : 6 <= k <= 16}
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def signals(batch: int, N: int, seed: int, dist: str = "uniform",
            dtype=np.complex64) -> np.ndarray:
    """[batch, N] complex signals; dtype complex64 or complex128."""
    g = rng(seed)
    real_t = np.float32 if np.dtype(dtype) == np.complex64 else np.float64
    out = np.empty((batch, N), dtype=dtype)
    view = out.view(real_t).reshape(batch, N, 2)
    if dist == "uniform":
        # draw in chunks to bound temporary memory for GiB-sized inputs
        rows = max(1, (1 << 24) // max(1, 2 * N))
        for lo in range(0, batch, rows):
            hi = min(batch, lo + rows)
            view[lo:hi] = g.uniform(-1.0, 1.0, size=(hi - lo, N, 2)).astype(real_t)
    elif dist == "normal":
        rows = max(1, (1 << 24) // max(1, 2 * N))
        for lo in range(0, batch, rows):
            hi = min(batch, lo + rows)
            view[lo:hi] = g.standard_normal(size=(hi - lo, N, 2)).astype(real_t)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return out


def weights(shape, seed: int, dtype=np.float32) -> np.ndarray:
    return rng(seed).uniform(0.0, 1.0, size=shape).astype(dtype)


RAGGED_SIZES = tuple(sorted([1 << k for k in range(6, 17)] + [3 << k for k in range(6, 17)]))


def ragged_sizes(count: int, seed: int, menu=RAGGED_SIZES) -> np.ndarray:
    """`count` sizes drawn uniformly from the menu (int64)."""
    g = rng(seed)
    idx = g.integers(0, len(menu), size=count)
    return np.asarray(menu, dtype=np.int64)[idx]


def sample_indices(total: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct indices in [0, total), always including the first and last."""
    count = min(count, total)
    g = rng(seed)
    pick = set([0, total - 1]) if total > 1 else {0}
    if count > len(pick):
        extra = g.choice(total, size=count, replace=False)
        for v in extra:
            if len(pick) >= count:
                break
            pick.add(int(v))
    return np.array(sorted(pick), dtype=np.int64)
