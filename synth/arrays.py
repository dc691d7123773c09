"""Seeded random iterates and directions (inputs only, no method arithmetic)."""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(shape, lo: float, hi: float, seed: int, dtype=np.float32) -> np.ndarray:
    """Uniform values in [lo, hi) of the given dtype."""
    return (lo + (hi - lo) * _rng(seed).random(shape)).astype(dtype)


def binary01(shape, seed: int, p: float = 0.5) -> np.ndarray:
    return (_rng(seed).random(shape) < p).astype(np.int8)


def spins(shape, seed: int) -> np.ndarray:
    return np.where(_rng(seed).random(shape) < 0.5, 1, -1).astype(np.int8)


def normal(shape, seed: int, dtype=np.float64) -> np.ndarray:
    return _rng(seed).standard_normal(shape).astype(dtype)


def integers(shape, lo: int, hi: int, seed: int, dtype=np.uint32) -> np.ndarray:
    return _rng(seed).integers(lo, hi, size=shape, dtype=np.int64).astype(dtype)
