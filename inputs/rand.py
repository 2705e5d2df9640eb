"""Plain seeded random arrays used as test inputs (no link arithmetic)."""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def gaussian(seed: int, shape, scale: float = 1.0, mean: float = 0.0, dtype=np.float64) -> np.ndarray:
    return (mean + scale * rng(seed).standard_normal(shape)).astype(dtype)


def uniform(seed: int, shape, lo: float, hi: float, dtype=np.float64) -> np.ndarray:
    return rng(seed).uniform(lo, hi, shape).astype(dtype)


def bits(seed: int, shape) -> np.ndarray:
    return rng(seed).integers(0, 2, shape, dtype=np.uint8)


def int8_uniform(seed: int, shape, lo: int, hi: int) -> np.ndarray:
    return rng(seed).integers(lo, hi + 1, shape).astype(np.int8)
