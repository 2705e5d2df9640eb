"""Bit/block error counting and Wilson confidence intervals.

``compute_ber(b, b_hat)`` closes the paper's Listing 1; the block error
rate is the figure the paper names for end-to-end evaluation (Sec. "Why we
decided to create Sionna").  A block error is a codeword with at least one
wrong information bit.
"""
from __future__ import annotations

import math

import numpy as np


def count_errors(u: np.ndarray, u_hat: np.ndarray, bins: np.ndarray | None = None,
                 nbins: int = 1) -> np.ndarray:
    """``int64[nbins][3]``: (bit errors, block errors, codewords) per bin."""
    u = np.asarray(u, dtype=np.uint8)
    u_hat = np.asarray(u_hat, dtype=np.uint8)
    B = u.shape[0]
    bins = np.zeros(B, dtype=np.int64) if bins is None else np.asarray(bins, dtype=np.int64)
    err = (u != u_hat).sum(axis=1)
    out = np.zeros((nbins, 3), dtype=np.int64)
    for b in range(nbins):
        sel = bins == b
        out[b, 0] = int(err[sel].sum())
        out[b, 1] = int((err[sel] > 0).sum())
        out[b, 2] = int(sel.sum())
    return out


def wilson(errors: int, trials: int, z: float = 1.959963984540054) -> tuple[float, float]:
    """Wilson score interval for a binomial proportion."""
    if trials == 0:
        return 0.0, 1.0
    p = errors / trials
    den = 1.0 + z * z / trials
    ctr = (p + z * z / (2 * trials)) / den
    half = z * math.sqrt(p * (1 - p) / trials + z * z / (4 * trials * trials)) / den
    return max(0.0, ctr - half), min(1.0, ctr + half)


def q_function(x):
    """Gaussian tail Q(x) = erfc(x / sqrt 2) / 2."""
    return 0.5 * math.erfc(x / math.sqrt(2.0))
