"""Gray QAM mapper, AWGN channel, demappers and the LLR quantizer.

The paper's Listing 1 builds ``Constellation("qam", m)``, maps code bits to
symbols, adds AWGN given the noise variance ``no`` and demaps with the exact
("app") demapper given the same ``no``.  Listing 2 trains against the LLRs
with a binary cross-entropy whose labels are the code bits, which makes an
LLR the logit of bit = 1.  The labelling and formulas below are textbook:
the square Gray QAM of 3GPP TS 38.211 Sec. 5.1 and the max-log / exact
bitwise posteriors.
"""
from __future__ import annotations

import itertools

import numpy as np


def pam_level(bits) -> int:
    """Gray PAM level of ``h`` bits a_0..a_{h-1}:
    (1-2a_0)(2^{h-1} - (1-2a_1)(2^{h-2} - ... - (1-2a_{h-1})))."""
    h = len(bits)
    v = 1
    for l in range(h - 1, 0, -1):
        v = 2 ** (h - l) - (1 - 2 * bits[l]) * v
    return (1 - 2 * bits[0]) * v


def constellation(m: int) -> np.ndarray:
    """Points ``complex128[2^m]`` indexed by the label read MSB-first as
    c_0 c_1 ... c_{m-1}.  BPSK (m=1) is x = 1 - 2 c_0.  Square QAM takes
    I bits c_0, c_2, ... and Q bits c_1, c_3, ..., with unit mean energy."""
    if m == 1:
        return np.array([1.0 + 0j, -1.0 + 0j])
    if m % 2:
        raise ValueError("square QAM needs even m")
    h = m // 2
    scale = np.sqrt(2.0 * (4 ** h - 1) / 3.0)
    pts = np.empty(2 ** m, dtype=np.complex128)
    for idx, lab in enumerate(itertools.product((0, 1), repeat=m)):
        pts[idx] = (pam_level(lab[0::2]) + 1j * pam_level(lab[1::2])) / scale
    return pts


def labels(m: int) -> np.ndarray:
    """``u8[2^m][m]`` label bits of each constellation index."""
    return np.array(list(itertools.product((0, 1), repeat=m)), dtype=np.uint8)


def map_bits(t: np.ndarray, m: int) -> np.ndarray:
    """Symbols ``complex128[B][S]`` for transmitted bits ``u8[B][S*m]``;
    symbol s takes bits t[s*m .. s*m+m-1] in order."""
    B, n = t.shape
    S = n // m
    tb = np.asarray(t, dtype=np.int64).reshape(B, S, m)
    idx = np.zeros((B, S), dtype=np.int64)
    for b in range(m):
        idx = idx * 2 + tb[:, :, b]
    return constellation(m)[idx]


def ebn0_to_n0(ebn0_db, rate: float, m: int):
    """N0 = 1 / (R m 10^(EbN0/10)) for unit symbol energy."""
    return 1.0 / (rate * m * 10.0 ** (np.asarray(ebn0_db, dtype=np.float64) / 10.0))


def awgn(x: np.ndarray, n0: np.ndarray, g: np.ndarray) -> np.ndarray:
    """y = x + sqrt(N0/2) g with complex standard normals g (E|g|^2 = 2),
    so that the complex noise has variance N0 (the ``no`` of Listing 1)."""
    n0 = np.asarray(n0, dtype=np.float64).reshape(-1, 1)
    return x + np.sqrt(n0 / 2.0) * g


def demap_bruteforce(y: np.ndarray, n0: np.ndarray, m: int, method: str) -> np.ndarray:
    """Boundary LLRs ``float64[B][S*m]`` by enumerating all 2^m points.

    exact:   L_i = ln sum_{x: b_i=1} e^{-|y-x|^2/N0} - ln sum_{x: b_i=0} e^{-|y-x|^2/N0}
    maxlog:  L_i = (min_{b_i=0} |y-x|^2 - min_{b_i=1} |y-x|^2) / N0
    """
    pts = constellation(m)
    lab = labels(m)
    n0 = np.asarray(n0, dtype=np.float64).reshape(-1, 1, 1)
    d2 = np.abs(y[:, :, None] - pts[None, None, :]) ** 2            # (B, S, 2^m)
    B, S = y.shape
    L = np.empty((B, S, m))
    for i in range(m):
        one = lab[:, i] == 1
        if method == "maxlog":
            L[:, :, i] = (d2[:, :, ~one].min(-1) - d2[:, :, one].min(-1)) / n0[:, :, 0]
        elif method == "exact":
            a1 = -d2[:, :, one] / n0
            a0 = -d2[:, :, ~one] / n0
            L[:, :, i] = _lse(a1) - _lse(a0)
        else:
            raise ValueError(method)
    return L.reshape(B, S * m)


def demap_prior_bruteforce(y: np.ndarray, n0: np.ndarray, m: int, method: str, La: np.ndarray,
                           extrinsic: bool = False) -> np.ndarray:
    """Demapper with prior ("Demapper with prior", Sec. III-B): bitwise LLRs
    ``float64[B][S*m]`` given a-priori LLRs ``La[B][S*m]`` (logits of bit 1)
    of the symbol's bits, by enumerating all 2^m points.  Each point's
    metric is ``-|y-x|^2/N0 + sum_j b_j(x) La_j`` (ln P(b_j) = b_j La_j -
    ln(1 + e^{La_j}); the second term is common to numerator and
    denominator).

    exact:   L_i = ln sum_{b_i=1} e^{metric} - ln sum_{b_i=0} e^{metric}
    maxlog:  L_i = max_{b_i=1} metric - max_{b_i=0} metric

    These are a-posteriori LLRs (they include La_i); ``extrinsic`` returns
    L_i - La_i, the part passed on in iterative demapping and decoding."""
    pts = constellation(m)
    lab = labels(m).astype(np.float64)                       # (2^m, m)
    B, S = y.shape
    La = np.asarray(La, dtype=np.float64).reshape(B, S, m)
    n0 = np.asarray(n0, dtype=np.float64).reshape(-1, 1, 1)
    metric = -np.abs(y[:, :, None] - pts[None, None, :]) ** 2 / n0 + La @ lab.T   # (B, S, 2^m)
    L = np.empty((B, S, m))
    for i in range(m):
        one = lab[:, i] == 1
        if method == "maxlog":
            L[:, :, i] = metric[:, :, one].max(-1) - metric[:, :, ~one].max(-1)
        elif method == "exact":
            L[:, :, i] = _lse(metric[:, :, one]) - _lse(metric[:, :, ~one])
        else:
            raise ValueError(method)
    if extrinsic:
        L = L - La
    return L.reshape(B, S * m)


def _lse(a: np.ndarray) -> np.ndarray:
    mx = a.max(-1)
    return mx + np.log(np.exp(a - mx[..., None]).sum(-1))


def demap_bpsk(y: np.ndarray, n0: np.ndarray) -> np.ndarray:
    """Closed form for BPSK: L = -4 Re(y) / N0."""
    return -4.0 * y.real / np.asarray(n0, dtype=np.float64).reshape(-1, 1)


def quantize(L: np.ndarray, scale: float = 2.0, sat: int = 31) -> np.ndarray:
    """q = clamp(rint(L * scale), -sat, sat), round half to even, int8."""
    return np.clip(np.rint(np.asarray(L) * scale), -sat, sat).astype(np.int8)
