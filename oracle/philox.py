"""Counter-based random numbers: Philox4x32-10 and Box-Muller normals.

Philox4x32-10 follows Salmon, Moraes, Dror & Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): a 4x32-bit counter and a 2x32-bit key; each of
the 10 rounds multiplies counter words 0 and 2 by two fixed odd constants
(64-bit products split into high and low halves), XORs the high halves with
the other two words and the key, and the key advances by two Weyl constants
between rounds.

Counter layout of this link (the paper asks for a binary source and AWGN,
Listing 1; it fixes no generator):

* key = (seed mod 2^32, seed >> 32)
* counter = (block j, codeword mod 2^32, codeword >> 32, stream)
* stream 0: information bits.  Bit i of codeword b is bit (i mod 32) of word
  (i // 32) mod 4 of Philox(key, (i // 128, b, stream 0)).
* stream 1: noise.  Symbols 2j and 2j+1 of codeword b use the four words of
  Philox(key, (j, b, stream 1)); a symbol takes (x_a, x_b) = words (0, 1) or
  (2, 3) and forms u_a = (x_a + 1) 2^-32 in (0, 1], u_b = x_b 2^-32,
  rho = sqrt(-2 ln u_a), g = rho (cos 2 pi u_b + j sin 2 pi u_b)
  (Box & Muller 1958).
* stream 2: real normals for a-priori LLRs (``normals_real``).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
SH = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on broadcastable uint32-valued arrays.

    Returns four ``uint32`` arrays."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> SH, p0 & MASK
        hi1, lo1 = p1 >> SH, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def _key(seed: int):
    return np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF)


def source_bits(seed: int, cw0: int, B: int, k: int) -> np.ndarray:
    """Information bits ``u8[B][k]`` of codewords ``cw0 .. cw0+B-1`` (stream 0)."""
    k0, k1 = _key(seed)
    nblk = -(-k // 128)
    b = (np.arange(B, dtype=np.uint64) + np.uint64(cw0))[:, None]
    j = np.arange(nblk, dtype=np.uint64)[None, :]
    w = philox4x32_10(j, b & MASK, b >> SH, np.uint64(0), k0, k1)
    words = np.stack(w, axis=-1).reshape(B, nblk * 4)        # word index = i // 32
    i = np.arange(k)
    bits = (words[:, i // 32] >> (i % 32).astype(np.uint32)) & np.uint32(1)
    return bits.astype(np.uint8)


def normals(seed: int, cw0: int, B: int, S: int) -> np.ndarray:
    """Complex standard normals ``g`` (E|g|^2 = 2) ``complex128[B][S]`` (stream 1)."""
    k0, k1 = _key(seed)
    npair = -(-S // 2)
    b = (np.arange(B, dtype=np.uint64) + np.uint64(cw0))[:, None]
    j = np.arange(npair, dtype=np.uint64)[None, :]
    x0, x1, x2, x3 = philox4x32_10(j, b & MASK, b >> SH, np.uint64(1), k0, k1)
    xa = np.stack([x0, x2], axis=-1).reshape(B, 2 * npair)[:, :S].astype(np.float64)
    xb = np.stack([x1, x3], axis=-1).reshape(B, 2 * npair)[:, :S].astype(np.float64)
    ua = (xa + 1.0) * 2.0 ** -32
    ub = xb * 2.0 ** -32
    rho = np.sqrt(-2.0 * np.log(ua))
    return rho * np.cos(2 * np.pi * ub) + 1j * rho * np.sin(2 * np.pi * ub)


def normals_real(seed: int, cw0: int, B: int, n: int, stream: int = 2) -> np.ndarray:
    """Real standard normals ``float64[B][n]`` (stream 2: the a-priori LLRs
    of EXIT simulations).  Entries 4j .. 4j+3 of codeword b come from
    Philox(key, (j, b, stream)): Box-Muller on words (0, 1) gives entries
    4j (cosine) and 4j+1 (sine), on words (2, 3) entries 4j+2 and 4j+3, with
    u_a, u_b as for the channel noise."""
    k0, k1 = _key(seed)
    nblk = -(-n // 4)
    b = (np.arange(B, dtype=np.uint64) + np.uint64(cw0))[:, None]
    j = np.arange(nblk, dtype=np.uint64)[None, :]
    x0, x1, x2, x3 = philox4x32_10(j, b & MASK, b >> SH, np.uint64(stream), k0, k1)
    out = np.empty((B, nblk, 4))
    for col, (xa, xb) in enumerate(((x0, x1), (x2, x3))):
        ua = (xa.astype(np.float64) + 1.0) * 2.0 ** -32
        ub = xb.astype(np.float64) * 2.0 ** -32
        rho = np.sqrt(-2.0 * np.log(ua))
        out[:, :, 2 * col] = rho * np.cos(2 * np.pi * ub)
        out[:, :, 2 * col + 1] = rho * np.sin(2 * np.pi * ub)
    return out.reshape(B, nblk * 4)[:, :n]
