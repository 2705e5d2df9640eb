"""Polar codes: construction, encoder, CRC and the SC / SCL / SCL-CRC
decoders (the paper lists Polar codes and "SC, SCL, and SCL-CRC Polar
decoders" among its FEC features, Sec. III-B, and names the SCL decoder as
a custom-kernel case, Sec. IV-A).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this package.

The paper prints none of the algorithms; these are the textbook ones:

* Transform (Arikan 2009): x = u F^{(x)n}, F = [[1, 0], [1, 1]], natural
  order: x = [x_a + x_b, x_b] with x_a, x_b the transforms of the two
  halves of u.
* Construction: Bhattacharyya parameters of the synthetic channels from
  z = exp(-Es/N0) of the BPSK channel at a design Eb/N0, with the BEC
  recursion z -> (2z - z^2, z^2) for (upper, lower) child; the K indices
  with the smallest z carry information (ties to the larger index).
* CRC: polynomial division of the data bits (first bit highest degree,
  zero initial value, no reflection, no final xor); the r CRC bits follow
  the data in the last r information positions.
* SC decoding on LLRs lambda = ln P(0)/P(1) (= -L of the boundary): a node
  passes f(a, b) = sgn(a) sgn(b) min(|a|, |b|) to its left child and
  g(a, b, x) = b + (1 - 2x) a to its right child, and returns
  [x_a xor x_b, x_b]; a leaf decides u = [lambda < 0], frozen leaves 0.
* SCL (Tal & Vardy 2015) in the LLR form of Balatsoukas-Stimming et al.
  (2015) with the approximate path metric: a leaf adds |lambda| to the
  metric of a path whose bit differs from [lambda < 0].  At an information
  leaf every path forks (bit 0 then bit 1); of the candidates the L with
  the smallest metric survive (ties: lower parent slot, then bit 0).
  Slots: a parent whose two children survive keeps bit 0 in its slot and
  the bit-1 child moves to the lowest free slot; a parent with one
  surviving child keeps it in its slot; free slots are those of parents
  without surviving children.  The decision is the path with the smallest
  metric (ties: lowest slot); SCL-CRC takes, in that order, the first path
  whose CRC checks, else the first path.

Channel values are read with NaN as 0 and clamped to +-2^100 (the paper
says nothing of non-finite inputs; with the clamp every intermediate LLR and
metric stays finite, at most 2^100 times the 2N terms a node and a metric
sum, so no value is ever inf - inf).

Two arithmetic modes: "fp64" (float64) and "fp32" (every operation in IEEE
single precision, as the device computes it; f, the path metric and the
decisions involve only min, negation and one rounding per add, so the
device's results match bit for bit).
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------ transform

def transform(u: np.ndarray) -> np.ndarray:
    """x = u F^{(x)n} over GF(2) for rows u ``u8[B][N]``."""
    u = np.asarray(u, dtype=np.uint8)
    N = u.shape[-1]
    if N == 1:
        return u.copy()
    a = transform(u[..., : N // 2])
    b = transform(u[..., N // 2:])
    return np.concatenate([a ^ b, b], axis=-1)


def generator(n: int) -> np.ndarray:
    """F^{(x)n} as a dense ``u8[N][N]`` matrix (Kronecker power)."""
    G = np.array([[1]], dtype=np.uint8)
    F = np.array([[1, 0], [1, 1]], dtype=np.uint8)
    for _ in range(n):
        G = np.kron(G, F).astype(np.uint8)
    return G


# --------------------------------------------------------- construction

def bhattacharyya(n: int, design_ebn0_db: float, rate: float) -> np.ndarray:
    """Bhattacharyya parameters ``float64[N]`` of the synthetic channels,
    index i of u."""
    es_n0 = rate * 10.0 ** (design_ebn0_db / 10.0)
    z = np.array([np.exp(-es_n0)])
    for _ in range(n):
        nz = np.empty(2 * z.size)
        # child 0 of each node is the worse (check) channel, child 1 the
        # better (variable) channel; a node's children are adjacent after
        # the last step of the recursion (natural order: index bits from
        # the most significant down)
        nz[0::2] = 2 * z - z * z
        nz[1::2] = z * z
        z = nz
    return z


def info_mask(n: int, K: int, design_ebn0_db: float) -> np.ndarray:
    """``u8[N]``: 1 at the K most reliable indices (smallest Bhattacharyya
    parameter; equal values: the larger index first)."""
    N = 1 << n
    z = bhattacharyya(n, design_ebn0_db, K / N)
    order = sorted(range(N), key=lambda i: (z[i], -i))
    mask = np.zeros(N, dtype=np.uint8)
    mask[order[:K]] = 1
    return mask


# ------------------------------------------------------------------ CRC

def crc(bits: np.ndarray, poly: int, r: int) -> np.ndarray:
    """CRC remainder bits ``u8[..., r]`` (highest degree first) of rows of
    data bits: remainder of d(x) x^r modulo g(x) = x^r + poly."""
    bits = np.asarray(bits, dtype=np.uint8)
    flat = bits.reshape(-1, bits.shape[-1])
    out = np.zeros((flat.shape[0], r), dtype=np.uint8)
    g = np.array([(poly >> (r - 1 - j)) & 1 for j in range(r)], dtype=np.uint8)
    for b in range(flat.shape[0]):
        reg = np.zeros(r, dtype=np.uint8)
        for bit in flat[b]:
            fb = reg[0] ^ bit
            reg = np.concatenate([reg[1:], [0]]).astype(np.uint8)
            if fb:
                reg ^= g
        out[b] = reg
    return out.reshape(bits.shape[:-1] + (r,))


def crc_ok(bits_with_crc: np.ndarray, poly: int, r: int) -> np.ndarray:
    k = bits_with_crc.shape[-1] - r
    return (crc(bits_with_crc[..., :k], poly, r) == bits_with_crc[..., k:]).all(-1)


# -------------------------------------------------------------- encoder

def encode(data: np.ndarray, mask: np.ndarray, poly: int = 0, r: int = 0) -> np.ndarray:
    """Codewords ``u8[B][N]`` of data ``u8[B][K - r]``: CRC appended, the K
    bits placed at the information indices in increasing order, frozen 0."""
    data = np.asarray(data, dtype=np.uint8)
    info = np.flatnonzero(mask)
    bits = np.concatenate([data, crc(data, poly, r)], axis=-1) if r else data
    u = np.zeros((data.shape[0], mask.size), dtype=np.uint8)
    u[:, info] = bits
    return transform(u)


# ------------------------------------------------------------- decoders

def _f(a, b, dt):
    m = np.minimum(np.abs(a), np.abs(b))
    neg = (a < 0) ^ (b < 0)
    return np.where(neg, -m, m).astype(dt)


def _g(a, b, x, dt):
    return np.where(x.astype(bool), b - a, b + a).astype(dt)


def read_channel(lam, dt):
    """Channel LLRs as the decoders read them: NaN -> 0, clamped to
    +-2^100."""
    lam = np.asarray(lam, dtype=dt)
    return np.clip(np.where(np.isnan(lam), dt(0), lam), dt(-2.0 ** 100), dt(2.0 ** 100)).astype(dt)


def sc_decode(lam: np.ndarray, mask: np.ndarray, mode: str = "fp64") -> np.ndarray:
    """Successive cancellation: ``u_hat u8[N]`` for channel LLRs
    ``lam[N]`` (ln P(0)/P(1))."""
    dt = np.float32 if mode == "fp32" else np.float64
    lam = read_channel(lam, dt)

    def rec(l, m):
        N = l.size
        if N == 1:
            u = 0 if not m[0] else int(l[0] < 0)
            return np.array([u], np.uint8), np.array([u], np.uint8)
        h = N // 2
        ua, xa = rec(_f(l[:h], l[h:], dt), m[:h])
        ub, xb = rec(_g(l[:h], l[h:], xa, dt), m[h:])
        return np.concatenate([ua, ub]), np.concatenate([xa ^ xb, xb])

    return rec(lam, np.asarray(mask))[0]


def scl_decode(lam: np.ndarray, mask: np.ndarray, L: int, poly: int = 0, r: int = 0,
               mode: str = "fp64"):
    """Successive-cancellation list decoding with list size L (SCL-CRC when
    r > 0).  Returns (u_hat u8[N] of the chosen path, metrics of the final
    list by slot, u_hat of every slot)."""
    dt = np.float32 if mode == "fp32" else np.float64
    lam = read_channel(lam, dt)
    mask = np.asarray(mask)
    N = lam.size
    n = N.bit_length() - 1
    # per slot: LLRs of the current node at every stage (stage s has 2^s
    # values; stage n is the channel), left-child partial sums per stage,
    # decided bits, metric, active flag
    alpha = [[None] * (n + 1) for _ in range(L)]
    beta = [[None] * (n + 1) for _ in range(L)]
    uh = np.zeros((L, N), dtype=np.uint8)
    pm = np.zeros(L, dtype=dt)
    active = np.zeros(L, dtype=bool)
    active[0] = True
    for s in range(L):
        alpha[s][n] = lam
    for i in range(N):
        top = n - 1 if i == 0 else (i & -i).bit_length() - 1
        for p in np.flatnonzero(active):
            for s in range(top, -1, -1):
                par = alpha[p][s + 1]
                h = par.size // 2
                if s == top and i != 0:
                    alpha[p][s] = _g(par[:h], par[h:], beta[p][s], dt)
                else:
                    alpha[p][s] = _f(par[:h], par[h:], dt)
        leaf = {p: alpha[p][0][0] for p in np.flatnonzero(active)}
        if not mask[i]:
            for p, l in leaf.items():
                uh[p, i] = 0
                if l < 0:
                    pm[p] = dt(pm[p] + abs(l))
        else:
            cand = []  # (metric, parent slot, bit)
            for p, l in leaf.items():
                hard = int(l < 0)
                for bit in (0, 1):
                    m = pm[p] if bit == hard else dt(pm[p] + abs(l))
                    cand.append((m, p, bit))
            cand.sort(key=lambda c: (c[0], c[1], c[2]))
            keep = cand[:L]
            kept = {}
            for m, p, bit in keep:
                kept.setdefault(p, []).append((bit, m))
            free = sorted(set(range(L)) - set(kept.keys()))
            new_alpha = [row[:] for row in alpha]
            new_beta = [row[:] for row in beta]
            new_uh = uh.copy()
            new_pm = pm.copy()
            new_active = np.zeros(L, dtype=bool)
            for p in sorted(kept):
                ch = sorted(kept[p])
                for j, (bit, m) in enumerate(ch):
                    slot = p if j == 0 else free.pop(0)
                    new_alpha[slot] = alpha[p][:]
                    new_beta[slot] = beta[p][:]
                    new_uh[slot] = uh[p]
                    new_uh[slot, i] = bit
                    new_pm[slot] = m
                    new_active[slot] = True
            alpha, beta, uh, pm, active = new_alpha, new_beta, new_uh, new_pm, new_active
        # partial sums upward
        for p in np.flatnonzero(active):
            x = np.array([uh[p, i]], np.uint8)
            s = 0
            idx = i
            while idx & 1:
                x = np.concatenate([beta[p][s] ^ x, x])
                s += 1
                idx >>= 1
            if s < n:
                beta[p][s] = x
    order = sorted(np.flatnonzero(active), key=lambda p: (pm[p], p))
    choice = order[0]
    if r:
        info = np.flatnonzero(mask)
        for p in order:
            if crc_ok(uh[p, info][None, :], poly, r)[0]:
                choice = p
                break
    return uh[choice], pm.copy(), uh.copy()


def data_bits(u_hat: np.ndarray, mask: np.ndarray, r: int = 0) -> np.ndarray:
    info = np.flatnonzero(mask)
    bits = np.asarray(u_hat)[..., info]
    return bits[..., : bits.shape[-1] - r]
