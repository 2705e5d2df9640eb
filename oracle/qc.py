"""Quasi-cyclic LDPC codes: Tanner graph, encoder, syndrome, GF(2) rank.

The paper lists 5G LDPC codes with rate matching among its FEC components
and uses an LDPC encoder/decoder pair in Listing 1 (Sec. "Hello, World!").
It gives no construction; the synthetic dual-diagonal QC codes and the
back-substitution encoder below are the standard ones for that layout
(IEEE 802.11n-style parity part; the 5G base graphs have the same core).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    """Decoded Tanner graph of a QC code.

    ``rows`` x ``cols`` is the decoded part of the base matrix; ``entries``
    lists its nonzeros in row-major order as (row, col, shift).  Edge
    ``e * Z + r`` joins check ``row_e * Z + r`` and variable node
    ``col_e * Z + (r + shift_e) mod Z``."""

    base: np.ndarray          # full base matrix, int
    Z: int
    kb: int
    n_punct_cols: int
    e_tx: int
    rows: int                 # decoded base rows
    cols: int                 # decoded base columns
    entries: np.ndarray       # (nnz, 3) int64: row, col, shift

    @property
    def k(self) -> int:
        return self.kb * self.Z

    @property
    def n_dec(self) -> int:
        return self.cols * self.Z

    @property
    def m_dec(self) -> int:
        return self.rows * self.Z

    @property
    def nnz(self) -> int:
        return int(self.entries.shape[0])

    @property
    def E(self) -> int:
        return self.nnz * self.Z

    @property
    def tx_lo(self) -> int:
        return self.n_punct_cols * self.Z

    def edge_vn(self) -> np.ndarray:
        """Variable node of every edge, canonical order, ``int64[E]``."""
        Z = self.Z
        r = np.arange(Z)
        out = np.empty(self.E, dtype=np.int64)
        for e, (_, j, s) in enumerate(self.entries):
            out[e * Z:(e + 1) * Z] = j * Z + (r + s) % Z
        return out

    def edge_check(self) -> np.ndarray:
        Z = self.Z
        r = np.arange(Z)
        out = np.empty(self.E, dtype=np.int64)
        for e, (i, _, _) in enumerate(self.entries):
            out[e * Z:(e + 1) * Z] = i * Z + r
        return out

    def row_entries(self, i: int) -> np.ndarray:
        return np.nonzero(self.entries[:, 0] == i)[0]

    def row_edge_ids(self, i: int) -> np.ndarray:
        """Edge ids of base row ``i`` as a ``(d_i, Z)`` array: element
        ``[a, r]`` is the a-th edge (column order) of check ``i * Z + r``."""
        es = self.row_entries(i)
        return es[:, None] * self.Z + np.arange(self.Z)[None, :]


def decoded_shape(base: np.ndarray, kb: int, Z: int, n_punct_cols: int, e_tx: int,
                  family: str) -> tuple[int, int]:
    """Rows and columns of the base matrix that the decoder keeps.

    The 11n family keeps everything.  For the BG-shaped family the core rows
    0..3 are kept plus every extension row whose own parity column
    ``kb + r`` holds at least one transmitted bit; an extension row whose
    column is never transmitted meets an all-zero-LLR degree-1 variable node
    and sends exactly zero to every other variable node, so dropping it
    leaves every kept posterior unchanged."""
    mb, nb = base.shape
    if family == "11n":
        return mb, nb
    end = n_punct_cols * Z + e_tx
    rows = 4
    for r in range(4, mb):
        if (kb + r) * Z < end:
            rows = r + 1
    return rows, kb + rows


def make_graph(base: np.ndarray, kb: int, Z: int, n_punct_cols: int, e_tx: int,
               family: str = "bg", full: bool = False) -> Graph:
    base = np.asarray(base, dtype=np.int64)
    mb, nb = base.shape
    if full:
        rows, cols = mb, nb
    else:
        rows, cols = decoded_shape(base, kb, Z, n_punct_cols, e_tx, family)
    if n_punct_cols * Z + e_tx > nb * Z:
        raise ValueError("transmitted length exceeds the mother code")
    ent = [(i, j, int(base[i, j])) for i in range(rows) for j in range(cols) if base[i, j] >= 0]
    if any(base[i, j] >= 0 for i in range(rows) for j in range(cols, nb)):
        raise ValueError("decoded rows reach beyond the decoded columns")
    return Graph(base=base, Z=Z, kb=kb, n_punct_cols=n_punct_cols, e_tx=e_tx,
                 rows=rows, cols=cols, entries=np.array(ent, dtype=np.int64).reshape(-1, 3))


def graph_from_qcbase(qb, e_tx: int, full: bool = False) -> Graph:
    return make_graph(qb.base, qb.kb, qb.Z, qb.n_punct_cols, e_tx, qb.family, full=full)


# --------------------------------------------------------------------------
# Encoder (back-substitution through the dual-diagonal parity part)
# --------------------------------------------------------------------------

def _rot(x: np.ndarray, s: int) -> np.ndarray:
    """(P^s x)[r] = x[(r + s) mod Z] on the last axis."""
    return np.roll(x, -s, axis=-1)


def encode(base: np.ndarray, kb: int, Z: int, family: str, u: np.ndarray) -> np.ndarray:
    """Systematic encoding ``c = [u, p]`` of ``u8[B][kb*Z]`` into the mother
    code ``u8[B][nb*Z]``.

    With lambda_i the XOR over information blocks j of P^{h_ij} u_j and m
    the number of dual-diagonal rows (all rows for 11n, the 4 core rows for
    the BG shape), mid = m // 2:  p_0 is the XOR of all lambda_i (the two
    shift-1 entries of the weight-3 column cancel), p_1 = lambda_0 + P^1 p_0,
    p_{i+1} = lambda_i + p_i (+ p_0 when i = mid).  Each extension row r of
    the BG shape then fixes its own parity block as the XOR over columns
    j < kb + 4 of P^{h_rj} c_j."""
    base = np.asarray(base, dtype=np.int64)
    mb, nb = base.shape
    u = np.asarray(u, dtype=np.uint8)
    B = u.shape[0]
    c = np.zeros((B, nb, Z), dtype=np.uint8)
    c[:, :kb] = u.reshape(B, kb, Z)
    m = mb if family == "11n" else 4
    mid = m // 2
    lam = np.zeros((B, m, Z), dtype=np.uint8)
    for i in range(m):
        for j in range(kb):
            if base[i, j] >= 0:
                lam[:, i] ^= _rot(c[:, j], int(base[i, j]))
    p0 = np.bitwise_xor.reduce(lam, axis=1)
    c[:, kb] = p0
    c[:, kb + 1] = lam[:, 0] ^ _rot(p0, 1)
    for i in range(1, m - 1):
        nxt = lam[:, i] ^ c[:, kb + i]
        if i == mid:
            nxt ^= p0
        c[:, kb + i + 1] = nxt
    if family != "11n":
        for r in range(4, mb):
            acc = np.zeros((B, Z), dtype=np.uint8)
            for j in range(kb + 4):
                if base[r, j] >= 0:
                    acc ^= _rot(c[:, j], int(base[r, j]))
            c[:, kb + r] = acc
    return c.reshape(B, nb * Z)


def syndrome(base: np.ndarray, Z: int, c: np.ndarray) -> np.ndarray:
    """H c over GF(2) for every codeword; ``u8[B][mb*Z]``."""
    base = np.asarray(base, dtype=np.int64)
    mb, nb = base.shape
    B = c.shape[0]
    cb = np.asarray(c, dtype=np.uint8).reshape(B, nb, Z)
    s = np.zeros((B, mb, Z), dtype=np.uint8)
    for i in range(mb):
        for j in range(nb):
            if base[i, j] >= 0:
                s[:, i] ^= _rot(cb[:, j], int(base[i, j]))
    return s.reshape(B, mb * Z)


def dense_H(base: np.ndarray, Z: int) -> np.ndarray:
    """The expanded parity-check matrix as a dense ``u8[mb*Z][nb*Z]``."""
    base = np.asarray(base, dtype=np.int64)
    mb, nb = base.shape
    H = np.zeros((mb * Z, nb * Z), dtype=np.uint8)
    r = np.arange(Z)
    for i in range(mb):
        for j in range(nb):
            s = base[i, j]
            if s >= 0:
                H[i * Z + r, j * Z + (r + s) % Z] = 1
    return H


def gf2_rank(H: np.ndarray) -> int:
    """Rank over GF(2) by Gaussian elimination on bit-packed rows."""
    A = np.packbits(np.asarray(H, dtype=np.uint8), axis=1)
    rows, ncols = H.shape
    rank = 0
    for col in range(ncols):
        byte, bit = divmod(col, 8)
        mask = np.uint8(0x80 >> bit)
        piv = np.nonzero(A[rank:, byte] & mask)[0]
        if piv.size == 0:
            continue
        p = rank + piv[0]
        if p != rank:
            A[[rank, p]] = A[[p, rank]]
        hit = np.nonzero(A[:, byte] & mask)[0]
        hit = hit[hit != rank]
        A[hit] ^= A[rank]
        rank += 1
        if rank == rows:
            break
    return rank
