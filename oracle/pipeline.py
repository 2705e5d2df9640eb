"""The whole link of Listing 1, in the paper's order: binary source ->
LDPC encoder -> mapper -> AWGN (noise variance N0) -> demapper -> decoder
-> error count (Sec. "Hello, World!").

Transmission takes the mother-code bits ``tx_lo .. tx_lo + e_tx - 1``
(column-order rate matching: the first ``n_punct_cols`` information blocks
are punctured, the tail is not sent), maps them ``m`` at a time and sends
them with N0 = 1 / (R m 10^(EbN0/10)), R = k / e_tx.
"""
from __future__ import annotations

import time

import numpy as np

from . import decoders, modem, philox, qc, stats


def transmit(g: qc.Graph, family: str, seed: int, cw0: int, B: int, n0: np.ndarray, m: int,
             demap: str = "maxlog"):
    u = philox.source_bits(seed, cw0, B, g.k)
    c = qc.encode(g.base, g.kb, g.Z, family, u)
    t = c[:, g.tx_lo:g.tx_lo + g.e_tx]
    x = modem.map_bits(t, m)
    gn = philox.normals(seed, cw0, B, x.shape[1])
    y = modem.awgn(x, n0, gn)
    if m == 1:
        L = modem.demap_bpsk(y, n0)
    else:
        L = modem.demap_bruteforce(y, n0, m, demap)
    return {"u": u, "c": c, "x": x, "y": y, "L": L}


def n0_for(g: qc.Graph, ebn0_db, m: int):
    return modem.ebn0_to_n0(ebn0_db, g.k / g.e_tx, m)


def decode(g: qc.Graph, L: np.ndarray, algo: str, iters: int = 20):
    """Decode boundary LLRs ``L[B][e_tx]``; returns (hard info bits, APP)."""
    if algo == "spa":
        app = decoders.spa_flood(g, decoders.channel_lam(g, L), iters)
    elif algo == "oms":
        q = modem.quantize(L)
        app = decoders.oms_flood(g, decoders.channel_lam(g, q, dtype=np.int64), iters)
    elif algo == "nms":
        app = decoders.nms_layered(g, decoders.channel_lam(g, L), iters, mode="fp64")
    elif algo == "nms_grouped":
        app = decoders.nms_layered(g, decoders.channel_lam(g, L), iters, mode="fp64",
                                   order=decoders.grouped_order(g))
    elif algo == "nms32":
        lam = decoders.channel_lam(g, np.asarray(L, dtype=np.float32), dtype=np.float32)
        app = decoders.nms_layered(g, lam, iters, mode="fp32")
    else:
        raise ValueError(algo)
    return decoders.hard_bits(app, g.k), app


def run_point(g: qc.Graph, family: str, seed: int, B: int, ebn0_db: float, m: int,
              demap: str, algo: str, iters: int = 20, chunk: int = 256):
    """Error counts (bit errors, block errors, codewords) at one Eb/N0 point
    and the wall time of the whole chain."""
    n0 = float(n0_for(g, ebn0_db, m))
    tot = np.zeros(3, dtype=np.int64)
    t0 = time.perf_counter()
    for cw0 in range(0, B, chunk):
        nb = min(chunk, B - cw0)
        tx = transmit(g, family, seed, cw0, nb, np.full(nb, n0), m, demap)
        bits, _ = decode(g, tx["L"], algo, iters)
        tot += stats.count_errors(tx["u"], bits)[0]
    return tot, time.perf_counter() - t0
