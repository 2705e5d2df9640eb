"""Shared test helpers: codes, devices, seeded link inputs from the oracle."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from inputs.workloads import BG1, BG2, SMALL  # noqa: E402
from oracle import modem, pipeline, qc  # noqa: E402

CODES = {"small": (SMALL, 648, 1), "bg2": (BG2, 3840, 4), "bg1": (BG1, 25344, 6)}


def graph(name, full=False):
    spec, e_tx, _ = CODES[name]
    qb = spec.load()
    return qb, qc.graph_from_qcbase(qb, e_tx, full=full)


def oracle_llrs(name, B, ebn0_db, seed, cw0=0, demap="maxlog"):
    """Boundary LLRs float64[B][e_tx] from the oracle's link at one Eb/N0."""
    spec, e_tx, m = CODES[name]
    qb, g = graph(name)
    n0 = float(pipeline.n0_for(g, ebn0_db, m))
    tx = pipeline.transmit(g, qb.family, seed, cw0, B, np.full(B, n0), m,
                           "exact" if m == 1 else demap)
    return tx


def rel_close(a, b, rtol):
    """|a - b| <= rtol * max(1, |b|) elementwise; returns (ok, worst ratio)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    err = np.abs(a - b) / np.maximum(1.0, np.abs(b))
    worst = float(err.max()) if err.size else 0.0
    return worst <= rtol, worst
