"""Workload descriptions: code shape, transmitted length, modulation,
Eb/N0 points, batch sizes and seeds.

Nothing here computes any part of the link; it only names the synthetic
inputs.  The five workloads are

* ``small``: 11n-style rate-1/2 code, 12x24 base, Z=27 (n=648, k=324), BPSK,
  Eb/N0 in {1, 2, 3} dB, 1000 codewords per point, flooding sum-product.
* ``bg2``: BG2-shaped 42x52 base, Z=128, k=1280 (the first 2Z information
  bits punctured), 3840 transmitted bits (rate 1/3), Gray 16-QAM, max-log
  demapper, Eb/N0 0:0.5:4 dB, batch 4096, FP32 flooding sum-product and
  int8 offset min-sum (offset 1, saturation 31).
* ``bg1``: BG1-shaped 46x68 base, Z=384 (n=26112, k=8448), rate 1/3, Gray
  64-QAM, Eb/N0 1:0.5:5 dB, batch 1024, layered normalized min-sum (0.75).
* ``mixed``: eight BG2/BG1-shaped codes with Z in {16,...,384}, rates 1/3 to
  8/9 by column-order rate matching, per-codeword modulation and Eb/N0.
* ``wbp``: the ``bg2`` code, weighted BP with 10 iterations, a neural
  demapper on 16-QAM, batch 2048, Eb/N0 uniform in [1, 4] dB.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .qc_base import QCBase, draw_base, load_fixture

DATA_SEED_BASE = 0x2203118500000000


def data_seed(config_index: int, point: int) -> int:
    """Philox key for workload ``config_index`` (1-based) at point ``point``."""
    return DATA_SEED_BASE + 256 * config_index + point


@dataclass(frozen=True)
class CodeSpec:
    name: str          # fixture name
    family: str
    mb: int
    nb: int
    Z: int
    seed: int
    decoded_rows: int
    p_info: float = 0.3
    p_core: float = 0.9
    p_ext: float = 0.21

    def draw(self) -> QCBase:
        return draw_base(self.family, self.mb, self.nb, self.Z, self.seed,
                         decoded_rows=self.decoded_rows, p_info=self.p_info,
                         p_core=self.p_core, p_ext=self.p_ext)

    def load(self) -> QCBase:
        return load_fixture(self.name)


def e_tx_for_rate(k: int, rate_num: int, rate_den: int) -> int:
    """Transmitted bits for information length ``k`` at rate num/den:
    ceil(k / R) rounded up to a multiple of 4 (so QPSK and 16-QAM fit)."""
    e = -(-k * rate_den // rate_num)
    return -(-e // 4) * 4


def decoded_rows_for(family: str, mb: int, kb: int, Z: int, n_punct_cols: int, e_tx: int) -> int:
    """Core rows plus every extension row whose own parity column carries at
    least one transmitted bit."""
    if family == "11n":
        return mb
    last = n_punct_cols * Z + e_tx           # one past the last transmitted VN
    rows = 4
    for r in range(4, mb):
        if (kb + r) * Z < last:
            rows = r + 1
    return rows


SMALL = CodeSpec("small_11n_z27", "11n", 12, 24, 27, seed=1, decoded_rows=12)
BG2 = CodeSpec("bg2_z128", "bg", 42, 52, 128, seed=2, decoded_rows=22, p_ext=0.21)
BG1 = CodeSpec("bg1_z384", "bg", 46, 68, 384, seed=3, decoded_rows=46, p_ext=0.17)

# (Z, base graph, rate numerator, rate denominator)
MIXED_SHAPES = [
    (16, "bg2", 1, 3), (32, "bg2", 2, 5), (64, "bg2", 1, 2), (96, "bg2", 2, 3),
    (128, "bg1", 1, 3), (192, "bg1", 1, 2), (256, "bg1", 3, 4), (384, "bg1", 8, 9),
]


def mixed_specs() -> list[tuple[CodeSpec, int]]:
    """The eight mixed-batch code shapes (fixture seeds 100..107) and their
    transmitted lengths."""
    out = []
    for idx, (Z, bg, rn, rd) in enumerate(MIXED_SHAPES):
        if bg == "bg2":
            mb, nb, pe = 42, 52, 0.21
        else:
            mb, nb, pe = 46, 68, 0.17
        kb = nb - mb
        e_tx = e_tx_for_rate(kb * Z, rn, rd)
        rows = decoded_rows_for("bg", mb, kb, Z, 2, e_tx)
        spec = CodeSpec(f"mixed{idx}_{bg}_z{Z}", "bg", mb, nb, Z, seed=100 + idx,
                        decoded_rows=rows, p_ext=pe)
        out.append((spec, e_tx))
    return out


def mixed_counts(seed: int = 0x5EED4) -> list[int]:
    """Codewords per mixed shape: round(exp(U[ln 16, ln 4096]))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random(len(MIXED_SHAPES))
    return [int(round(math.exp(math.log(16) + x * (math.log(4096) - math.log(16))))) for x in u]


@dataclass(frozen=True)
class Workload:
    index: int
    name: str
    code: CodeSpec
    e_tx: int
    bits_per_sym: int
    demap: str            # "exact" | "maxlog" | "neural"
    ebn0_db: tuple
    batch: int
    iters: int


SMALL_WL = Workload(1, "small", SMALL, 648, 1, "exact", (1.0, 2.0, 3.0), 1000, 20)
BG2_WL = Workload(2, "bg2", BG2, 3840, 4, "maxlog",
                  tuple(0.5 * i for i in range(9)), 4096, 20)
BG1_WL = Workload(3, "bg1", BG1, 25344, 6, "maxlog",
                  tuple(1.0 + 0.5 * i for i in range(9)), 1024, 20)
WBP_WL = Workload(5, "wbp", BG2, 3840, 4, "neural",
                  tuple(0.5 * i for i in range(9)), 2048, 10)

ALL_CODES = [SMALL, BG2, BG1] + [s for s, _ in mixed_specs()]
