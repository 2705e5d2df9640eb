"""Seeded quasi-cyclic base matrices and the ``.qc`` fixture format.

A base matrix has ``mb`` rows, ``nb`` columns and ``kb = nb - mb`` systematic
(information) columns.  Entry ``-1`` is an all-zero Z x Z block; entry
``s`` in ``[0, Z)`` is the identity shifted right by ``s``: check ``(i, r)``
joins variable node ``(j, (r + s) mod Z)``.

Two families are drawn (the paper lists 5G LDPC codes among its FEC
components, Sec. "Features"; the shapes below are synthetic stand-ins, since
the 3GPP base-graph tables are not used):

* ``11n``: an 802.11n-style rate-1/2 layout.  The parity part is
  dual-diagonal: parity column ``kb`` has entries at row 0 (shift 1), row
  ``mb // 2`` (shift 0) and row ``mb - 1`` (shift 1); parity column
  ``kb + j`` (``j >= 1``) has shift-0 entries at rows ``j - 1`` and ``j``.
  Information entries are present with probability ``p_info``.
* ``bg``: a 5G-NR-base-graph-shaped layout.  Rows 0..3 form a core whose
  parity columns ``kb..kb+3`` use the same dual-diagonal pattern with
  ``m = 4``; core-row information entries are present with probability
  ``p_core``.  Extension row ``r >= 4`` has a shift-0 identity at column
  ``kb + r`` and entries in columns ``< kb + 4`` present with probability
  ``p_ext``.

Draws use ``numpy.random.Generator(PCG64(seed))`` in row-major order, a
presence draw then (if present) a shift draw per eligible entry.  An
information column with fewer than two entries among the decoded rows would
leave a variable node without extrinsic information, and an extension row
holding only its own identity would be a degree-1 check; such columns (same
per-row probabilities, rows in order) and rows (columns in order) are redrawn
until neither is left, and the number of redraws is written into the
fixture header.
"""
from __future__ import annotations

import os
from dataclasses import dataclass, field

import numpy as np

FIXTURE_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fixtures")


@dataclass
class QCBase:
    """A base matrix plus its metadata.

    ``base`` is an ``int16`` array of shape ``(mb, nb)``.  ``family`` is
    ``"11n"`` or ``"bg"``.  ``n_punct_cols`` counts leading information
    columns that are never transmitted (2 for the ``bg`` family, 0 for
    ``11n``)."""

    base: np.ndarray
    Z: int
    kb: int
    family: str
    n_punct_cols: int
    meta: dict = field(default_factory=dict)

    @property
    def mb(self) -> int:
        return int(self.base.shape[0])

    @property
    def nb(self) -> int:
        return int(self.base.shape[1])

    @property
    def k(self) -> int:
        return self.kb * self.Z

    @property
    def n_mother(self) -> int:
        return self.nb * self.Z


def _eligible_columns(family: str, i: int, kb: int) -> list[int]:
    if family == "11n":
        return list(range(kb))
    if i < 4:
        return list(range(kb))
    return list(range(kb + 4))


def _row_prob(family: str, i: int, p: dict) -> float:
    if family == "11n":
        return p["p_info"]
    return p["p_core"] if i < 4 else p["p_ext"]


def _set_parity(H: np.ndarray, family: str, kb: int) -> None:
    mb = H.shape[0]
    m = mb if family == "11n" else 4
    mid = m // 2
    H[0, kb] = 1
    H[mid, kb] = 0
    H[m - 1, kb] = 1
    for j in range(1, m):
        H[j - 1, kb + j] = 0
        H[j, kb + j] = 0
    if family == "bg":
        for r in range(4, mb):
            H[r, kb + r] = 0


def draw_base(family: str, mb: int, nb: int, Z: int, seed: int, *,
              decoded_rows: int | None = None, p_info: float = 0.3,
              p_core: float = 0.9, p_ext: float = 0.21) -> QCBase:
    """Draw a base matrix of the given family from ``seed``."""
    if family not in ("11n", "bg"):
        raise ValueError(family)
    kb = nb - mb
    if family == "bg" and mb < 4:
        raise ValueError("bg family needs at least the 4 core rows")
    decoded_rows = mb if decoded_rows is None else decoded_rows
    probs = {"p_info": p_info, "p_core": p_core, "p_ext": p_ext}
    rng = np.random.Generator(np.random.PCG64(seed))
    H = -np.ones((mb, nb), dtype=np.int16)
    for i in range(mb):
        p = _row_prob(family, i, probs)
        for j in _eligible_columns(family, i, kb):
            if rng.random() < p:
                H[i, j] = rng.integers(0, Z)
    _set_parity(H, family, kb)
    redraws = 0
    changed = True
    while changed:
        changed = False
        if family == "bg":
            for i in range(4, decoded_rows):
                while int((H[i, :kb + 4] >= 0).sum()) < 1:
                    redraws += 1
                    changed = True
                    for j in _eligible_columns(family, i, kb):
                        if rng.random() < _row_prob(family, i, probs):
                            H[i, j] = rng.integers(0, Z)
        for j in range(kb):
            while int((H[:decoded_rows, j] >= 0).sum()) < 2:
                redraws += 1
                changed = True
                for i in range(mb):
                    if j not in _eligible_columns(family, i, kb):
                        continue
                    H[i, j] = -1
                    if rng.random() < _row_prob(family, i, probs):
                        H[i, j] = rng.integers(0, Z)
    meta = {"seed": seed, "redraws": redraws, "decoded_rows": decoded_rows}
    meta.update({k: v for k, v in probs.items()
                 if (family == "11n") == (k == "p_info")})
    return QCBase(base=H, Z=Z, kb=kb, family=family,
                  n_punct_cols=0 if family == "11n" else 2, meta=meta)


def write_qc(path: str, qb: QCBase) -> None:
    with open(path, "w") as f:
        f.write(f"# family={qb.family} n_punct_cols={qb.n_punct_cols}")
        for k, v in sorted(qb.meta.items()):
            f.write(f" {k}={v}")
        f.write("\n")
        f.write(f"{qb.mb} {qb.nb} {qb.kb} {qb.Z}\n")
        for row in qb.base:
            f.write(" ".join(str(int(x)) for x in row) + "\n")


def read_qc(path: str) -> QCBase:
    meta: dict = {}
    family, npunct = "bg", 2
    rows = []
    header = None
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line:
                continue
            if line.startswith("#"):
                for tok in line[1:].split():
                    k, _, v = tok.partition("=")
                    if k == "family":
                        family = v
                    elif k == "n_punct_cols":
                        npunct = int(v)
                    else:
                        try:
                            meta[k] = int(v)
                        except ValueError:
                            try:
                                meta[k] = float(v)
                            except ValueError:
                                meta[k] = v
                continue
            vals = [int(t) for t in line.split()]
            if header is None:
                header = vals
            else:
                rows.append(vals)
    mb, nb, kb, Z = header
    base = np.array(rows, dtype=np.int16)
    if base.shape != (mb, nb):
        raise ValueError(f"{path}: expected {mb}x{nb} entries, got {base.shape}")
    return QCBase(base=base, Z=Z, kb=kb, family=family, n_punct_cols=npunct, meta=meta)


def fixture_path(name: str) -> str:
    return os.path.join(FIXTURE_DIR, name + ".qc")


def load_fixture(name: str) -> QCBase:
    return read_qc(fixture_path(name))
