"""The committed .qc fixtures equal a fresh draw from their seeds."""
import numpy as np

from inputs import qc_base
from inputs.workloads import ALL_CODES, decoded_rows_for, e_tx_for_rate, mixed_counts, mixed_specs


def test_fixtures_match_seeds():
    for spec in ALL_CODES:
        fresh = spec.draw()
        stored = spec.load()
        assert np.array_equal(fresh.base, stored.base), spec.name
        assert stored.Z == spec.Z and stored.kb == spec.nb - spec.mb


def test_roundtrip(tmp_path):
    qb = ALL_CODES[1].draw()
    p = tmp_path / "x.qc"
    qc_base.write_qc(str(p), qb)
    back = qc_base.read_qc(str(p))
    assert np.array_equal(back.base, qb.base) and back.family == qb.family


def test_structure():
    for spec in ALL_CODES:
        qb = spec.load()
        H = qb.base[:spec.decoded_rows]
        assert ((H[:, :qb.kb] >= 0).sum(0) >= 2).all()
        assert ((H >= 0).sum(1) >= 2).all()
        assert (qb.base < qb.Z).all() and (qb.base >= -1).all()


def test_mixed_shapes():
    specs = mixed_specs()
    assert len(specs) == 8
    for spec, e_tx in specs:
        assert e_tx % 4 == 0
        kb = spec.nb - spec.mb
        assert decoded_rows_for("bg", spec.mb, kb, spec.Z, 2, e_tx) == spec.decoded_rows
    c = mixed_counts()
    assert all(16 <= x <= 4096 for x in c)
    assert e_tx_for_rate(8448, 8, 9) == 9504
