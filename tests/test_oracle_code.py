"""Pins of the code construction and the back-substitution encoder: full
GF(2) rank, H c = 0 for every codeword, systematic form, linearity, and on
tiny lifts the encodings fill exactly the null space of H (brute force)."""
import itertools

import numpy as np
import pytest

from inputs import qc_base, rand
from inputs.workloads import ALL_CODES, BG1, BG2, SMALL
from oracle import philox, qc


def test_rank_small_full():
    qb = SMALL.load()
    H = qc.dense_H(qb.base, qb.Z)
    assert qc.gf2_rank(H) == qb.mb * qb.Z


@pytest.mark.parametrize("fam,mb,nb,pe", [("bg", 42, 52, 0.21), ("bg", 46, 68, 0.17)])
def test_rank_bg_shaped_z16(fam, mb, nb, pe):
    qb = qc_base.draw_base(fam, mb, nb, 16, seed=5, p_ext=pe)
    assert qc.gf2_rank(qc.dense_H(qb.base, 16)) == mb * 16


def test_gf2_rank_known():
    # rank of a known singular matrix and of the identity
    A = np.array([[1, 1, 0], [0, 1, 1], [1, 0, 1]], dtype=np.uint8)
    assert qc.gf2_rank(A) == 2
    assert qc.gf2_rank(np.eye(9, dtype=np.uint8)) == 9


@pytest.mark.parametrize("spec", ALL_CODES, ids=lambda s: s.name)
def test_encode_syndrome_zero(spec):
    qb = spec.load()
    u = philox.source_bits(17, 0, 8, qb.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    assert c.shape == (8, qb.n_mother)
    assert np.array_equal(c[:, :qb.k], u)
    assert not qc.syndrome(qb.base, qb.Z, c).any()
    # the sparse syndrome agrees with the dense H product
    if qb.n_mother <= 7000:
        H = qc.dense_H(qb.base, qb.Z).astype(np.int64)
        assert not ((H @ c[:2].T.astype(np.int64)) % 2).any()


def test_encoder_linear():
    qb = BG2.load()
    u1 = philox.source_bits(1, 0, 4, qb.k)
    u2 = philox.source_bits(2, 0, 4, qb.k)
    enc = lambda u: qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    assert np.array_equal(enc(u1) ^ enc(u2), enc(u1 ^ u2))


@pytest.mark.parametrize("fam,mb,nb,Z", [("11n", 4, 6, 2), ("11n", 3, 5, 3), ("bg", 5, 7, 2)])
def test_tiny_nullspace_bruteforce(fam, mb, nb, Z):
    qb = qc_base.draw_base(fam, mb, nb, Z, seed=3, p_info=0.6, p_ext=0.5)
    H = qc.dense_H(qb.base, Z).astype(np.int64)
    n = nb * Z
    k = qb.k
    null = {v for v in itertools.product((0, 1), repeat=n) if not ((H @ np.array(v)) % 2).any()}
    us = np.array(list(itertools.product((0, 1), repeat=k)), dtype=np.uint8)
    cw = {tuple(int(x) for x in row) for row in qc.encode(qb.base, qb.kb, Z, fam, us)}
    assert cw == null
    assert len(null) == 2 ** k


def test_decoded_graph_shapes():
    g2 = qc.graph_from_qcbase(BG2.load(), 3840)
    assert (g2.rows, g2.cols, g2.n_dec, g2.k) == (22, 32, 4096, 1280)
    g1 = qc.graph_from_qcbase(BG1.load(), 25344)
    assert (g1.rows, g1.cols, g1.n_dec, g1.m_dec) == (46, 68, 26112, 17664)
    gs = qc.graph_from_qcbase(SMALL.load(), 648)
    assert (gs.n_dec, gs.k, gs.m_dec) == (648, 324, 324)
    # each row block meets each VN at most once
    vn = g1.edge_vn()
    for i in range(g1.rows):
        v = vn[g1.row_edge_ids(i)].reshape(-1)
        assert len(np.unique(v)) == v.size
