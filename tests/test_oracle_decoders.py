"""Pins of the oracle decoders.

* Tree codes: flooding sum-product equals brute-force bitwise MAP.
* Single parity check: one check pass is exact MAP.
* Degree-2 checks pass the other input through (minus the offset for OMS).
* phi form equals the tanh form; both equal a per-edge Python loop.
* Offset min-sum with offset 0 and no saturation equals a per-check loop.
* Codeword symmetry: flipping the LLR signs on a codeword's ones flips
  every posterior the same way.
* Pruned and full graphs give identical posteriors.
* Layered min-sum equals a check-by-check Python loop and, on a single row,
  one flooding min-sum round.
* Noiseless codewords are fixed points and decode with zero syndrome.
"""
import itertools
import math

import numpy as np
import pytest

from inputs import rand
from inputs.workloads import BG2, SMALL
from oracle import decoders as D
from oracle import philox, qc


def tiny_graph(base, Z):
    base = np.array(base)
    mb, nb = base.shape
    return qc.make_graph(base, nb - mb, Z, 0, nb * Z, family="11n")


def codewords(g):
    H = qc.dense_H(g.base, g.Z).astype(np.int64)
    n = H.shape[1]
    allv = np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int64)
    return allv[~((allv @ H.T) % 2).any(axis=1)]


def map_llr(g, L):
    """Bitwise MAP LLRs (boundary convention) by enumerating the code."""
    C = codewords(g).astype(np.float64)
    out = np.empty_like(L)
    for b in range(L.shape[0]):
        s = C @ L[b]
        for i in range(C.shape[1]):
            one = C[:, i] == 1
            out[b, i] = np.logaddexp.reduce(s[one]) - np.logaddexp.reduce(s[~one])
    return out


@pytest.mark.parametrize("base,Z", [([[0, 0, -1], [-1, 0, 0]], 1),
                                    ([[3, 1, -1], [-1, 4, 2]], 5),
                                    ([[0, 0, 0, -1, -1], [-1, -1, 0, 0, 0]], 2)])
def test_tree_bp_equals_map(base, Z):
    g = tiny_graph(base, Z)
    L = rand.gaussian(1, (6, g.n_dec), scale=1.5)
    app = D.spa_flood(g, -L, iters=6)
    assert np.allclose(-app, map_llr(g, L), rtol=1e-10, atol=1e-10)


def test_spc_one_pass_is_map():
    g = tiny_graph([[0, 0, 0, 0, 0]], 1)
    L = rand.gaussian(2, (8, 5), scale=2.0)
    app = D.spa_flood(g, -L, iters=1)
    assert np.allclose(-app, map_llr(g, L), rtol=1e-10, atol=1e-10)


def test_degree2_passthrough():
    q = rand.gaussian(3, (4, 2, 7), scale=5.0)
    r = D.cn_spa_phi(q)
    assert np.allclose(r[:, 0], q[:, 1], rtol=1e-9, atol=1e-9)
    assert np.allclose(r[:, 1], q[:, 0], rtol=1e-9, atol=1e-9)
    qi = rand.int8_uniform(4, (4, 2, 7), -31, 31).astype(np.int64)
    ro = D.cn_oms(qi, offset=1)
    exp0 = np.sign(np.where(qi[:, 1] < 0, -1, 1)) * np.maximum(np.abs(qi[:, 1]) - 1, 0)
    assert np.array_equal(ro[:, 0], exp0)


def test_phi_tanh_and_loop_agree():
    q = rand.gaussian(5, (3, 6, 4), scale=3.0)
    a = D.cn_spa_phi(q)
    b = D.cn_spa_tanh(q)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-10)
    # per-edge loop in the tanh form
    for bb in range(3):
        for z in range(4):
            for v in range(6):
                p = 1.0
                for u in range(6):
                    if u != v:
                        p *= math.tanh(q[bb, u, z] / 2)
                assert abs(a[bb, v, z] - 2 * math.atanh(p)) < 1e-10


def test_phi_special_values():
    assert D.phi(np.array([0.0]))[0] == np.inf
    assert D.phi(np.array([np.inf]))[0] == 0.0
    x = np.array([0.1, 1.0, 5.0, 20.0])
    assert np.allclose(D.phi(D.phi(x)), x, rtol=1e-12)
    assert np.allclose(D.phi(x), -np.log(np.tanh(x / 2)), rtol=1e-12)


def test_oms_offset0_equals_minsum_loop():
    q = rand.int8_uniform(6, (5, 7, 3), -40, 40).astype(np.int64)
    r = D.cn_oms(q, offset=0)
    for b in range(5):
        for z in range(3):
            for v in range(7):
                others = [q[b, u, z] for u in range(7) if u != v]
                s = 1
                for x in others:
                    s *= -1 if x < 0 else 1
                assert r[b, v, z] == s * min(abs(x) for x in others)


def _flood_loop_spa(g, lam, iters):
    """Per-edge Python loop, tanh rule, for a tiny graph."""
    ev, ec = g.edge_vn(), g.edge_check()
    B = lam.shape[0]
    q = np.clip(lam[:, ev], -20, 20)
    app = lam.copy()
    for _ in range(iters):
        r = np.zeros_like(q)
        for b in range(B):
            for e in range(g.E):
                p = 1.0
                for f in range(g.E):
                    if f != e and ec[f] == ec[e]:
                        p *= math.tanh(q[b, f] / 2)
                r[b, e] = min(max(2 * math.atanh(p), -20), 20)
        app = lam.copy()
        for e in range(g.E):
            app[:, ev[e]] += r[:, e]
        q = np.clip(app[:, ev] - r, -20, 20)
    return app


def test_spa_flood_equals_loop_on_cyclic_code():
    g = tiny_graph([[0, 1, 2, 0, -1], [2, -1, 1, 0, 0], [1, 0, -1, -1, 0]], 3)
    lam = rand.gaussian(7, (2, g.n_dec), scale=1.2, mean=0.3)
    assert np.allclose(D.spa_flood(g, lam, 4), _flood_loop_spa(g, lam, 4), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("algo", ["spa", "oms"])
def test_codeword_symmetry(algo):
    qb = SMALL.load()
    g = qc.graph_from_qcbase(qb, 648)
    u = philox.source_bits(8, 0, 3, g.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)[:, :g.n_dec].astype(np.int64)
    sgn = 1 - 2 * c
    if algo == "spa":
        lam = rand.gaussian(9, (3, g.n_dec), scale=2.0, mean=0.5)
        a0 = D.spa_flood(g, lam, 7)
        a1 = D.spa_flood(g, lam * sgn, 7)
        assert np.allclose(a1, a0 * sgn, rtol=1e-12, atol=1e-12)
    else:
        lam = rand.int8_uniform(9, (3, g.n_dec), -12, 20).astype(np.int64)
        a0 = D.oms_flood(g, lam, 7)
        a1 = D.oms_flood(g, lam * sgn, 7)
        assert np.array_equal(a1, a0 * sgn)


@pytest.mark.parametrize("algo", ["spa", "oms"])
def test_pruned_equals_full(algo):
    qb = BG2.load()
    gp = qc.graph_from_qcbase(qb, 3840)
    gf = qc.graph_from_qcbase(qb, 3840, full=True)
    assert gf.rows == 42 and gp.rows == 22
    L = rand.gaussian(10, (3, 3840), scale=2.0, mean=-1.0)
    if algo == "spa":
        ap = D.spa_flood(gp, D.channel_lam(gp, L), 6)
        af = D.spa_flood(gf, D.channel_lam(gf, L), 6)
        assert np.array_equal(ap, af[:, :gp.n_dec])
    else:
        Lq = np.clip(np.rint(2 * L), -31, 31)
        ap = D.oms_flood(gp, D.channel_lam(gp, Lq, np.int64), 6)
        af = D.oms_flood(gf, D.channel_lam(gf, Lq, np.int64), 6)
        assert np.array_equal(ap, af[:, :gp.n_dec])


def _layered_loop(g, lam, iters, alpha, order=None):
    """Layered min-sum one check at a time, written from the message
    definitions: the message from variable node v to check x is v's channel
    value plus the messages of every other check of v; a check's outputs all
    use the messages it received before its own update."""
    ev = g.edge_vn()
    B = lam.shape[0]
    r = np.zeros((B, g.E))
    Z = g.Z
    edges_of = {}
    for x, v in enumerate(ev):
        edges_of.setdefault(int(v), []).append(x)
    for _ in range(iters):
        for i in (range(g.rows) if order is None else order):
            es = g.row_entries(i)
            for z in range(Z):
                ids = [e * Z + z for e in es]
                for b in range(B):
                    t = [lam[b, ev[x]] + sum(r[b, y] for y in edges_of[int(ev[x])] if y != x)
                         for x in ids]
                    new = []
                    for a in range(len(ids)):
                        others = [t[u] for u in range(len(ids)) if u != a]
                        s = 1.0
                        for y in others:
                            s *= -1.0 if y < 0 else 1.0
                        new.append(s * alpha * min(abs(y) for y in others))
                    for a, x in enumerate(ids):
                        r[b, x] = new[a]
    app = lam.astype(np.float64).copy()
    for x, v in enumerate(ev):
        app[:, v] += r[:, x]
    return app


# the second graph has two columns of degree one (one closing its row, one
# inside a row), the first none
LAYERED_GRAPHS = [([[0, 1, 2, 0, -1], [2, -1, 1, 0, 0], [1, 0, -1, -1, 0]], 3),
                  ([[0, 1, -1, 2, 0, -1], [2, -1, 1, 0, 1, -1], [1, 0, -1, 2, -1, 0]], 3)]


@pytest.mark.parametrize("gi", [0, 1])
def test_layered_equals_check_loop(gi):
    g = tiny_graph(*LAYERED_GRAPHS[gi])
    lam = rand.gaussian(11, (3, g.n_dec), scale=1.5, mean=0.4)
    got = D.nms_layered(g, lam, 3, alpha=0.75)
    assert np.allclose(got, _layered_loop(g, lam, 3, 0.75), rtol=1e-12, atol=1e-12)


def test_layered_order_is_the_visiting_order():
    """Another row order follows the check-by-check loop in that order and
    differs from the natural order's result; the natural order given
    explicitly is the default."""
    g = tiny_graph(*LAYERED_GRAPHS[1])
    lam = rand.gaussian(16, (3, g.n_dec), scale=1.5, mean=0.4)
    order = [2, 0, 1]
    got = D.nms_layered(g, lam, 3, alpha=0.75, order=order)
    assert np.allclose(got, _layered_loop(g, lam, 3, 0.75, order), rtol=1e-12, atol=1e-12)
    nat = D.nms_layered(g, lam, 3, alpha=0.75)
    assert not np.allclose(got, nat)
    assert np.array_equal(nat, D.nms_layered(g, lam, 3, alpha=0.75, order=[0, 1, 2]))
    with pytest.raises(ValueError):
        D.nms_layered(g, lam, 1, order=[0, 0, 1])


def test_grouped_order_on_a_five_cycle():
    """Rows i and i+1 (mod 5) share column i+1: the conflict graph is a
    five-cycle, which DSatur colours 0, 1, 0, 1, 2 for rows 0..4 (row 0
    first, then the saturated rows in index order), so the groups are
    {0, 2}, {1, 3}, {4}.  Each row also has a column of its own."""
    base = -np.ones((5, 10), dtype=int)
    for i in range(5):
        base[i, i] = 0
        base[i, (i - 1) % 5] = 0
        base[i, 5 + i] = 0
    g = tiny_graph(base, 3)
    assert D.grouped_order(g) == [0, 2, 1, 3, 4]


@pytest.mark.parametrize("name", ["bg2", "bg1", "small"])
def test_grouped_order_is_a_proper_colouring(name):
    """On the workload codes: a permutation of the rows whose consecutive
    groups (maximal runs of rows with no common column) never put two rows
    with a common column together, and with fewer groups than rows."""
    from inputs.workloads import BG1
    spec, e_tx = {"bg2": (BG2, 3840), "bg1": (BG1, 25344), "small": (SMALL, 648)}[name]
    g = qc.graph_from_qcbase(spec.load(), e_tx)
    order = D.grouped_order(g)
    assert sorted(order) == list(range(g.rows))
    cols = [set(g.entries[g.row_entries(i), 1].tolist()) for i in order]
    groups, cur = 0, set()
    for c in cols:
        if c & cur:
            groups, cur = groups + 1, set()
        cur |= c
    assert groups + 1 < g.rows


def test_layered_degree_one_message_is_the_channel_value():
    """fp32 mode: a degree-one variable node's posterior is, after every
    iteration, its channel value plus its one check message, rounded once."""
    g = tiny_graph(*LAYERED_GRAPHS[1])
    deg = np.bincount(g.entries[:, 1], minlength=g.cols)
    lam = rand.gaussian(15, (4, g.n_dec), scale=3.0, mean=0.3, dtype=np.float32)
    _, hist = D.nms_layered(g, lam, 6, alpha=0.75, mode="fp32", trace=True)
    ev = g.edge_vn()
    one = [x for x in range(g.E) if deg[ev[x] // g.Z] == 1]
    assert len(one) == 2 * g.Z
    for r, app in hist:
        for x in one:
            assert np.array_equal(app[:, ev[x]], lam[:, ev[x]] + r[:, x])


def test_layered_single_row_is_one_flood_round():
    g = tiny_graph([[0, 2, 1, 3, 0, 4]], 5)
    lam = rand.gaussian(12, (4, g.n_dec), scale=2.0)
    got = D.nms_layered(g, lam, 1, alpha=1.0)
    # one flooding min-sum round with no offset, written with the OMS update
    # on an exact scaling: multiply by 2^20 and round to integers
    q = lam[:, g.edge_vn()]
    ids = g.row_edge_ids(0)
    scale = 2.0 ** 20
    qi = np.rint(q[:, ids] * scale).astype(np.int64)
    rm = D.cn_oms(qi, offset=0) / scale
    exp = lam.copy()
    for a, e in enumerate(g.row_entries(0)):
        for z in range(g.Z):
            exp[:, g.edge_vn()[e * g.Z + z]] += rm[:, a, z]
    assert np.allclose(got, exp, atol=1e-5)


def test_layered_fp32_mode_is_float32_arithmetic():
    g = tiny_graph([[0, 1, 2, 0, -1], [2, -1, 1, 0, 0], [1, 0, -1, -1, 0]], 3)
    lam = rand.gaussian(13, (2, g.n_dec), scale=1.5, dtype=np.float32)
    got = D.nms_layered(g, lam, 3, alpha=0.75, mode="fp32")
    assert got.dtype == np.float32
    ref = D.nms_layered(g, lam.astype(np.float64), 3, alpha=0.75, mode="fp64")
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("algo", ["spa", "oms", "nms"])
def test_noiseless_codewords_decode(algo):
    qb = BG2.load()
    g = qc.graph_from_qcbase(qb, 3840)
    u = philox.source_bits(14, 0, 2, g.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    t = c[:, g.tx_lo:g.tx_lo + g.e_tx].astype(np.int64)
    L = 8.0 * (2 * t - 1)
    if algo == "spa":
        app = D.spa_flood(g, D.channel_lam(g, L), 20)
    elif algo == "oms":
        app = D.oms_flood(g, D.channel_lam(g, np.clip(2 * L, -31, 31), np.int64), 20)
    else:
        app = D.nms_layered(g, D.channel_lam(g, L), 20)
    hard = (app < 0).astype(np.uint8)
    assert np.array_equal(hard, c[:, :g.n_dec])
    assert np.array_equal(D.hard_bits(app, g.k), u)
    sub = qc.syndrome(qb.base[:g.rows, :g.cols], qb.Z, hard)
    assert not sub.any()


def test_oms_saturated_inputs():
    qb = SMALL.load()
    g = qc.graph_from_qcbase(qb, 648)
    u = philox.source_bits(15, 0, 2, g.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u).astype(np.int64)
    lam = 31 * (1 - 2 * c)
    app, rs, qs = D.oms_flood(g, lam, 3, trace=True)
    assert (np.abs(rs[-1]) == 30).all()
    assert (np.abs(qs[-1]) == 31).all()
    assert np.array_equal((app < 0).astype(np.int64), c)
