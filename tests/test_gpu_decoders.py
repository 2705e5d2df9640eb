"""GPU decoder parity against the oracle.

int8 offset min-sum: bit-exact r and q after every round, posteriors, hard
decisions.  Layered normalized min-sum (FP32): bit-exact (float equality)
against the oracle's single-precision mode.  FP32 sum-product: one round
from the same state (oracle state, cast to float32) within 1e-4 relative,
and after 20 rounds on every frame the oracle decodes to a codeword.
Inputs are LLRs of the oracle's own link at a waterfall Eb/N0, so every
regime (saturated, weak, punctured) is exercised.
"""
import numpy as np
import pytest
import torch

from helpers import graph, oracle_llrs, rel_close
from oracle import decoders as D
from oracle import modem, qc

pytestmark = pytest.mark.gpu

lsim = pytest.importorskip("paper_2203_11854_amd")
dev = "cuda"


def T(x):
    """Host array -> contiguous host tensor (moved to the device by the caller)."""
    return torch.from_numpy(np.ascontiguousarray(x))


def gcode(name):
    qb, g = graph(name)
    return qb, g, lsim.Code.from_qcbase(qb, g.e_tx)


def q8_inputs(name, B, ebn0, seed):
    tx = oracle_llrs(name, B, ebn0, seed)
    return tx, modem.quantize(tx["L"].astype(np.float32))


@pytest.mark.parametrize("name,B,ebn0", [("bg2", 37, 3.0), ("small", 29, 1.5)])
def test_oms_bit_exact_every_round(name, B, ebn0):
    qb, g, code = gcode(name)
    tx, q = q8_inputs(name, B, ebn0, 41)
    lam = D.channel_lam(g, q, np.int64)
    app, rs, qs = D.oms_flood(g, lam, 20, offset=1, sat=31, trace=True)
    tq = T(q).to(dev)
    for t in (1, 2, 3, 7, 20):
        p = lsim.params(lsim.OMS_I8, iters=t, offset=1, sat=31)
        r, qq, lp = lsim.decode_state(code, tq, p)
        assert np.array_equal(r.cpu().numpy(), rs[t - 1]), t
        assert np.array_equal(qq.cpu().numpy(), qs[t - 1]), t
    p = lsim.params(lsim.OMS_I8, iters=20, offset=1, sat=31)
    bits, lpost = lsim.decode(code, tq, p, want_app=True)
    assert np.array_equal(lpost.cpu().numpy(), -app)
    assert np.array_equal(bits.cpu().numpy(), D.hard_bits(app, g.k))


@pytest.mark.parametrize("name,B,ebn0", [("bg2", 23, 3.0), ("small", 17, 1.5), ("bg1", 3, 2.5)])
def test_nms_layered_bit_exact(name, B, ebn0):
    qb, g, code = gcode(name)
    tx = oracle_llrs(name, B, ebn0, 43)
    L32 = tx["L"].astype(np.float32)
    lam = D.channel_lam(g, L32, dtype=np.float32)
    app, hist = D.nms_layered(g, lam, 20, alpha=0.75, mode="fp32", trace=True)
    tl = T(L32).to(dev)
    for t in (1, 2, 20):
        p = lsim.params(lsim.NMS_F32, iters=t, alpha=0.75)
        r, _, lp = lsim.decode_state(code, tl, p)
        assert np.array_equal(r.cpu().numpy(), hist[t - 1][0]), t
        assert np.array_equal(lp.cpu().numpy(), -hist[t - 1][1]), t
    bits, _ = lsim.decode(code, tl, lsim.params(lsim.NMS_F32, iters=20, alpha=0.75))
    assert np.array_equal(bits.cpu().numpy(), D.hard_bits(app, g.k))


@pytest.mark.parametrize("name,B,ebn0,order", [("bg2", 19, 3.0, "grouped"), ("bg1", 3, 2.5, "grouped"),
                                              ("bg2", 13, 3.0, "shuffled"), ("small", 11, 1.5, "grouped")])
def test_nms_layer_order_bit_exact(name, B, ebn0, order):
    """Other row orders (the grouped one, whose workgroup barriers fall only
    between groups of disjoint rows, and a random permutation) against the
    oracle in the same order, state after 1, 2 and 20 iterations; the
    natural order is restored bit for bit."""
    qb, g, code = gcode(name)
    nat_order, nat_barriers = code.layer_order()
    assert nat_order == list(range(g.rows)) and 1 <= nat_barriers <= g.rows
    if order == "grouped":
        code.set_layer_order("grouped")
        perm, barriers = code.layer_order()
        assert sorted(perm) == list(range(g.rows)) and barriers <= nat_barriers
    else:
        perm = np.random.default_rng(5).permutation(g.rows).tolist()
        code.set_layer_order(perm)
        assert code.layer_order()[0] == perm
    print(name, order, "barriers", nat_barriers, "->", code.layer_order()[1], flush=True)
    tx = oracle_llrs(name, B, ebn0, 59)
    L32 = tx["L"].astype(np.float32)
    lam = D.channel_lam(g, L32, dtype=np.float32)
    app, hist = D.nms_layered(g, lam, 20, alpha=0.75, mode="fp32", trace=True, order=perm)
    tl = T(L32).to(dev)
    for t in (1, 2, 20):
        r, _, lp = lsim.decode_state(code, tl, lsim.params(lsim.NMS_F32, iters=t, alpha=0.75))
        assert np.array_equal(r.cpu().numpy(), hist[t - 1][0]), t
        assert np.array_equal(lp.cpu().numpy(), -hist[t - 1][1]), t
    bits, _ = lsim.decode(code, tl, lsim.params(lsim.NMS_F32, iters=20, alpha=0.75))
    assert np.array_equal(bits.cpu().numpy(), D.hard_bits(app, g.k))
    code.set_layer_order("natural")
    assert code.layer_order() == (nat_order, nat_barriers)
    ref = D.nms_layered(g, lam, 20, alpha=0.75, mode="fp32")
    _, lp = lsim.decode(code, tl, lsim.params(lsim.NMS_F32, iters=20, alpha=0.75), want_app=True)
    assert np.array_equal(lp.cpu().numpy(), -ref)
    with pytest.raises(lsim.LsimError, match="permutation"):
        code.set_layer_order([0] * g.rows)


@pytest.mark.parametrize("name,B,ebn0", [("bg2", 21, 3.0), ("small", 17, 1.5)])
def test_spa_one_round_from_oracle_state(name, B, ebn0):
    qb, g, code = gcode(name)
    tx = oracle_llrs(name, B, ebn0, 47)
    L32 = tx["L"].astype(np.float32)
    lam = np.clip(D.channel_lam(g, L32.astype(np.float64)), -20, 20)
    _, rs, qs = D.spa_flood(g, lam, 19, trace=True)
    tl = T(L32).to(dev)
    states = [lam[:, g.edge_vn()]] + [qs[t] for t in (0, 4, 9, 18)]
    p = lsim.params(lsim.SPA_F32, iters=1, llr_max=20.0)
    worst = 0.0
    for q0 in states:
        q32 = q0.astype(np.float32)
        r_ref, app_ref, q_ref = D.spa_iteration(g, lam, q32.astype(np.float64))
        r, qq, lp = lsim.decode_state(code, tl, p, q_in=T(q32).to(dev))
        for got, ref in ((r, r_ref), (qq, q_ref), (lp, -app_ref)):
            ok, w = rel_close(got.cpu().numpy(), ref, 1e-4)
            worst = max(worst, w)
            assert ok, w
    print("worst relative error", worst)


@pytest.mark.parametrize("name,B,ebn0", [("bg2", 64, 3.5), ("small", 64, 2.0)])
def test_spa_end_to_end_on_converged_frames(name, B, ebn0):
    qb, g, code = gcode(name)
    tx = oracle_llrs(name, B, ebn0, 53)
    L32 = tx["L"].astype(np.float32)
    app = D.spa_flood(g, D.channel_lam(g, L32.astype(np.float64)), 20)
    hard = (app < 0).astype(np.uint8)
    conv = ~qc.syndrome(qb.base[:g.rows, :g.cols], qb.Z, hard).any(axis=1)
    assert conv.sum() >= B // 4
    bits, lp = lsim.decode(code, T(L32).to(dev),
                           lsim.params(lsim.SPA_F32, iters=20), want_app=True)
    bits, lp = bits.cpu().numpy(), lp.cpu().numpy()
    ok, w = rel_close(lp[conv], -app[conv], 1e-4)
    assert ok, w
    assert np.array_equal(bits[conv], D.hard_bits(app, g.k)[conv])


@pytest.mark.parametrize("algo", ["spa", "oms", "nms"])
def test_deterministic(algo):
    qb, g, code = gcode("bg2")
    tx = oracle_llrs("bg2", 40, 3.0, 59)
    if algo == "oms":
        llr = T(modem.quantize(tx["L"].astype(np.float32))).to(dev)
        p = lsim.params(lsim.OMS_I8)
    else:
        llr = T(tx["L"].astype(np.float32)).to(dev)
        p = lsim.params(lsim.SPA_F32 if algo == "spa" else lsim.NMS_F32)
    a = lsim.decode(code, llr, p, want_app=True)[1]
    b = lsim.decode(code, llr, p, want_app=True)[1]
    assert torch.equal(a, b)


def test_workgroup_size_invariance():
    qb, g, code = gcode("bg2")
    tx = oracle_llrs("bg2", 16, 3.0, 61)
    llr = T(tx["L"].astype(np.float32)).to(dev)
    q8 = T(modem.quantize(tx["L"].astype(np.float32))).to(dev)
    for algo, x in ((lsim.SPA_F32, llr), (lsim.OMS_I8, q8)):
        outs = [lsim.decode(code, x, lsim.params(algo, threads=t), want_app=True)[1]
                for t in (256, 512, 1024)]
        assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    outs = [lsim.decode(code, llr, lsim.params(lsim.NMS_F32, threads=t), want_app=True)[1]
            for t in (256, 384, 512, 1024)]
    for o in outs[1:]:
        assert torch.equal(outs[0], o)


def test_layered_large_lift_tile_invariance():
    """BG1 (Z=384): the default launch (768 threads, two codewords per
    workgroup, two workgroups per CU at the 80-VGPR budget) and launches of
    384 threads (one codeword) and 1024 threads (two codewords, 256 idle
    lanes, the compiler's register budget) give the same bits and
    posteriors, and so do the record placements: every row streamed and the
    first rows' records in LDS."""
    qb, g, code = gcode("bg1")
    tx = oracle_llrs("bg1", 3, 2.5, 67)
    llr = T(tx["L"].astype(np.float32)).to(dev)
    shapes = [(t, k) for t in (0, 384, 768, 1024) for k in (0, -1)] + [(1024, 4), (384, 3)]
    outs = []
    for t, k in shapes:
        p = lsim.params(lsim.NMS_F32, threads=t, lds_rows=k)
        print((t, k), lsim.decode_launch(code, p), flush=True)
        outs.append(lsim.decode(code, llr, p, want_app=True))
    for o in outs[1:]:
        assert torch.equal(outs[0][0], o[0]) and torch.equal(outs[0][1], o[1])


@pytest.mark.parametrize("case", ["11n_three_layers", "bg2_core_layers_only"])
def test_nms_layered_few_layers(case):
    """Codes with as few layers as the check-state prefetch distance (four
    core rows of a BG-shaped code sent at its highest rate) and fewer (an
    11n-shaped code with three rows) against the oracle, every round."""
    from inputs.qc_base import draw_base
    from inputs.workloads import BG2
    from oracle import pipeline
    if case == "11n_three_layers":
        qb = draw_base("11n", 3, 12, 27, seed=11)
        e_tx, want_rows = 12 * 27, 3
    else:
        qb = BG2.load()
        e_tx, want_rows = (qb.kb + 4) * qb.Z - 2 * qb.Z, 4
    g = qc.graph_from_qcbase(qb, e_tx)
    assert g.rows == want_rows
    code = lsim.Code.from_qcbase(qb, e_tx)
    B = 9
    n0 = np.full(B, float(pipeline.n0_for(g, 4.5, 1)))
    tx = pipeline.transmit(g, qb.family, 71, 0, B, n0, 1)
    L32 = tx["L"].astype(np.float32)
    lam = D.channel_lam(g, L32, dtype=np.float32)
    app, hist = D.nms_layered(g, lam, 20, alpha=0.75, mode="fp32", trace=True)
    tl = T(L32).to(dev)
    for t in (1, 2, 3, 5, 20):
        r, _, lp = lsim.decode_state(code, tl, lsim.params(lsim.NMS_F32, iters=t, alpha=0.75))
        assert np.array_equal(r.cpu().numpy(), hist[t - 1][0]), t
        assert np.array_equal(lp.cpu().numpy(), -hist[t - 1][1]), t
    bits, _ = lsim.decode(code, tl, lsim.params(lsim.NMS_F32, iters=20, alpha=0.75))
    assert np.array_equal(bits.cpu().numpy(), D.hard_bits(app, g.k))


def test_grouped_order_equals_the_oracles():
    """The library's grouped layer order (its own DSatur colouring) is the
    oracle's on every workload code and mixed shape, and the number of
    workgroup barriers the schedule table takes per iteration, for the
    natural, grouped and a shuffled order, is the count of runs of rows
    with no common column (plus the end of the iteration), recomputed here
    from the graph."""
    from inputs.workloads import BG1, BG2, SMALL, mixed_specs
    cases = [(BG1, 25344), (BG2, 3840), (SMALL, 648)] + list(mixed_specs())
    for spec, e_tx in cases:
        qb = spec.load()
        g = qc.graph_from_qcbase(qb, e_tx)
        code = lsim.Code.from_qcbase(qb, e_tx)
        code.set_layer_order("grouped")
        assert code.layer_order()[0] == D.grouped_order(g), spec.name
        # the workgroup barriers the schedule takes: a barrier before a row
        # that shares a column with a row since the last one, and one at the
        # end of every iteration
        cols = [set(g.entries[g.row_entries(i), 1].tolist()) for i in range(g.rows)]

        def barriers(order):
            n, cur = 1, set()
            for i in order:
                if cols[i] & cur:
                    n, cur = n + 1, set()
                cur |= cols[i]
            return n

        assert code.layer_order()[1] == barriers(D.grouped_order(g)), spec.name
        shuffled = np.random.default_rng(9).permutation(g.rows).tolist()
        code.set_layer_order(shuffled)
        assert code.layer_order()[1] == barriers(shuffled), spec.name
        code.set_layer_order("natural")
        assert code.layer_order()[1] == barriers(range(g.rows)), spec.name


@pytest.mark.parametrize("name,B", [("bg2", 4096), ("bg1", 1024)])
def test_layered_full_batch_is_deterministic_in_both_orders(name, B):
    """Full-batch decodes repeated in natural and grouped order (whose
    schedules skip the barriers between layers with disjoint LDS columns)
    give identical bits and posteriors every time: a missing barrier would
    show as run-to-run differences."""
    qb, g, code = gcode(name)
    gen = torch.Generator(device="cpu").manual_seed(17)
    llr = (torch.randn((B, g.e_tx), generator=gen) * 3 + 1.0).to(dev)
    p = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
    for order in ("natural", "grouped"):
        code.set_layer_order(order)
        ref = lsim.decode(code, llr, p, want_app=True)
        for _ in range(6):
            out = lsim.decode(code, llr, p, want_app=True)
            assert torch.equal(out[0], ref[0]) and torch.equal(out[1], ref[1]), order
    code.set_layer_order("natural")


def test_layered_rejects_an_inner_degree_one_column():
    """The layered decoder reads a degree-one variable node's message from
    the channel only where the node closes its row; any other degree-one
    column is refused (never decoded in a different arithmetic), while the
    flooding decoders take the code."""
    from inputs.workloads import SMALL
    qb = SMALL.load()
    b = qb.base.copy()
    rows = np.nonzero(b[:, 0] >= 0)[0]
    b[rows[1:], 0] = -1                       # information column 0 in one row only
    code = lsim.Code(b, qb.Z, qb.family, qb.n_punct_cols, 648)
    llr = -torch.ones(3, 648, device=dev)    # the all-zero codeword, L = ln p(1)/p(0)
    with pytest.raises(lsim.LsimError, match="degree one"):
        lsim.decode(code, llr, lsim.params(lsim.NMS_F32))
    bits, _ = lsim.decode(code, llr, lsim.params(lsim.SPA_F32))
    assert not bits.any()


@pytest.mark.parametrize("offset,sat", [(0, 31), (2, 31), (1, 15), (1, 127)])
def test_oms_parameters_bit_exact(offset, sat):
    """int8 offset min-sum with other offsets and saturation levels (the
    packed 16-bit kernel keeps every value exact up to sat = 127)."""
    qb, g, code = gcode("bg2")
    tx = oracle_llrs("bg2", 11, 3.0, 83)
    q = modem.quantize(tx["L"].astype(np.float32), 2.0, sat)
    app = D.oms_flood(g, D.channel_lam(g, q, np.int64), 20, offset=offset, sat=sat)
    p = lsim.params(lsim.OMS_I8, iters=20, offset=offset, sat=sat)
    bits, lp = lsim.decode(code, T(q).to(dev), p, want_app=True)
    assert np.array_equal(lp.cpu().numpy(), -app)
    assert np.array_equal(bits.cpu().numpy(), D.hard_bits(app, g.k))


@pytest.mark.parametrize("alpha", [0.5, 1.0])
def test_nms_alpha_bit_exact(alpha):
    qb, g, code = gcode("bg2")
    tx = oracle_llrs("bg2", 9, 3.0, 89)
    L32 = tx["L"].astype(np.float32)
    app = D.nms_layered(g, D.channel_lam(g, L32, dtype=np.float32), 20, alpha=alpha, mode="fp32")
    _, lp = lsim.decode(code, T(L32).to(dev), lsim.params(lsim.NMS_F32, alpha=alpha),
                        want_app=True)
    assert np.array_equal(lp.cpu().numpy(), -app)


def test_spa_other_clamp():
    """Sum-product with messages clamped at 10 instead of 20."""
    qb, g, code = gcode("bg2")
    tx = oracle_llrs("bg2", 32, 3.5, 97)
    L32 = tx["L"].astype(np.float32)
    app = D.spa_flood(g, D.channel_lam(g, L32.astype(np.float64)), 20, llr_max=10.0)
    hard = (app < 0).astype(np.uint8)
    conv = ~qc.syndrome(qb.base[:g.rows, :g.cols], qb.Z, hard).any(axis=1)
    assert conv.sum() >= 8
    _, lp = lsim.decode(code, T(L32).to(dev), lsim.params(lsim.SPA_F32, llr_max=10.0),
                        want_app=True)
    ok, w = rel_close(lp.cpu().numpy()[conv], -app[conv], 1e-4)
    assert ok, w


def test_layered_at_the_largest_lift():
    """The 11n-style base matrix lifted by Z = 1024 (the largest lift the
    library takes; n = 24576): layered NMS with 1024 threads, bit for bit
    against the oracle's single-precision mode."""
    qb, _ = graph("small")
    Z = 1024
    n = qb.base.shape[1] * Z
    code = lsim.Code(qb.base, Z, qb.family, 0, n)
    g = qc.make_graph(qb.base, qb.kb, Z, 0, n, family=qb.family)
    B = 2
    u = np.random.default_rng(11).integers(0, 2, (B, qb.kb * Z)).astype(np.uint8)
    c = qc.encode(qb.base, qb.kb, Z, qb.family, u)
    n0 = float(modem.ebn0_to_n0(2.0, 0.5, 1))
    y = (1.0 - 2.0 * c) + np.sqrt(n0 / 2.0) * np.random.default_rng(12).standard_normal(c.shape)
    L = (-4.0 * y / n0).astype(np.float32)
    p = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75, threads=1024)
    bits, app = lsim.decode(code, T(L).to(dev), p, want_app=True)
    ref = D.nms_layered(g, D.channel_lam(g, L, dtype=np.float32), 20, 0.75, mode="fp32")
    assert np.array_equal(app.cpu().numpy(), -ref)
    assert np.array_equal(bits.cpu().numpy(), D.hard_bits(ref, code.k))


def test_spa_one_round_with_the_largest_lds_state():
    """The BG2-shaped base lifted by Z = 256 (31.2 k edges: 122 KiB of
    messages plus 32 KiB of channel values, 154 KiB of the 160 KiB of LDS,
    a runtime lift): one sum-product round from an oracle state against
    the oracle, 1e-4 relative."""
    qb, _ = graph("bg2")
    Z = 256
    e_tx = 30 * Z
    code = lsim.Code(qb.base, Z, qb.family, qb.n_punct_cols, e_tx)
    g = qc.make_graph(qb.base, qb.kb, Z, qb.n_punct_cols, e_tx, family=qb.family)
    assert 4 * (g.E + g.n_dec) > 128 * 1024
    B = 3
    rng = np.random.default_rng(21)
    L32 = (rng.standard_normal((B, e_tx)) * 4.0).astype(np.float32)
    lam = np.clip(D.channel_lam(g, L32.astype(np.float64)), -20, 20)
    _, _, qs = D.spa_flood(g, lam, 3, trace=True)
    q32 = qs[2].astype(np.float32)
    r_ref, app_ref, q_ref = D.spa_iteration(g, lam, q32.astype(np.float64))
    p = lsim.params(lsim.SPA_F32, iters=1, llr_max=20.0)
    r, qq, lp = lsim.decode_state(code, T(L32).to(dev), p, q_in=T(q32).to(dev))
    for got, ref in ((r, r_ref), (qq, q_ref), (lp, -app_ref)):
        ok, w = rel_close(got.cpu().numpy(), ref, 1e-4)
        assert ok, w


def test_oms_with_the_largest_lds_state():
    """int8 offset min-sum on the BG2-shaped base at Z = 256 (packed pair
    state 154 KiB of LDS, runtime lift), three codewords (the second pair
    half empty): posteriors and bits equal the oracle's after 20 rounds."""
    qb, _ = graph("bg2")
    Z = 256
    e_tx = 30 * Z
    code = lsim.Code(qb.base, Z, qb.family, qb.n_punct_cols, e_tx)
    g = qc.make_graph(qb.base, qb.kb, Z, qb.n_punct_cols, e_tx, family=qb.family)
    B = 3
    rng = np.random.default_rng(22)
    u = rng.integers(0, 2, (B, qb.kb * Z)).astype(np.uint8)
    c = qc.encode(qb.base, qb.kb, Z, qb.family, u)
    t = c[:, g.tx_lo:g.tx_lo + e_tx].astype(np.float64)
    L = (2.0 * t - 1.0) * 2.0 + rng.standard_normal(t.shape) * 2.0
    q = modem.quantize(L.astype(np.float32))
    p = lsim.params(lsim.OMS_I8, iters=20)
    bits, lp = lsim.decode(code, T(q).to(dev), p, want_app=True)
    ref = D.oms_flood(g, D.channel_lam(g, q, dtype=np.int64), 20)
    assert np.array_equal(lp.cpu().numpy(), -ref.astype(np.float32))
    assert np.array_equal(bits.cpu().numpy(), D.hard_bits(ref, code.k))
