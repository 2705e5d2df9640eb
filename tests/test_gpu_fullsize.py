"""Parity at the benchmark's full sizes and launch configuration, on
sampled codewords the oracle decodes one by one, plus edge cases.

* BG2 workload: 4096 codewords through lsim_link_run (the bench step,
  codewords kept on chip), sampled codewords re-run through the oracle's
  link from the same Philox seeds: information bits bit-exact; int8 OMS
  posteriors bit-exact on
  the same quantized LLRs; FP32 SPA within 1e-4 on converged frames.
* BG1 workload: 1024 codewords layered NMS, sampled codewords bit-exact.
* Mixed batch at the benchmark's counts: sampled codewords per shape
  bit-exact against the oracle.
* Edge cases: a batch of one, an all-zero LLR input, saturated inputs,
  invalid sizes rejected.
"""
import numpy as np
import pytest
import torch

from helpers import graph, rel_close
from inputs.workloads import BG1, BG2, data_seed, mixed_counts, mixed_specs
from oracle import decoders as D
from oracle import modem, pipeline, qc

pytestmark = pytest.mark.gpu

lsim = pytest.importorskip("paper_2203_11854_amd")
dev = "cuda"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x))


# Codewords of the 4096-codeword BG2 batch compared with the oracle.  Row b
# runs at Eb/N0 0.5*(b % 9) dB: LOW rows sit at 0-2 dB (mostly undecodable),
# HIGH rows at 3.0, 3.5 and 4.0 dB spread over the whole batch, where most
# frames converge and the FP32 posteriors are compared element by element.
LOW = [0, 1, 1234, 2047, 3071, 4095]
HIGH = [9 * j + o for j in (0, 113, 227, 340, 454) for o in (6, 7, 8)]
SAMPLE = LOW + HIGH


def _bg2_link(algo, seed):
    qb = BG2.load()
    code = lsim.Code.from_qcbase(qb, 3840)
    g = qc.graph_from_qcbase(qb, 3840)
    B, m = 4096, 4
    n0 = pipeline.n0_for(g, np.arange(9) * 0.5, m)[np.arange(B) % 9].astype(np.float32)
    p = lsim.params(lsim.SPA_F32 if algo == "spa" else lsim.OMS_I8)
    link = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p, B, T(n0).to(dev), device=dev)
    link.run(seed, 0)
    # the oracle's own link on the sampled codewords (same Philox seeds)
    tx = {b: pipeline.transmit(g, qb.family, seed, b, 1, n0[b:b + 1].astype(np.float64), m,
                               "maxlog") for b in SAMPLE}
    return qb, g, code, p, link, tx


def _converged(qb, g, app):
    hard = (app < 0).astype(np.uint8)
    return ~qc.syndrome(qb.base[:g.rows, :g.cols], qb.Z, hard).any(axis=1)


@pytest.mark.parametrize("algo", ["spa", "oms"])
def test_bg2_full_batch_sampled(algo):
    """The bench's BG2 step (4096 codewords through lsim_link_run), then the
    4096-codeword decoder launch on the oracle's LLRs of the sampled rows."""
    seed = data_seed(2, 4242)
    qb, g, code, p, link, tx = _bg2_link(algo, seed)
    u, bits = link.u.cpu().numpy(), link.bits.cpu().numpy()
    llr_gpu = link.llr.cpu().numpy()
    # oracle LLRs of the sampled rows: float32 boundary LLRs, int8 for OMS
    L32 = {b: tx[b]["L"].astype(np.float32) for b in SAMPLE}
    Lin = {b: (modem.quantize(L32[b]) if algo == "oms" else L32[b]) for b in SAMPLE}
    ref_app = {}
    for b in SAMPLE:
        assert np.array_equal(u[b], tx[b]["u"][0]), b
        if algo == "oms":
            # the link's fused demap + quantize against the oracle's: a level
            # may differ only where 2L lies within float32 rounding of a
            # half-integer
            d = np.abs(llr_gpu[b].astype(np.int32) - Lin[b][0].astype(np.int32))
            assert d.max() <= 1 and (d.sum() <= 2), b
            ref_app[b] = D.oms_flood(g, D.channel_lam(g, Lin[b], np.int64), 20)[0]
        else:
            ok, w = rel_close(llr_gpu[b], tx[b]["L"][0], 1e-4)
            assert ok, (b, w)
            ref_app[b] = D.spa_flood(g, D.channel_lam(g, L32[b].astype(np.float64)), 20)[0]
    conv = {b: bool(_converged(qb, g, ref_app[b][None])[0]) for b in SAMPLE}
    # the link's own decisions on frames the oracle decodes to a codeword
    for b in SAMPLE:
        if conv[b]:
            assert np.array_equal(bits[b], D.hard_bits(ref_app[b][None], g.k)[0]), b
    # the full 4096-codeword decoder launch with the sampled rows replaced by
    # the oracle's LLRs: posteriors row by row
    full = link.llr.clone()
    for b in SAMPLE:
        full[b] = T(Lin[b][0]).to(dev)
    gb, lp = lsim.decode(code, full, p, want_app=True)
    lp, gb = lp.cpu().numpy(), gb.cpu().numpy()
    compared = 0
    for b in SAMPLE:
        if algo == "oms":
            assert np.array_equal(lp[b], -ref_app[b]), b
            assert np.array_equal(gb[b], D.hard_bits(ref_app[b][None], g.k)[0]), b
            compared += 1
        elif conv[b]:
            ok, w = rel_close(lp[b], -ref_app[b], 1e-4)
            assert ok, (b, w)
            assert np.array_equal(gb[b], D.hard_bits(ref_app[b][None], g.k)[0]), b
            compared += 1
    print(f"{algo}: {compared} of {len(SAMPLE)} sampled posteriors compared")
    assert compared >= (len(SAMPLE) if algo == "oms" else 10)


@pytest.mark.parametrize("algo", ["spa", "oms"])
def test_bg2_full_batch_one_round_from_oracle_state(algo):
    """One teacher-forced round over the whole 4096-codeword batch
    (lsim_decode_state): the sampled rows start from the oracle's messages
    after t rounds, every other row from zero messages; their r, q and
    posteriors after the round against the oracle's round from the same
    state."""
    seed = data_seed(2, 4243)
    qb, g, code, p, link, tx = _bg2_link(algo, seed)
    B, E = link.llr.shape[0], code.E
    full = link.llr.clone()
    mt = np.int8 if algo == "oms" else np.float32
    q_in = np.zeros((B, E), dtype=mt)
    refs = {}
    for j, b in enumerate(SAMPLE):
        L32 = tx[b]["L"].astype(np.float32)
        t0 = (0, 1, 4, 9, 18)[j % 5]
        if algo == "oms":
            x = modem.quantize(L32)
            lam = D.channel_lam(g, x, np.int64)
            _, _, qs = D.oms_flood(g, lam, max(t0, 1), trace=True)
            q0 = lam[:, g.edge_vn()] if t0 == 0 else qs[t0 - 1]
            q0 = np.clip(q0, -31, 31)
            r_ref, app_ref, q_ref = D.oms_iteration(g, lam, q0)
        else:
            x = L32
            lam = np.clip(D.channel_lam(g, L32.astype(np.float64)), -20, 20)
            _, _, qs = D.spa_flood(g, lam, max(t0, 1), trace=True)
            q0 = (lam[:, g.edge_vn()] if t0 == 0 else qs[t0 - 1]).astype(np.float32)
            r_ref, app_ref, q_ref = D.spa_iteration(g, lam, q0.astype(np.float64))
        full[b] = T(x[0]).to(dev)
        q_in[b] = q0[0].astype(mt)
        refs[b] = (r_ref[0], q_ref[0], -app_ref[0])
    pr = lsim.params(lsim.SPA_F32 if algo == "spa" else lsim.OMS_I8, iters=1)
    r, qq, lpo = lsim.decode_state(code, full, pr, q_in=T(q_in).to(dev))
    r, qq, lpo = r.cpu().numpy(), qq.cpu().numpy(), lpo.cpu().numpy()
    worst = 0.0
    for b in SAMPLE:
        for got, ref in zip((r[b], qq[b], lpo[b]), refs[b]):
            if algo == "oms":
                assert np.array_equal(got, ref), b
            else:
                ok, w = rel_close(got, ref, 1e-4)
                worst = max(worst, w)
                assert ok, (b, w)
    print(f"{algo}: worst relative error {worst:.2e}")


def test_bg1_full_batch_sampled():
    qb = BG1.load()
    code = lsim.Code.from_qcbase(qb, 25344)
    g = qc.graph_from_qcbase(qb, 25344)
    B, m = 1024, 6
    n0 = np.full(B, pipeline.n0_for(g, 3.0, m), dtype=np.float32)
    p = lsim.params(lsim.NMS_F32)
    link = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p, B, T(n0).to(dev), device=dev)
    seed = data_seed(3, 77)
    link.run(seed, 0)
    llr = link.llr.cpu().numpy()
    bits = link.bits.cpu().numpy()
    for b in (0, 511, 1023):
        lam = D.channel_lam(g, llr[b:b + 1], dtype=np.float32)
        app = D.nms_layered(g, lam, 20, 0.75, mode="fp32")
        assert np.array_equal(bits[b], D.hard_bits(app, g.k)[0]), b


def test_mixed_bench_counts_sampled():
    specs = mixed_specs()
    counts = mixed_counts()
    p = lsim.params(lsim.NMS_F32)
    codes, llrs, graphs = [], [], []
    for s, ((spec, e_tx), cnt) in enumerate(zip(specs, counts)):
        qb = spec.load()
        code = lsim.Code.from_qcbase(qb, e_tx)
        m = 2 if s % 2 else 4
        no = T(np.full(cnt, lsim.ebn0_to_n0(2.0 + 0.3 * s, code.k / e_tx, m), dtype=np.float32)).to(dev)
        u = lsim.source_bits(data_seed(4, s), 0, cnt, code.k, dev)
        c = lsim.encode(code, u)
        y = lsim.map_awgn(code, m, c, no, data_seed(4, s), 0)
        llrs.append(lsim.demap(m, lsim.DEMAP_MAXLOG, y, no))
        codes.append(code)
        graphs.append(qc.graph_from_qcbase(qb, e_tx))
    plan = lsim.MixedPlan(codes, counts, p)
    cat = torch.cat([x.reshape(-1) for x in llrs])
    app = torch.empty(plan.n_app, dtype=torch.float32, device=dev)
    plan.decode(cat, app=app)
    app = app.cpu().numpy()
    for s, (code, L, g) in enumerate(zip(codes, llrs, graphs)):
        Lh = L.cpu().numpy()
        o = plan.app_offsets[s]
        for b in sorted({0, counts[s] // 2, counts[s] - 1}):
            ref = D.nms_layered(g, D.channel_lam(g, Lh[b:b + 1], dtype=np.float32), 20, 0.75,
                                mode="fp32")
            got = app[o + b * code.n_dec:o + (b + 1) * code.n_dec]
            assert np.array_equal(got, -ref[0]), (s, b)


@pytest.mark.parametrize("algo", ["spa", "oms", "nms"])
def test_edge_cases(algo):
    qb, g = graph("bg2")
    code = lsim.Code.from_qcbase(qb, 3840)
    dt = np.int8 if algo == "oms" else np.float32
    p = lsim.params({"spa": lsim.SPA_F32, "oms": lsim.OMS_I8, "nms": lsim.NMS_F32}[algo])
    # batch of one, all-zero channel: posteriors stay exactly zero, bits 0
    z = T(np.zeros((1, 3840), dtype=dt)).to(dev)
    bits, lp = lsim.decode(code, z, p, want_app=True)
    assert not bits.any() and not lp.abs().max().item()
    # saturated correct inputs decode the codeword
    u = np.random.default_rng(3).integers(0, 2, (2, code.k)).astype(np.uint8)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    t = c[:, g.tx_lo:g.tx_lo + g.e_tx].astype(np.float32)
    L = (2 * t - 1) * (15.0 if algo == "oms" else 1e6)
    x = T(L.astype(dt) if algo != "oms" else np.clip(L, -31, 31).astype(np.int8)).to(dev)
    bits, _ = lsim.decode(code, x, p)
    assert np.array_equal(bits.cpu().numpy(), u)
    with pytest.raises(lsim.LsimError):
        lsim.decode(code, T(np.zeros((0, 3840), dtype=dt)).to(dev), p)
