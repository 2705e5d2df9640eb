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


SAMPLE = [0, 1, 1234, 2047, 3071, 4095]


@pytest.mark.parametrize("algo", ["spa", "oms"])
def test_bg2_full_batch_sampled(algo):
    qb = BG2.load()
    code = lsim.Code.from_qcbase(qb, 3840)
    g = qc.graph_from_qcbase(qb, 3840)
    B, m = 4096, 4
    pts = np.arange(9) * 0.5
    n0 = lsim.ebn0_to_n0(pts, code.k / code.e_tx, m)[np.arange(B) % 9].astype(np.float32)
    p = lsim.params(lsim.SPA_F32 if algo == "spa" else lsim.OMS_I8)
    link = lsim.Link(code, m, lsim.DEMAP_MAXLOG, p, B, T(n0).to(dev), device=dev)
    seed = data_seed(2, 4242)
    link.run(seed, 0)
    u, bits = link.u.cpu().numpy(), link.bits.cpu().numpy()
    llr_gpu = link.llr.cpu().numpy()
    for b in SAMPLE:
        tx = pipeline.transmit(g, qb.family, seed, b, 1, n0[b:b + 1].astype(np.float64), m, "maxlog")
        assert np.array_equal(u[b], tx["u"][0]), b
        if algo == "oms":
            # same int8 LLRs on both sides: posteriors bit-exact
            q = llr_gpu[b:b + 1]
            app = D.oms_flood(g, D.channel_lam(g, q, np.int64), 20)
            assert np.array_equal(bits[b], D.hard_bits(app, g.k)[0]), b
        else:
            L = llr_gpu[b:b + 1].astype(np.float64)
            app = D.spa_flood(g, D.channel_lam(g, L), 20)
            hard = (app < 0).astype(np.uint8)
            if not qc.syndrome(qb.base[:g.rows, :g.cols], qb.Z, hard).any():
                assert np.array_equal(bits[b], D.hard_bits(app, g.k)[0]), b
    # posteriors of the sampled codewords through lsim_decode on the same LLRs
    sel = T(np.array(SAMPLE)).to(dev)
    sub = link.llr.index_select(0, sel).contiguous()
    _, lp = lsim.decode(code, sub, p, want_app=True)
    lp = lp.cpu().numpy()
    for j, b in enumerate(SAMPLE):
        if algo == "oms":
            app = D.oms_flood(g, D.channel_lam(g, llr_gpu[b:b + 1], np.int64), 20)
            assert np.array_equal(lp[j], -app[0])
        else:
            app = D.spa_flood(g, D.channel_lam(g, llr_gpu[b:b + 1].astype(np.float64)), 20)
            hard = (app < 0).astype(np.uint8)
            if not qc.syndrome(qb.base[:g.rows, :g.cols], qb.Z, hard).any():
                ok, w = rel_close(lp[j], -app[0], 1e-4)
                assert ok, (b, w)


def test_bg1_full_batch_sampled():
    qb = BG1.load()
    code = lsim.Code.from_qcbase(qb, 25344)
    g = qc.graph_from_qcbase(qb, 25344)
    B, m = 1024, 6
    n0 = np.full(B, lsim.ebn0_to_n0(3.0, code.k / code.e_tx, m), dtype=np.float32)
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
