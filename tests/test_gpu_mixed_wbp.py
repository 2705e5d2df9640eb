"""GPU parity of the mixed-shape persistent decoder and of the
differentiable forms (weighted BP forward/adjoint, neural demapper, BCE,
Adam)."""
import numpy as np
import pytest
import torch

from helpers import rel_close
from inputs import rand
from inputs.workloads import BG2, mixed_specs
from oracle import decoders as D
from oracle import ndm as ondm
from oracle import modem, pipeline, qc, wbp

pytestmark = pytest.mark.gpu

lsim = pytest.importorskip("paper_2203_11854_amd")
dev = "cuda"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x))


def mixed_inputs(counts, seed=71):
    shapes, llrs, graphs, qbs = [], [], [], []
    for s, ((spec, e_tx), cnt) in enumerate(zip(mixed_specs(), counts)):
        qb = spec.load()
        g = qc.graph_from_qcbase(qb, e_tx)
        m = 2 if s % 2 == 0 else 4
        eb = rand.uniform(seed + s, cnt, 0.0, 6.0)
        n0 = pipeline.n0_for(g, eb, m)
        tx = pipeline.transmit(g, qb.family, seed + 100 + s, 0, cnt, n0, m, "maxlog")
        llrs.append(tx["L"].astype(np.float32))
        graphs.append(g)
        qbs.append(qb)
        shapes.append(lsim.Code.from_qcbase(qb, e_tx))
    return shapes, llrs, graphs, qbs


def test_mixed_persistent_equals_per_shape_and_oracle():
    counts = [5, 9, 3, 7, 4, 6, 2, 3]
    codes, llrs, graphs, _ = mixed_inputs(counts)
    p = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
    plan = lsim.MixedPlan(codes, counts, p)
    cat = T(np.concatenate([x.reshape(-1) for x in llrs])).to(dev)
    bits = torch.zeros(plan.n_bits, dtype=torch.uint8, device=dev)
    app = torch.zeros(plan.n_app, dtype=torch.float32, device=dev)
    plan.decode(cat, bits=bits, app=app, persistent=True)
    bits2 = torch.zeros_like(bits)
    app2 = torch.zeros_like(app)
    plan.decode(cat, bits=bits2, app=app2, persistent=False)
    assert torch.equal(bits, bits2) and torch.equal(app, app2)
    for s, (code, L, g) in enumerate(zip(codes, llrs, graphs)):
        b1, a1 = lsim.decode(code, T(L).to(dev), p, want_app=True)
        lo, n = plan.app_offsets[s], counts[s] * code.n_dec
        assert torch.equal(app[lo:lo + n].view(counts[s], -1), a1), s
        bo = plan.bits_offsets[s]
        assert torch.equal(bits[bo:bo + counts[s] * code.k].view(counts[s], -1), b1), s
        ref = D.nms_layered(g, D.channel_lam(g, L, dtype=np.float32), 20, 0.75, mode="fp32")
        assert np.array_equal(a1.cpu().numpy(), -ref), s


def test_mixed_graph_replay():
    counts = [4, 3, 5, 2, 3, 2, 1, 2]
    codes, llrs, _, _ = mixed_inputs(counts, seed=90)
    p = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
    plan = lsim.MixedPlan(codes, counts, p)
    cat = T(np.concatenate([x.reshape(-1) for x in llrs])).to(dev)
    work = plan.workspace(dev)
    ref = torch.zeros(plan.n_app, dtype=torch.float32, device=dev)
    plan.decode(cat, app=ref, work=work)
    torch.cuda.synchronize()
    out = torch.zeros_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.decode(cat, app=out, work=work)     # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.decode(cat, app=out, work=work)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        _ = (cat * 2).sum()                        # unrelated eager work between replays
        torch.cuda.synchronize()


def oms_fit(codes, llrs, graphs, counts):
    """The shapes whose packed int8 state (4 B per edge and per variable
    node for a codeword pair) fits the 160 KiB of LDS."""
    keep = [s for s, c in enumerate(codes) if 4 * (c.E + c.n_dec) <= 160 * 1024 - 96]
    assert len(keep) >= 4
    return ([codes[s] for s in keep], [llrs[s] for s in keep], [graphs[s] for s in keep],
            [counts[s] for s in keep])


@pytest.mark.parametrize("threads", [0, 256, 1024])
def test_mixed_oms_equals_per_shape_and_oracle(threads):
    """The int8 offset min-sum decoder over the shapes whose state fits the
    LDS, in one persistent launch (odd counts leave a half-empty last pair):
    bits and posteriors equal the per-shape launches and the oracle bit for
    bit."""
    codes, llrs, graphs, _ = mixed_inputs([5, 9, 3, 7, 4, 6, 2, 3], seed=75)
    codes, llrs, graphs, counts = oms_fit(codes, llrs, graphs, [5, 9, 3, 7, 4, 6, 2, 3])
    p = lsim.params(lsim.OMS_I8, iters=20, offset=1.0, sat=31)
    q8 = [lsim.quantize(T(L).to(dev)) for L in llrs]
    plan = lsim.MixedPlan(codes, counts, p, threads=threads)
    cat = torch.cat([q.reshape(-1) for q in q8])
    bits = torch.zeros(plan.n_bits, dtype=torch.uint8, device=dev)
    app = torch.zeros(plan.n_app, dtype=torch.float32, device=dev)
    plan.decode(cat, bits=bits, app=app, persistent=True)
    bits2, app2 = torch.zeros_like(bits), torch.zeros_like(app)
    plan.decode(cat, bits=bits2, app=app2, persistent=False)
    assert torch.equal(bits, bits2) and torch.equal(app, app2)
    for s, (code, q, g) in enumerate(zip(codes, q8, graphs)):
        b1, a1 = lsim.decode(code, q, p, want_app=True)
        lo, n = plan.app_offsets[s], counts[s] * code.n_dec
        assert torch.equal(app[lo:lo + n].view(counts[s], -1), a1), s
        bo = plan.bits_offsets[s]
        assert torch.equal(bits[bo:bo + counts[s] * code.k].view(counts[s], -1), b1), s
        qo = modem.quantize(llrs[s])                     # the oracle's own quantizer
        assert np.array_equal(q.cpu().numpy(), qo), s
        ref = D.oms_flood(g, D.channel_lam(g, qo, dtype=np.int64), 20)
        assert np.array_equal(a1.cpu().numpy(), -ref.astype(np.float32)), s


def test_mixed_oms_covers_every_shape():
    """All eight shapes in one int8 offset min-sum launch: the shapes whose
    pair state does not fit the LDS take one codeword per tile (16-bit
    state); bits and posteriors equal the per-shape launches and, on
    sampled codewords, the oracle bit for bit."""
    counts = [5, 4, 3, 7, 3, 4, 2, 3]
    codes, llrs, graphs, _ = mixed_inputs(counts, seed=77)
    assert any(4 * (c.E + c.n_dec) > 160 * 1024 - 96 for c in codes)
    p = lsim.params(lsim.OMS_I8, iters=20, offset=1.0, sat=31)
    q8 = [T(modem.quantize(L)).to(dev) for L in llrs]
    plan = lsim.MixedPlan(codes, counts, p)
    cat = torch.cat([q.reshape(-1) for q in q8])
    bits = torch.zeros(plan.n_bits, dtype=torch.uint8, device=dev)
    app = torch.zeros(plan.n_app, dtype=torch.float32, device=dev)
    plan.decode(cat, bits=bits, app=app)
    for s, (code, q, g, L) in enumerate(zip(codes, q8, graphs, llrs)):
        b1, a1 = lsim.decode(code, q, p, want_app=True)
        lo, n = plan.app_offsets[s], counts[s] * code.n_dec
        assert torch.equal(app[lo:lo + n].view(counts[s], -1), a1), s
        bo = plan.bits_offsets[s]
        assert torch.equal(bits[bo:bo + counts[s] * code.k].view(counts[s], -1), b1), s
        rows = [0, counts[s] - 1]
        ref = D.oms_flood(g, D.channel_lam(g, modem.quantize(L[rows]), dtype=np.int64), 20)
        assert np.array_equal(a1.cpu().numpy()[rows], -ref.astype(np.float32)), s


def test_oms_single_codeword_tiles_equal_pairs():
    """Forcing one codeword per tile on shapes whose pairs fit gives the
    pair tiles' bits and posteriors exactly, through the persistent launch
    and one workgroup per tile."""
    counts = [5, 9, 3, 7, 4, 6, 2, 3]
    codes, llrs, graphs, _ = mixed_inputs(counts, seed=79)
    codes, llrs, graphs, counts = oms_fit(codes, llrs, graphs, counts)
    p = lsim.params(lsim.OMS_I8, iters=20)
    cat = torch.cat([T(modem.quantize(L)).to(dev).reshape(-1) for L in llrs])
    outs = []
    for cpt in ([2] * len(codes), [1] * len(codes)):
        plan = lsim.MixedPlan(codes, counts, p, codewords_per_tile=cpt)
        for persistent in (True, False):
            bits = torch.zeros(plan.n_bits, dtype=torch.uint8, device=dev)
            app = torch.zeros(plan.n_app, dtype=torch.float32, device=dev)
            plan.decode(cat, bits=bits, app=app, persistent=persistent)
            outs.append((bits, app))
    for b, a in outs[1:]:
        assert torch.equal(b, outs[0][0]) and torch.equal(a, outs[0][1])


def test_mixed_oms_graph_replay():
    codes, llrs, graphs, _ = mixed_inputs([4, 3, 5, 2, 3, 2, 1, 2], seed=91)
    codes, llrs, _, counts = oms_fit(codes, llrs, graphs, [4, 3, 5, 2, 3, 2, 1, 2])
    p = lsim.params(lsim.OMS_I8, iters=20)
    plan = lsim.MixedPlan(codes, counts, p)
    cat = torch.cat([lsim.quantize(T(L).to(dev)).reshape(-1) for L in llrs])
    work = plan.workspace(dev)
    ref = torch.zeros(plan.n_bits, dtype=torch.uint8, device=dev)
    plan.decode(cat, bits=ref, work=work)
    torch.cuda.synchronize()
    out = torch.zeros_like(ref)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.decode(cat, bits=out, work=work)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.decode(cat, bits=out, work=work)
    for rep in range(3):
        out.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), rep
        _ = (cat.float() * 2).sum()
        torch.cuda.synchronize()


def test_autotuner_mixed_oms():
    from paper_2203_11854_amd import autotune
    codes, llrs, graphs, _ = mixed_inputs([3, 4, 5, 2, 3, 2, 3, 2], seed=93)
    codes, llrs, _, counts = oms_fit(codes, llrs, graphs, [3, 4, 5, 2, 3, 2, 3, 2])
    p = lsim.params(lsim.OMS_I8, iters=20)
    cat = torch.cat([lsim.quantize(T(L).to(dev)).reshape(-1) for L in llrs])
    best = autotune.tune_mixed(codes, counts, p, cat, cache_path=None)
    assert best["threads"] in (256, 512, 1024) and best["codewords_per_tile"] == [2] * len(codes)
    ref = lsim.MixedPlan(codes, counts, p).decode(cat, bits=torch.zeros(
        sum(c.k * k for c, k in zip(codes, counts)), dtype=torch.uint8, device=dev))[0]
    tuned = lsim.MixedPlan(codes, counts, p, codewords_per_tile=best["codewords_per_tile"],
                           threads=best["threads"])
    out = tuned.decode(cat, bits=torch.zeros_like(ref), persistent=best["persistent"])[0]
    assert torch.equal(out, ref)


def wbp_case(B=5, Tn=3, ebn0=1.0, seed=81):
    qb = BG2.load()
    g = qc.graph_from_qcbase(qb, 3840)
    n0 = float(pipeline.n0_for(g, ebn0, 4))
    tx = pipeline.transmit(g, qb.family, seed, 0, B, np.full(B, n0), 4, "maxlog")
    L32 = tx["L"].astype(np.float32)
    w = rand.uniform(seed + 1, (Tn, g.E), 0.7, 1.3).astype(np.float32)
    c = tx["c"][:, :g.n_dec]
    return qb, g, L32, w, c


def test_wbp_forward_vs_oracle():
    qb, g, L32, w, c = wbp_case()
    code = lsim.Code.from_qcbase(qb, 3840)
    lp, ck = lsim.wbp_forward(code, T(w).to(dev), T(L32).to(dev), 3)
    ref = wbp.forward_numpy(g, D.channel_lam(g, L32.astype(np.float64)), w.astype(np.float64))
    ok, worst = rel_close(lp.cpu().numpy(), -ref, 1e-4)
    assert ok, worst
    # unit weights: the plain sum-product decoder (the two kernels may
    # contract multiply-adds differently, hence a few-ulp tolerance)
    ones = torch.ones((3, code.E), device=dev)
    lp1, _ = lsim.wbp_forward(code, ones, T(L32).to(dev), 3, want_ckpt=False)
    _, lp2 = lsim.decode(code, T(L32).to(dev), lsim.params(lsim.SPA_F32, iters=3), want_bits=False,
                         want_app=True)
    ok, worst = rel_close(lp1.cpu().numpy(), lp2.cpu().numpy(), 1e-5)
    assert ok, worst


def test_wbp_checkpoints_are_the_oracles_messages():
    """Each round's checkpoint is the variable-to-check messages entering
    that round (q^(1) = lam, then q^(t+1) after the weighted round t), in
    canonical edge order and natural units, against the oracle's float64
    iteration with the same weights."""
    qb, g, L32, w, c = wbp_case()
    code = lsim.Code.from_qcbase(qb, 3840)
    _, ck = lsim.wbp_forward(code, T(w).to(dev), T(L32).to(dev), 3)
    ck = ck.cpu().numpy()
    lam = np.clip(D.channel_lam(g, L32.astype(np.float64)), -D.LLR_MAX, D.LLR_MAX)
    q = lam[:, g.edge_vn()]
    for t in range(3):
        ok, worst = rel_close(ck[t], q, 1e-4)
        print(f"checkpoint {t}: worst {worst:.2e}")
        assert ok, (t, worst)
        _, _, q = D.spa_iteration(g, lam, q, D.LLR_MAX, w=w[t].astype(np.float64))


def test_wbp_gradient_vs_autograd():
    qb, g, L32, w, c = wbp_case()
    code = lsim.Code.from_qcbase(qb, 3840)
    B, Tn = L32.shape[0], w.shape[0]
    tl, tw = T(L32).to(dev), T(w).to(dev)
    lp, ck = lsim.wbp_forward(code, tw, tl, Tn)
    tc = T(c.astype(np.uint8)).to(dev)
    gpost, loss = lsim.bce_grad(lp, tc, 1.0 / (B * g.n_dec))
    gllr, gw = lsim.wbp_backward(code, tw, tl, ck, gpost, Tn)
    Lch = np.zeros((B, g.n_dec))
    Lch[:, g.tx_lo:g.tx_lo + g.e_tx] = L32
    loss_ref, gL_ref, gw_ref, hits = wbp.grad_autograd(g, Lch, w.astype(np.float64), c.astype(np.float64))
    assert abs(loss.item() - loss_ref) <= 1e-4 * abs(loss_ref)
    for got, ref in ((gllr.cpu().numpy(), gL_ref[:, g.tx_lo:g.tx_lo + g.e_tx]), (gw.cpu().numpy(), gw_ref)):
        rel = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        cos = float((got * ref).sum() / (np.linalg.norm(got) * np.linalg.norm(ref)))
        print(f"rel {rel:.2e} cos {cos:.8f} clamp hits {hits}")
        assert rel <= 1e-3 and cos >= 0.99999


def _elementwise(got, ref, what, tol=1e-3):
    """|got - ref| <= tol * max(|ref|, 0.01 * rms(ref)) for every element;
    prints and returns the worst element's ratio."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(ref ** 2)))
    floor = np.maximum(np.abs(ref), 0.01 * rms)
    ratio = np.abs(got - ref) / np.where(floor > 0, floor, 1.0)
    i = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    print(f"{what}: worst |d|/floor {ratio[i]:.2e} at {tuple(int(x) for x in i)} "
          f"(got {got[i]:.6e}, ref {ref[i]:.6e}, rms {rms:.3e})")
    assert ratio[i] <= tol, (what, i, got[i], ref[i])
    return float(ratio[i])


@pytest.mark.parametrize("Tn,B", [(10, 2048), (20, 2048), (10, 293)])
def test_wbp_adjoint_at_the_training_launch(Tn, B):
    """The adjoint at the training step's launch (BG2 code, B = 2048, T = 10,
    and T = 20 as the bench also times; and a batch of 293, where the
    workgroups take unequal numbers of codewords): the loss gradient is
    nonzero only on a few sampled codewords, so dL/dw equals the oracle's
    float64 autograd over those codewords alone.  dL/dL_ch of the sampled
    rows and dL/dw are compared element by element; every other row's
    dL/dL_ch must be exactly zero.  Sampled rows are taken only where no
    clamped value of the oracle's forward lies within 1e-3 of the clamp
    threshold (there float32 and float64 may take different sides)."""
    qb = BG2.load()
    g = qc.graph_from_qcbase(qb, 3840)
    code = lsim.Code.from_qcbase(qb, 3840)
    m = 4
    rows = (np.array([5, 700, 1401, 2046, 333, 1999]) if B == 2048
            else np.array([5, 270, 141, 292, 33, 199]))
    ebn0 = np.array([1.0, 1.6, 2.2, 2.8, 3.4, 4.0])
    seed = 0x2203118500000590 + Tn + (0 if B == 2048 else 0x40)
    w = rand.uniform(seed + 1, (Tn, g.E), 0.7, 1.3).astype(np.float32)
    pool = [pipeline.transmit(g, qb.family, seed, int(b), 1,
                              np.array([pipeline.n0_for(g, e, m)]), m, "maxlog")
            for b, e in zip(rows, ebn0)]
    L32 = np.concatenate([t["L"] for t in pool]).astype(np.float32)
    c = np.concatenate([t["c"][:, :g.n_dec] for t in pool]).astype(np.float64)
    Lch = np.zeros((len(rows), g.n_dec))
    Lch[:, g.tx_lo:g.tx_lo + g.e_tx] = L32
    *_, margin = wbp.grad_autograd(g, Lch, w.astype(np.float64), c, want_margin=True)
    keep = margin >= 1e-3
    print("clamp margins", margin, "kept", int(keep.sum()))
    assert keep.sum() >= 3
    rows, L32, c, Lch = rows[keep], L32[keep], c[keep], Lch[keep]
    K = len(rows)
    loss_ref, gL_ref, gw_ref, hits = wbp.grad_autograd(g, Lch, w.astype(np.float64), c)
    print("clamp hits on the kept rows", hits)
    # the full batch: the sampled rows carry the oracle's LLRs, the others
    # seeded Gaussian LLRs
    full = rand.gaussian(seed + 2, (B, g.e_tx), scale=4.0).astype(np.float32)
    full[rows] = L32
    labels = np.zeros((B, g.n_dec), dtype=np.uint8)
    labels[rows] = c.astype(np.uint8)
    tl, tw = T(full).to(dev), T(w).to(dev)
    lp, ck = lsim.wbp_forward(code, tw, tl, Tn)
    gpost, _ = lsim.bce_grad(lp, T(labels).to(dev), 1.0 / (K * g.n_dec))
    mask = torch.zeros((B, 1), dtype=torch.float32, device=dev)
    mask[T(rows).to(dev)] = 1.0
    gpost = (gpost * mask).contiguous()
    gllr, gw = lsim.wbp_backward(code, tw, tl, ck, gpost, Tn)
    gllr, gw = gllr.cpu().numpy(), gw.cpu().numpy()
    # the workspace holds one partial row per resident adjoint workgroup
    # (at most B) and 32 slice rows
    parts = lsim.wbp_workspace(code, Tn, B) // (Tn * g.E * 4) - 32
    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    print("weight-gradient partial rows", parts)
    assert 1 <= parts <= B and (parts == B or parts % ncu == 0)
    other = np.ones(B, dtype=bool)
    other[rows] = False
    assert not np.any(gllr[other]), "rows with zero output gradient got a nonzero dL/dL_ch"
    _elementwise(gllr[rows], gL_ref[:, g.tx_lo:g.tx_lo + g.e_tx], f"dL/dL_ch T={Tn}")
    _elementwise(gw, gw_ref, f"dL/dw T={Tn}")
    # checkpoints on and off: the same posteriors bit for bit
    lp2, _ = lsim.wbp_forward(code, tw, tl, Tn, want_ckpt=False)
    assert torch.equal(lp, lp2)


def test_wbp_autograd_function_and_determinism():
    qb, g, L32, w, c = wbp_case(B=4, Tn=2)
    code = lsim.Code.from_qcbase(qb, 3840)
    tl = T(L32).to(dev).requires_grad_(True)
    tw = T(w).to(dev).requires_grad_(True)
    out = lsim.WBPFunction.apply(tl, tw, code, 2, 20.0)
    (out ** 2).mean().backward()
    g1 = (tl.grad.clone(), tw.grad.clone())
    tl.grad, tw.grad = None, None
    out = lsim.WBPFunction.apply(tl, tw, code, 2, 20.0)
    (out ** 2).mean().backward()
    assert torch.equal(g1[0], tl.grad) and torch.equal(g1[1], tw.grad)


def glorot(seed):
    r = rand.rng(seed)
    out = []
    for shape in ondm.SIZES:
        if len(shape) == 2:
            lim = np.sqrt(6.0 / (shape[0] + shape[1]))
            out.append(r.uniform(-lim, lim, shape).reshape(-1))
        else:
            out.append(r.uniform(-0.1, 0.1, shape))
    return np.concatenate(out)


def test_ndm_forward_backward_vs_oracle():
    params = glorot(5).astype(np.float32)
    B, S = 7, 301
    y = (rand.gaussian(6, (B, S)) + 1j * rand.gaussian(7, (B, S))).astype(np.complex64)
    n0 = rand.uniform(8, B, 0.1, 1.0).astype(np.float32)
    yy = np.stack([y.real, y.imag], -1).astype(np.float32)
    tp, ty, tn = T(params).to(dev), T(yy).to(dev), T(n0).to(dev)
    out = lsim.ndm_forward(tp, ty, tn).cpu().numpy()
    ref = ondm.forward_numpy(params.astype(np.float64), y.astype(np.complex128), n0.astype(np.float64))
    assert np.abs(out - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    gl = rand.gaussian(9, (B, S * 4)).astype(np.float32)
    gp = lsim.ndm_backward(tp, ty, tn, T(gl).to(dev)).cpu().numpy()
    gref = ondm.grad_params(params.astype(np.float64), y.astype(np.complex128), n0.astype(np.float64),
                            gl.astype(np.float64))
    rel = np.linalg.norm(gp - gref) / np.linalg.norm(gref)
    assert rel <= 1e-5, rel
    _check_groups(gp, gref, 1e-5)
    _elementwise(gp, gref, "NDM dL/dparams", tol=1e-4)


def _check_groups(gp, gref, tol):
    """Relative error per parameter group (W1, b1, W2, b2, W3, b3)."""
    o, errs = 0, []
    for shape in ondm.SIZES:
        n = int(np.prod(shape))
        a, b = gp[o:o + n], gref[o:o + n]
        errs.append((shape, float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))))
        o += n
    print("relative error per group", errs)
    for shape, rel in errs:
        assert rel <= tol, (shape, rel, errs)


def test_ndm_full_size():
    """The training step's demapper shape (2048 codewords x 960 16-QAM
    symbols, the launch bench.py times): sampled forward outputs and the
    full parameter gradient, per group, against the oracle."""
    params = glorot(21).astype(np.float32)
    B, S = 2048, 960
    y = (rand.gaussian(22, (B, S)) + 1j * rand.gaussian(23, (B, S))).astype(np.complex64)
    n0 = rand.uniform(24, B, 0.05, 1.0).astype(np.float32)
    yy = np.stack([y.real, y.imag], -1).astype(np.float32)
    tp, ty, tn = T(params).to(dev), T(yy).to(dev), T(n0).to(dev)
    out = lsim.ndm_forward(tp, ty, tn).cpu().numpy()
    rows = np.array([0, 1, 777, 1500, 2047])
    ref = ondm.forward_numpy(params.astype(np.float64), y[rows].astype(np.complex128),
                             n0[rows].astype(np.float64))
    assert np.abs(out[rows] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    gl = (rand.gaussian(25, (B, S * 4)) * 1e-3).astype(np.float32)
    # A ReLU has no derivative at its kink, and a pre-activation within
    # rounding of zero may fall on either side in float32 and float64 (one
    # such symbol moves a bias gradient by ~1e-4 here).  Symbols with a
    # hidden pre-activation within 1e-6 of zero get no output gradient, so
    # both sides agree on every mask that matters.
    W1, b1, W2, b2 = [a.astype(np.float64) for a in ondm.unpack(params)[:4]]
    x = np.stack([y.real, y.imag, np.broadcast_to(np.log(n0.astype(np.float64))[:, None], y.shape)],
                 -1).reshape(-1, 3).astype(np.float64)
    a1 = x @ W1.T + b1
    a2 = np.maximum(a1, 0) @ W2.T + b2
    near = ((np.abs(a1) < 1e-6).any(1) | (np.abs(a2) < 1e-6).any(1)).reshape(B, S)
    del x, a1, a2
    gl.reshape(B, S, 4)[near] = 0.0
    gp = lsim.ndm_backward(tp, ty, tn, T(gl).to(dev)).cpu().numpy()
    gref = ondm.grad_params(params.astype(np.float64), y.astype(np.complex128),
                            n0.astype(np.float64), gl.astype(np.float64))
    print("symbols next to a kink:", int(near.sum()))
    _check_groups(gp, gref, 1e-5)
    _elementwise(gp, gref, "NDM dL/dparams, full size", tol=1e-3)


def test_bce_and_adam():
    L = rand.gaussian(10, (6, 100), scale=4.0).astype(np.float32)
    c = rand.bits(11, (6, 120))
    g, loss = lsim.bce_grad(T(L).to(dev), T(c).to(dev), 0.01)
    cc = c[:, :100].astype(np.float64)
    L64 = L.astype(np.float64)
    assert np.allclose(g.cpu().numpy(), 0.01 * (1 / (1 + np.exp(-L64)) - cc), atol=1e-7)
    assert abs(loss.item() - 0.01 * float(np.sum(np.logaddexp(0, L64) - cc * L64))) < 1e-5
    p = rand.gaussian(12, 1000).astype(np.float32)
    gr = rand.gaussian(13, 1000).astype(np.float32)
    tp, tg = T(p.copy()).to(dev), T(gr).to(dev)
    tm, tv = torch.zeros_like(tp), torch.zeros_like(tp)
    m = np.zeros(1000)
    v = np.zeros(1000)
    pp = p.astype(np.float64)
    for step in (1, 2, 3):
        lsim.adam_step(tp, tg, tm, tv, step, lr=1e-2)
        m = 0.9 * m + 0.1 * gr
        v = 0.999 * v + 0.001 * gr.astype(np.float64) ** 2
        pp -= 1e-2 * (m / (1 - 0.9 ** step)) / (np.sqrt(v / (1 - 0.999 ** step)) + 1e-8)
    assert np.allclose(tp.cpu().numpy(), pp, atol=1e-5)


def test_autotuner_mixed_and_decode(tmp_path):
    """The autotuner times only result-invariant knobs: its choice decodes
    to the default plan's bits, the choice is cached and read back."""
    from paper_2203_11854_amd import autotune
    specs = mixed_specs()[:4]
    counts = [5, 3, 4, 2]
    p = lsim.params(lsim.NMS_F32, iters=5)
    codes, parts = [], []
    for s, ((spec, e_tx), cnt) in enumerate(zip(specs, counts)):
        code = lsim.Code.from_qcbase(spec.load(), e_tx)
        codes.append(code)
        parts.append(rand.gaussian(700 + s, (cnt, e_tx), scale=3.0).astype(np.float32))
    cat = T(np.concatenate([x.reshape(-1) for x in parts])).to(dev)
    cache = str(tmp_path / "tune.json")
    best = autotune.tune_mixed(codes, counts, p, cat, cache_path=cache)
    assert set(best) >= {"threads", "codewords_per_tile", "persistent", "ms"}
    again = autotune.tune_mixed(codes, counts, p, cat, cache_path=cache)
    assert again == best
    ref = torch.zeros(sum(c.k * n for c, n in zip(codes, counts)), dtype=torch.uint8, device=dev)
    lsim.MixedPlan(codes, counts, p).decode(cat, bits=ref)
    tuned = torch.zeros_like(ref)
    plan = lsim.MixedPlan(codes, counts, p, codewords_per_tile=best["codewords_per_tile"],
                          threads=best["threads"])
    plan.decode(cat, bits=tuned, persistent=best["persistent"])
    assert torch.equal(ref, tuned)
    qb = BG2.load()
    code = lsim.Code.from_qcbase(qb, 3840)
    llr = T(rand.gaussian(710, (16, 3840), scale=3.0).astype(np.float32)).to(dev)
    for algo in (lsim.SPA_F32, lsim.NMS_F32):
        bd = autotune.tune_decode(code, llr, lsim.params(algo), cache_path=cache)
        assert bd["threads"] in (256, 384, 512, 768, 1024)


def test_schedule_tuner():
    """Result-changing knobs of the mixed batch: a shape moves from
    natural-order layered NMS to the grouped layer order or to flooding
    int8 offset min-sum only when its block error rate lies inside the
    default's Wilson 95% interval on the same data, and the scheduled
    launches give, shape by shape, exactly the bits of the decoders (and
    layer orders) the schedule names.  A schedule with every shape on NMS is
    the mixed plan."""
    from paper_2203_11854_amd import autotune
    counts = [40, 24, 30, 12, 10, 8, 16, 6]
    codes, llrs, graphs, qbs = mixed_inputs(counts, seed=131)
    parts, us = [], []
    for s, (code, L, g, qb) in enumerate(zip(codes, llrs, graphs, qbs)):
        parts.append(T(L).to(dev))
    # the transmitted bits of mixed_inputs' codewords, from the oracle's link
    for s, (g, qb) in enumerate(zip(graphs, qbs)):
        from oracle import philox
        us.append(T(philox.source_bits(131 + 100 + s, 0, counts[s], g.k)).to(dev))
    pn = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
    res = autotune.tune_schedule(codes, counts, parts, us, pn)
    po = lsim.params(lsim.OMS_I8, iters=20, offset=1, sat=31)
    for s, info in enumerate(res["shapes"]):
        lo, hi = info["nms_ci95"]
        if res["schedule"][s] == "oms":
            assert info["oms_fits"] and info["oms_accepted"]
            assert lo - 1e-9 <= info["oms_block_errors"] / counts[s] <= hi + 1e-9
        if res["layer_order"][s] == "grouped":
            assert res["schedule"][s] == "nms" and info["grouped_accepted"]
            assert lo - 1e-9 <= info["grouped_block_errors"] / counts[s] <= hi + 1e-9
        assert info["grouped_barriers"] <= info["natural_barriers"]
        assert codes[s].layer_order()[0] == (list(range(codes[s].rows))
                                             if res["layer_order"][s] == "natural" else
                                             codes[s].layer_order()[0])
    assert res["lds_rows"] in (0, -1)
    # the tuned orders stay set on the codes; then natural order everywhere
    for schedule, orders in ((res["schedule"], res["layer_order"]),
                             (["nms"] * len(codes), ["grouped"] * len(codes)),
                             (["nms"] * len(codes), ["natural"] * len(codes)),
                             (["oms" if autotune.oms_fits(c) else "nms" for c in codes],
                              ["natural"] * len(codes))):
        for code, o in zip(codes, orders):
            code.set_layer_order(o)
        sm = autotune.ScheduledMixed(codes, counts, schedule,
                                     lsim.params(lsim.NMS_F32, iters=20, alpha=0.75,
                                                 lds_rows=res["lds_rows"]), po)
        io = sm.inputs(parts)
        sm.decode(io)
        got = sm.bits(io)
        for s, (code, x) in enumerate(zip(codes, parts)):
            if schedule[s] == "oms":
                ref, _ = lsim.decode(code, lsim.quantize(x), po)
            else:
                ref, _ = lsim.decode(code, x, pn)
            assert torch.equal(got[s], ref), (schedule, orders, s)
    for code in codes:
        code.set_layer_order("natural")


def test_layer_order_tuner():
    """One code's layer order: grouped is taken only when its block error
    rate lies inside the natural order's Wilson 95% interval on the same
    frames and it decodes faster; the chosen order is left set on the code,
    and decoding with it equals the oracle in that order."""
    from paper_2203_11854_amd import autotune
    from inputs.workloads import BG2
    qb = BG2.load()
    g = qc.graph_from_qcbase(qb, 3840)
    code = lsim.Code.from_qcbase(qb, 3840)
    B = 512
    n0 = pipeline.n0_for(g, np.full(B, 3.0), 4)
    tx = pipeline.transmit(g, qb.family, 141, 0, B, n0, 4, "maxlog")
    L = tx["L"].astype(np.float32)
    x, u = T(L).to(dev), T(tx["u"]).to(dev)
    pn = lsim.params(lsim.NMS_F32, iters=20, alpha=0.75)
    res = autotune.tune_layer_order(code, x, u, pn)
    lo, hi = res["natural_ci95"]
    inside = lo - 1e-9 <= res["grouped"]["block_errors"] / B <= hi + 1e-9
    assert res["grouped_accepted"] == inside
    if res["chosen"] == "grouped":
        assert inside and res["grouped"]["ms"] < res["natural"]["ms"]
    assert res["grouped"]["barriers_per_iteration"] <= res["natural"]["barriers_per_iteration"]
    order = code.layer_order()[0]
    assert order == (D.grouped_order(g) if res["chosen"] == "grouped" else list(range(g.rows)))
    rows = [0, 1, B - 1]
    lam = D.channel_lam(g, L[rows], dtype=np.float32)
    ref = D.nms_layered(g, lam, 20, 0.75, mode="fp32", order=order)
    _, lp = lsim.decode(code, x[rows].contiguous(), pn, want_app=True)
    assert np.array_equal(lp.cpu().numpy(), -ref)
    code.set_layer_order("natural")
