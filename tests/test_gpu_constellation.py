"""GPU parity of the trainable constellation (mapper with a point table, its
adjoint, the demapper's input gradient and the whole training step) against
the oracle."""
import numpy as np
import pytest
import torch

from helpers import CODES
from inputs import rand
from oracle import constellation as oc
from oracle import modem, ndm, philox, qc

pytestmark = pytest.mark.gpu

lsim = pytest.importorskip("paper_2203_11854_amd")
dev = "cuda"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x))


def code_for(name):
    spec, e_tx, _ = CODES[name]
    qb = spec.load()
    return qb, lsim.Code.from_qcbase(qb, e_tx)


def glorot(seed):
    r = rand.rng(seed)
    out = []
    for fo, fi in ((64, 3), (64, 64), (4, 64)):
        lim = np.sqrt(6.0 / (fi + fo))
        out.append(r.uniform(-lim, lim, fo * fi))
        out.append(np.zeros(fo))
    return np.concatenate(out)


def coded(name, B, seed, cw0):
    qb, code = code_for(name)
    u = philox.source_bits(seed, cw0, B, qb.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    g = qc.graph_from_qcbase(qb, code.e_tx)
    return code, c, c[:, g.tx_lo:g.tx_lo + g.e_tx]


def near_kink(params, y, n0, tol=1e-6):
    """Symbols with a hidden pre-activation within tol of zero: there the
    ReLU mask may differ between float32 and float64."""
    W1, b1, W2, b2 = [a.astype(np.float64) for a in ndm.unpack(params)[:4]]
    B, S = y.shape
    x = np.stack([y.real, y.imag, np.broadcast_to(np.log(n0.astype(np.float64))[:, None], y.shape)],
                 -1).reshape(-1, 3)
    a1 = x @ W1.T + b1
    a2 = np.maximum(a1, 0) @ W2.T + b2
    return ((np.abs(a1) < tol).any(1) | (np.abs(a2) < tol).any(1)).reshape(B, S)


@pytest.mark.parametrize("name,m", [("small", 1), ("bg2", 2), ("bg2", 4), ("bg1", 6), ("small", 3)])
def test_map_points_vs_oracle(name, m):
    B, seed, cw0 = 7, 77, 5
    code, c, t = coded(name, B, seed, cw0)
    if code.e_tx % m:
        pytest.skip("e_tx not a multiple of m")
    K = 1 << m
    p = rand.gaussian(31 + m, (K, 2)).astype(np.float32)
    n0 = rand.uniform(32, B, 0.1, 1.5).astype(np.float32)
    y = lsim.map_points(code, m, T(p).to(dev), T(c).to(dev), T(n0).to(dev), seed, cw0).cpu().numpy()
    x = oc.map_points(p.astype(np.float64), t, m)
    ref = modem.awgn(x, n0.astype(np.float64), philox.normals(seed, cw0, B, x.shape[1]))
    got = y[..., 0] + 1j * y[..., 1]
    sig = np.sqrt(n0[:, None] / 2.0)
    # 1e-5 on the unit normals (as for the Gray mapper) plus a few float32
    # ulps on the normalised point
    err = np.abs(got - ref)
    assert (err <= 1e-5 * sig + 4e-7 * np.abs(x).max()).all(), float((err / sig).max())


@pytest.mark.parametrize("m", [2, 4, 6])
def test_map_points_with_qam_is_the_gray_mapper(m):
    B, seed, cw0 = 5, 78, 0
    code, c, _ = coded("bg2" if m != 6 else "bg1", B, seed, cw0)
    n0 = rand.uniform(33, B, 0.1, 1.0).astype(np.float32)
    tc, tn = T(c).to(dev), T(n0).to(dev)
    pts = T(oc.qam_points(m).astype(np.float32)).to(dev)
    a = lsim.map_points(code, m, pts, tc, tn, seed, cw0)
    b = lsim.map_awgn(code, m, tc, tn, seed, cw0)
    assert (a - b).abs().max().item() <= 4e-7


def test_ndm_input_gradient_vs_oracle():
    params = glorot(41).astype(np.float32)
    B, S = 7, 301
    y = (rand.gaussian(42, (B, S)) + 1j * rand.gaussian(43, (B, S))).astype(np.complex64)
    n0 = rand.uniform(44, B, 0.1, 1.0).astype(np.float32)
    gl = rand.gaussian(45, (B, S * 4)).astype(np.float32)
    near = near_kink(params, y, n0)
    gl.reshape(B, S, 4)[near] = 0.0
    yy = np.stack([y.real, y.imag], -1).astype(np.float32)
    tp, ty, tn, tg = (T(a).to(dev) for a in (params, yy, n0, gl))
    gp, gy = lsim.ndm_backward(tp, ty, tn, tg, gy=True)
    gp_only = lsim.ndm_backward(tp, ty, tn, tg)
    # asking for dy changes nothing in dparams
    assert torch.equal(gp, gp_only)
    ref = oc.ndm_input_vjp(params.astype(np.float64), y.astype(np.complex128),
                           n0.astype(np.float64), gl.astype(np.float64))
    got = gy.cpu().numpy()
    # each entry is a 64-term contraction of float32 products
    assert np.abs(got - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


def _points_tol(p, t, m, gy):
    """Per-entry bound for dL/dp: fixed-order float32 sums of depth d over the
    label's upstream terms, plus the radial term over all of them."""
    K = 1 << m
    x = oc.normalize(p.astype(np.float64))
    s = np.sqrt((p.astype(np.float64) ** 2).sum() / K)
    lab = oc.labels_of(t, m).reshape(-1)
    a = np.abs(gy.astype(np.float64)).reshape(-1, 2)
    per = np.zeros((K, 2))
    np.add.at(per, lab, a)
    n = lab.size
    depth = n / 65536 + 64 + 1024 + 16 + 8
    u = 2.0 ** -24
    return depth * u * (per + np.abs(x) * a.sum() / K) / s + 1e-30


@pytest.mark.parametrize("name,m,B", [("bg2", 4, 9), ("small", 1, 13), ("bg1", 6, 3), ("bg2", 2, 1)])
def test_points_grad_vs_oracle(name, m, B):
    code, c, t = coded(name, B, 79, 0)
    K = 1 << m
    p = (oc.qam_points(m) + rand.gaussian(50 + m, (K, 2), scale=0.2)).astype(np.float32)
    S = code.e_tx // m
    gy = rand.gaussian(51, (B, S, 2)).astype(np.float32)
    tp = T(p).to(dev)
    got = lsim.points_grad(code, m, tp, T(c).to(dev), T(gy).to(dev)).cpu().numpy()
    ref = oc.points_vjp(p.astype(np.float64), t, m, gy.astype(np.float64))
    tol = _points_tol(p, t, m, gy)
    assert (np.abs(got - ref) <= tol).all(), float((np.abs(got - ref) / tol).max())
    again = lsim.points_grad(code, m, tp, T(c).to(dev), T(gy).to(dev)).cpu().numpy()
    assert np.array_equal(got, again)


def _gpu_step(code, m, pts, params, c, no, seed, cw0, drop=None):
    """One end-to-end step: forward loss and the two gradients (no upstream
    gradient from the symbols where ``drop`` is True)."""
    B = c.shape[0]
    y = lsim.map_points(code, m, pts, c, no, seed, cw0)
    llr = lsim.ndm_forward(params, y, no)
    scale = 1.0 / (B * code.e_tx)
    g, loss = lsim.bce_grad(llr, c[:, code.tx_lo:], scale)
    if drop is not None:
        g.view(B, -1, m)[torch.from_numpy(drop).to(g.device)] = 0.0
    gp, gy = lsim.ndm_backward(params, y, no, g, gy=True)
    gpts = lsim.points_grad(code, m, pts, c, gy)
    return loss, gpts, gp


def test_training_step_vs_oracle():
    """Loss, dL/dpoints and dL/dparams of one step through map_points,
    ndm_forward, bce_grad, ndm_backward and points_grad against float64
    autograd on the same noise."""
    m, B, seed, cw0 = 4, 4, 80, 3
    code, c, t = coded("bg2", B, seed, cw0)
    S = code.e_tx // m
    params = glorot(81).astype(np.float32)
    p = (oc.qam_points(m) + rand.gaussian(82, (16, 2), scale=0.1)).astype(np.float32)
    n0 = rand.uniform(83, B, 0.2, 0.8).astype(np.float32)
    g = philox.normals(seed, cw0, B, S)
    y64 = oc.map_points(p.astype(np.float64), t, m) + np.sqrt(n0[:, None] / 2.0) * g
    # symbols next to a ReLU kink pass no gradient on either side
    near = near_kink(params, y64, n0, 1e-5)
    loss, gpts, gp = _gpu_step(code, m, T(p).to(dev), T(params).to(dev), T(c).to(dev),
                               T(n0).to(dev), seed, cw0, drop=near)
    rl, rp, rw = oc.loss_and_grads(p.astype(np.float64), params.astype(np.float64), t, m,
                                   n0.astype(np.float64), g, keep=~near)
    print("symbols next to a kink:", int(near.sum()))
    assert abs(loss.item() - rl) <= 1e-5 * abs(rl)
    assert np.linalg.norm(gpts.cpu().numpy() - rp) <= 1e-4 * np.linalg.norm(rp)
    assert np.linalg.norm(gp.cpu().numpy() - rw) <= 1e-4 * np.linalg.norm(rw)


def test_full_size_step():
    """The benchmark's shape (2048 codewords, 960 16-QAM symbols each):
    sampled rows of the mapper and of dL/dy, and dL/dpoints from the
    device's dL/dy against the oracle's adjoint over all symbols."""
    m, B, seed, cw0 = 4, 2048, 84, 0
    qb, code = code_for("bg2")
    u = lsim.source_bits(seed, cw0, B, qb.k, dev)
    c = lsim.encode(code, u)
    S = code.e_tx // m
    params = glorot(85).astype(np.float32)
    p = (oc.qam_points(m) + rand.gaussian(86, (16, 2), scale=0.1)).astype(np.float32)
    n0 = rand.uniform(87, B, 0.1, 1.0).astype(np.float32)
    tp, tw, tn = T(p).to(dev), T(params).to(dev), T(n0).to(dev)
    y = lsim.map_points(code, m, tp, c, tn, seed, cw0)
    rows = np.array([0, 1, 1023, 2047])
    ch = c.cpu().numpy()
    t = ch[:, code.tx_lo:code.tx_lo + code.e_tx]
    x = oc.map_points(p.astype(np.float64), t[rows], m)
    ref = x + np.sqrt(n0[rows, None] / 2.0) * philox.normals(seed, cw0, B, S)[rows]
    yh = y.cpu().numpy()
    got = yh[rows, :, 0] + 1j * yh[rows, :, 1]
    assert (np.abs(got - ref) <= 1e-5 * np.sqrt(n0[rows, None] / 2.0) + 4e-7 * np.abs(x).max()).all()
    gl = (rand.gaussian(88, (B, S * 4)) * 1e-3).astype(np.float32)
    yc = (yh[..., 0] + 1j * yh[..., 1])
    ri, si = near_kink(params, yc[rows], n0[rows]).nonzero()
    gl.reshape(B, S, 4)[rows[ri], si] = 0.0
    _, gy = lsim.ndm_backward(tw, y, tn, T(gl).to(dev), gy=True)
    gyh = gy.cpu().numpy()
    ref_gy = oc.ndm_input_vjp(params.astype(np.float64), yc[rows].astype(np.complex128),
                              n0[rows].astype(np.float64), gl[rows].astype(np.float64))
    assert np.abs(gyh[rows] - ref_gy).max() <= 1e-5 * max(1.0, np.abs(ref_gy).max())
    gpts = lsim.points_grad(code, m, tp, c, gy).cpu().numpy()
    ref_p = oc.points_vjp(p.astype(np.float64), t, m, gyh.astype(np.float64))
    tol = _points_tol(p, t, m, gyh)
    assert (np.abs(gpts - ref_p) <= tol).all(), float((np.abs(gpts - ref_p) / tol).max())


def test_training_lowers_the_loss():
    """150 Adam steps on points and demapper from 16-QAM and a random
    demapper at Eb/N0 ~ U[2, 6] dB: the BCE falls and the points keep unit
    energy after normalisation."""
    m, B = 4, 256
    qb, code = code_for("bg2")
    r = rand.rng(90)
    no = torch.tensor(lsim.ebn0_to_n0(r.uniform(2.0, 6.0, B), code.k / code.e_tx, m),
                      dtype=torch.float32, device=dev)
    pts = T(oc.qam_points(m).astype(np.float32)).to(dev)
    params = T(glorot(91).astype(np.float32)).to(dev)
    pm, pv = torch.zeros_like(pts), torch.zeros_like(pts)
    wm, wv = torch.zeros_like(params), torch.zeros_like(params)
    losses = []
    for step in range(1, 151):
        u = lsim.source_bits(92, step * B, B, qb.k, dev)
        c = lsim.encode(code, u)
        loss, gpts, gp = _gpu_step(code, m, pts, params, c, no, 92, step * B)
        losses.append(loss.item())
        lsim.adam_step(pts, gpts, pm, pv, step, lr=1e-2)
        lsim.adam_step(params, gp, wm, wv, step, lr=1e-2)
    first, last = np.mean(losses[:5]), np.mean(losses[-5:])
    print("loss", first, "->", last)
    assert np.isfinite(losses).all()
    # float32 torch on the CPU with the same shapes goes from 0.63 to 0.35
    assert last < 0.75 * first
    assert torch.isfinite(pts).all()
