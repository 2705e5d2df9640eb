"""GPU parity of the demapper with prior, the a-priori LLR source, the
mutual-information estimate, the decoder extrinsic output, an EXIT
measurement and iterative demapping and decoding against the oracle."""
import numpy as np
import pytest
import torch

from helpers import CODES, graph
from inputs import rand
from oracle import decoders, modem, philox, qc
from oracle import exit as ox

pytestmark = pytest.mark.gpu

lsim = pytest.importorskip("paper_2203_11854_amd")
dev = "cuda"


def T(x):
    return torch.from_numpy(np.ascontiguousarray(x))


def code_for(name):
    spec, e_tx, _ = CODES[name]
    qb = spec.load()
    return qb, lsim.Code.from_qcbase(qb, e_tx)


def _method(method):
    return "exact" if method == lsim.DEMAP_EXACT else "maxlog"


@pytest.mark.parametrize("m", [1, 2, 4, 6])
@pytest.mark.parametrize("method", [lsim.DEMAP_EXACT, lsim.DEMAP_MAXLOG])
@pytest.mark.parametrize("extrinsic", [True, False])
def test_demap_prior_vs_oracle(m, method, extrinsic):
    B, S = 11, 203
    y = (1.3 * (rand.gaussian(m, (B, S)) + 1j * rand.gaussian(m + 10, (B, S)))).astype(np.complex64)
    n0 = rand.uniform(m + 20, B, 0.05, 2.0).astype(np.float32)
    la = rand.gaussian(m + 30, (B, S * m), scale=4.0).astype(np.float32)
    yy = np.stack([y.real, y.imag], axis=-1).astype(np.float32)
    L = lsim.demap_prior(m, method, T(yy).to(dev), T(n0).to(dev), T(la).to(dev),
                         extrinsic=extrinsic).cpu().numpy()
    y64, n64, la64 = y.astype(np.complex128), n0.astype(np.float64), la.astype(np.float64)
    ref = modem.demap_prior_bruteforce(y64, n64, m, _method(method), la64, extrinsic=extrinsic)
    # FP32 rounding of the squared distances and of the prior sums
    scale = (np.abs(y64) + 2.0) ** 2 / n64[:, None]
    pri = np.abs(la64).reshape(B, S, m).sum(-1)
    tol = (1e-5 * np.maximum(1.0, np.abs(ref))
           + 2e-6 * np.repeat(scale + pri, m, axis=1))
    assert (np.abs(L - ref) <= tol).all(), float((np.abs(L - ref) / tol).max())


@pytest.mark.parametrize("m", [2, 4])
def test_demap_prior_zero_prior_is_demap(m):
    B, S = 5, 100
    y = (rand.gaussian(40, (B, S, 2))).astype(np.float32)
    n0 = rand.uniform(41, B, 0.1, 1.0).astype(np.float32)
    ty, tn = T(y).to(dev), T(n0).to(dev)
    z = torch.zeros((B, S * m), dtype=torch.float32, device=dev)
    a = lsim.demap_prior(m, lsim.DEMAP_MAXLOG, ty, tn, z)
    b = lsim.demap(m, lsim.DEMAP_MAXLOG, ty, tn)
    # max-log: the same minimum differences, with and without the prior
    assert (a - b).abs().max().item() <= 1e-5 * max(1.0, b.abs().max().item())


@pytest.mark.parametrize("name", ["small", "bg2"])
def test_apriori_llrs_vs_oracle(name):
    qb, code = code_for(name)
    g = qc.graph_from_qcbase(qb, code.e_tx)
    B, seed, cw0 = 6, 91, 2 ** 32 + 3
    u = philox.source_bits(seed, cw0, B, qb.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    t = c[:, g.tx_lo:g.tx_lo + g.e_tx]
    sigma = rand.uniform(92, B, 0.0, 6.0).astype(np.float32)
    la = lsim.apriori_llrs(code, T(c).to(dev), T(sigma).to(dev), seed, cw0).cpu().numpy()
    s64 = sigma.astype(np.float64)
    nrm = philox.normals_real(seed, cw0, B, g.e_tx, 2)
    ref = ox.apriori_llrs(t, s64, nrm)
    # 1e-5 on the unit normals (as for the channel noise) times sigma, plus
    # float32 rounding of the mean
    tol = 1e-5 * s64[:, None] + 1e-6 * np.abs(ref) + 1e-7
    assert (np.abs(la - ref) <= tol).all(), float((np.abs(la - ref) / tol).max())


def test_apriori_llrs_ragged_tail():
    """A transmitted length that is not a multiple of 4: the last Philox
    block is used in part."""
    spec, _, _ = CODES["small"]
    qb = spec.load()
    e_tx = 646
    code = lsim.Code.from_qcbase(qb, e_tx)
    g = qc.graph_from_qcbase(qb, e_tx)
    B, seed = 3, 93
    u = philox.source_bits(seed, 0, B, qb.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    t = c[:, g.tx_lo:g.tx_lo + g.e_tx]
    sigma = np.array([0.5, 2.0, 5.0], np.float32)
    la = lsim.apriori_llrs(code, T(c).to(dev), T(sigma).to(dev), seed, 0).cpu().numpy()
    ref = ox.apriori_llrs(t, sigma.astype(np.float64), philox.normals_real(seed, 0, B, e_tx, 2))
    assert la.shape == (B, e_tx)
    assert (np.abs(la - ref) <= 1e-5 * sigma[:, None] + 1e-6 * np.abs(ref) + 1e-7).all()


@pytest.mark.parametrize("B,n", [(1, 1), (5, 63), (3, 3841)])
def test_mutual_info_ragged(B, n):
    c = rand.bits(95 + n, (B, n))
    L = rand.gaussian(96 + n, (B, n), scale=4.0).astype(np.float32)
    mi_cw, mi_b = lsim.mutual_info(T(L).to(dev), T(c).to(dev))
    ref = ox.mutual_info(L.astype(np.float64), c)
    assert np.abs(mi_cw.cpu().numpy() - ref).max() <= 2e-6
    assert abs(mi_b.item() - ref.mean()) <= 2e-6


def test_mutual_info_vs_oracle_and_bins():
    B, n = 37, 3840
    c = rand.bits(93, (B, n + 256))
    L = (rand.gaussian(94, (B, n), scale=3.0) + (2.0 * c[:, :n] - 1.0) * 2.0).astype(np.float32)
    bins = (np.arange(B) % 5).astype(np.int32)
    bins[3] = 9                                     # outside [0, 5): left out
    mi_cw, mi_b = lsim.mutual_info(T(L).to(dev), T(c).to(dev)[:, :n], T(bins).to(dev), 5)
    ref = ox.mutual_info(L.astype(np.float64), c[:, :n])
    # fixed-order float32 sums of n terms <= 1 (plus log1p/exp rounding)
    assert np.abs(mi_cw.cpu().numpy() - ref).max() <= 2e-6
    mb = mi_b.cpu().numpy()
    for k in range(5):
        sel = bins == k
        assert abs(mb[k] - ref[sel].mean()) <= 2e-6
    again = lsim.mutual_info(T(L).to(dev), T(c).to(dev)[:, :n], T(bins).to(dev), 5)[1]
    assert torch.equal(mi_b, again)


def test_extrinsic_vs_definition():
    qb, code = code_for("bg2")
    B = 4
    app = rand.gaussian(95, (B, code.n_dec), scale=5.0).astype(np.float32)
    lin = rand.gaussian(96, (B, code.e_tx), scale=5.0).astype(np.float32)
    lo = code.tx_lo
    hi = min(lo + code.e_tx, code.n_dec)
    for llr_max in (0.0, 7.5):
        out = lsim.extrinsic(code, T(app).to(dev), T(lin).to(dev), llr_max).cpu().numpy()
        x = lin if llr_max == 0 else np.clip(lin, -llr_max, llr_max)
        ref = np.zeros((B, code.e_tx), np.float32)
        ref[:, :hi - lo] = app[:, lo:hi] - x[:, :hi - lo]
        assert np.array_equal(out, ref)


def test_decoder_exit_point_vs_oracle():
    """One point of the decoder's EXIT curve on the small code: a-priori
    LLRs in, 5 sum-product iterations, extrinsic out, mutual information;
    per codeword against the oracle's float64 chain on the same LLRs (few
    iterations, so that float32 and float64 decoding of frames that do not
    converge stay close)."""
    qb, code = code_for("small")
    g = qc.graph_from_qcbase(qb, code.e_tx)
    B, seed = 24, 97
    u = philox.source_bits(seed, 0, B, qb.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    t = c[:, g.tx_lo:g.tx_lo + g.e_tx]
    sigma = np.full(B, ox.J_inv(0.5), np.float32)
    tc = T(c).to(dev)
    la = lsim.apriori_llrs(code, tc, T(sigma).to(dev), seed, 0)
    p = lsim.params(lsim.SPA_F32, iters=5)
    _, app = lsim.decode(code, la, p, want_bits=False, want_app=True)
    le = lsim.extrinsic(code, app, la)
    mi_cw, mi = lsim.mutual_info(le, tc[:, code.tx_lo:])
    la64 = la.cpu().numpy().astype(np.float64)
    app_ref = decoders.spa_flood(g, decoders.channel_lam(g, la64), 5)
    le_ref = ox.decoder_extrinsic(g, app_ref, la64)
    ref = ox.mutual_info(le_ref, t)
    # the decoder matches the oracle within 1e-4 relative per round; the
    # MI estimate (mean over 648 bits of a 1-Lipschitz function of L / ln 2)
    # moves by less than that
    assert np.abs(mi_cw.cpu().numpy() - ref).max() <= 5e-4
    print("I_A 0.5 -> I_E", float(mi.item()), float(ref.mean()))


def test_bicm_id_two_passes_vs_oracle():
    """Iterative demapping and decoding on the small code with Gray 16-QAM:
    every demapper pass and the final posteriors against the oracle's loop."""
    qb, code = code_for("small")
    g = qc.graph_from_qcbase(qb, code.e_tx)
    B, m, seed = 8, 4, 98
    n0 = np.full(B, float(modem.ebn0_to_n0(4.0, qb.k / code.e_tx, m)), np.float32)
    u = lsim.source_bits(seed, 0, B, qb.k, dev)
    c = lsim.encode(code, u)
    tn = T(n0).to(dev)
    y = lsim.map_awgn(code, m, c, tn, seed, 0)
    p = lsim.params(lsim.SPA_F32, iters=10)
    prior = torch.zeros((B, code.e_tx), dtype=torch.float32, device=dev)
    got = []
    for _ in range(2):
        le = lsim.demap_prior(m, lsim.DEMAP_EXACT, y, tn, prior)
        got.append(le.cpu().numpy())
        _, app = lsim.decode(code, le, p, want_bits=False, want_app=True)
        prior = lsim.extrinsic(code, app, le)
    y64 = y.cpu().numpy().astype(np.float64)
    y64 = y64[..., 0] + 1j * y64[..., 1]
    app_ref, passes = ox.bicm_id(g, y64, n0.astype(np.float64), m, "exact", outer=2, iters=10)
    for a, b in zip(got, passes):
        err = np.abs(a - b) / np.maximum(1.0, np.abs(b))
        assert err.max() <= 1e-3, err.max()
    post = -app_ref
    a = app.cpu().numpy()
    agree = np.sign(a) == np.sign(post)
    assert agree.mean() > 0.999
