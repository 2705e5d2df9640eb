"""Pins of the demapper with prior, the EXIT-chart pieces and iterative
demapping and decoding in the oracle.

* Demapper with prior: zero prior is the plain demapper; BPSK and Gray QPSK
  in closed form (the prior adds to the channel LLR); with near-certain
  priors on the other bits the extrinsic LLR is the two-point LLR between
  the neighbours that differ in the bit; the extrinsic part does not depend
  on the bit's own prior.
* J: J(0) = 0, J(2/s) equals the BI-AWGN capacity computed from the
  differential entropy of the channel output, J_inv inverts J.
* Mutual information estimate: Monte-Carlo consistent LLRs give J(sigma)
  within the sampling error; perfect and empty LLRs give 1 and 0.
* Decoder extrinsic on a tree code equals the brute-force MAP extrinsic.
* BICM-ID with Gray QPSK: the demapper's extrinsic ignores the prior, so
  every pass equals the first.
* Real normals of stream 1 are the complex channel normals, interleaved.
"""
import numpy as np
import pytest
from scipy.integrate import quad

from helpers import CODES, graph
from inputs import rand
from oracle import exit as ox
from oracle import modem, philox, qc
from test_oracle_decoders import map_llr, tiny_graph


def _y(seed, B, S, scale=1.0):
    return rand.gaussian(seed, (B, S), scale=scale) + 1j * rand.gaussian(seed + 1, (B, S), scale=scale)


@pytest.mark.parametrize("m", [1, 2, 4, 6])
@pytest.mark.parametrize("method", ["exact", "maxlog"])
def test_zero_prior_is_plain_demapper(m, method):
    B, S = 3, 11
    y = _y(1, B, S)
    n0 = np.array([0.3, 0.8, 1.5])
    got = modem.demap_prior_bruteforce(y, n0, m, method, np.zeros((B, S * m)))
    ref = modem.demap_bpsk(y, n0) if m == 1 else modem.demap_bruteforce(y, n0, m, method)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("method", ["exact", "maxlog"])
def test_bpsk_and_qpsk_prior_adds(method):
    B, S = 2, 9
    y = _y(3, B, S)
    n0 = np.array([0.5, 1.1])
    La = rand.gaussian(4, (B, S), scale=3.0)
    got = modem.demap_prior_bruteforce(y, n0, 1, method, La)
    assert np.allclose(got, -4.0 * y.real / n0[:, None] + La, rtol=1e-12, atol=1e-12)
    # Gray QPSK: one bit per axis, x = ((1-2c0) + j(1-2c1))/sqrt(2)
    La2 = rand.gaussian(5, (B, 2 * S), scale=3.0)
    got = modem.demap_prior_bruteforce(y, n0, 2, method, La2).reshape(B, S, 2)
    ch = -2.0 * np.sqrt(2.0) / n0[:, None]
    assert np.allclose(got[..., 0], ch * y.real + La2.reshape(B, S, 2)[..., 0], rtol=1e-12, atol=1e-12)
    assert np.allclose(got[..., 1], ch * y.imag + La2.reshape(B, S, 2)[..., 1], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [4, 6])
@pytest.mark.parametrize("method", ["exact", "maxlog"])
def test_genie_prior_gives_two_point_llr(m, method):
    B, S = 2, 7
    t = rand.bits(6, (B, S * m))
    x = modem.map_bits(t, m)
    n0 = np.array([0.2, 0.6])
    y = x + _y(7, B, S, scale=0.3)
    La = (2.0 * t - 1.0) * 60.0
    Le = modem.demap_prior_bruteforce(y, n0, m, method, La, extrinsic=True).reshape(B, S, m)
    pts = modem.constellation(m)
    idx = (t.reshape(B, S, m).astype(np.int64) * (1 << np.arange(m - 1, -1, -1))).sum(-1)
    for i in range(m):
        bit = 1 << (m - 1 - i)
        x1 = pts[idx | bit]
        x0 = pts[idx & ~bit]
        ref = (np.abs(y - x0) ** 2 - np.abs(y - x1) ** 2) / n0[:, None]
        assert np.allclose(Le[..., i], ref, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("method", ["exact", "maxlog"])
def test_extrinsic_ignores_own_prior(method):
    m, B, S = 4, 2, 5
    y = _y(8, B, S)
    n0 = np.array([0.4, 0.9])
    La = rand.gaussian(9, (B, S * m), scale=2.0)
    a = modem.demap_prior_bruteforce(y, n0, m, method, La, extrinsic=True).reshape(B, S, m)
    for i in range(m):
        Lb = La.reshape(B, S, m).copy()
        Lb[..., i] += 7.5
        b = modem.demap_prior_bruteforce(y, n0, m, method, Lb.reshape(B, -1), extrinsic=True)
        assert np.allclose(a[..., i], b.reshape(B, S, m)[..., i], rtol=1e-10, atol=1e-10)


def _bi_awgn_capacity(s):
    """C = h(Y) - h(N) for Y = +-1 + N, N ~ N(0, s^2), equiprobable inputs."""
    def p(y):
        return 0.5 * (np.exp(-(y - 1) ** 2 / (2 * s * s)) + np.exp(-(y + 1) ** 2 / (2 * s * s))) \
            / np.sqrt(2 * np.pi * s * s)

    def f(y):
        v = p(y)
        return -v * np.log2(v) if v > 0 else 0.0

    hy, _ = quad(f, -1 - 40 * s, 1 + 40 * s, limit=400, epsabs=1e-13)
    return hy - 0.5 * np.log2(2 * np.pi * np.e * s * s)


def test_J_is_bi_awgn_capacity_and_invertible():
    assert ox.J(0.0) == 0.0
    for s in (0.5, 0.8, 1.0, 1.6, 3.0):
        # the LLR 2y/s^2 is consistent Gaussian with sigma = 2/s
        assert abs(ox.J(2.0 / s) - _bi_awgn_capacity(s)) < 1e-9, s
    vals = [ox.J(x) for x in np.linspace(0.1, 12, 25)]
    assert np.all(np.diff(vals) > 0) and vals[-1] > 0.999
    for I in (0.05, 0.3, 0.5, 0.9, 0.99):
        assert abs(ox.J(ox.J_inv(I)) - I) < 1e-10


def test_mutual_info_estimate():
    n = 400_000
    for sigma in (0.7, 2.0, 4.0):
        t = rand.bits(10, (1, n))
        L = ox.apriori_llrs(t, np.array([sigma]), rand.gaussian(11, (1, n)))
        sgn = 2.0 * t - 1.0
        v = ox.softplus(-sgn * L) / ox.LN2
        est = ox.mutual_info(L, t)[0]
        assert abs(est - ox.J(sigma)) < 5 * v.std() / np.sqrt(n), sigma
    t = rand.bits(12, (2, 1000))
    assert np.allclose(ox.mutual_info((2.0 * t - 1.0) * 60.0, t), 1.0, atol=1e-20)
    assert np.allclose(ox.mutual_info(np.zeros((2, 1000)), t), 0.0, atol=1e-15)


@pytest.mark.parametrize("base,Z", [([[0, 0, -1], [-1, 0, 0]], 1), ([[3, 1, -1], [-1, 4, 2]], 5)])
def test_decoder_extrinsic_on_tree_code_is_map(base, Z):
    from oracle import decoders as D
    g = tiny_graph(base, Z)
    L = rand.gaussian(13, (5, g.n_dec), scale=1.5)
    app = D.spa_flood(g, -L, iters=6)
    Le = ox.decoder_extrinsic(g, app, L)
    assert np.allclose(Le, map_llr(g, L) - L, rtol=1e-10, atol=1e-10)


def test_decoder_extrinsic_excludes_the_clamped_input():
    # a degree-1 variable node next to a single parity check: its posterior
    # is its (clamped) input plus the check message, the extrinsic part is
    # the check message alone, whatever the input's size
    from oracle import decoders as D
    g = tiny_graph([[0, 0, 0]], 1)
    L = np.array([[35.0, 2.0, -1.5], [-50.0, 0.7, 3.0]])
    app = D.spa_flood(g, -L, iters=1)
    Le = ox.decoder_extrinsic(g, app, L)
    lam = np.clip(L, -D.LLR_MAX, D.LLR_MAX)
    # check-to-variable message of an SPC in the boundary convention
    for b in range(2):
        for i in range(3):
            o = [j for j in range(3) if j != i]
            r = 2 * np.arctanh(np.prod(np.tanh(-lam[b, o] / 2)))
            assert abs(Le[b, i] - (-r)) < 1e-9


def test_bicm_id_with_gray_qpsk_is_plain_decoding():
    qb, g = graph("small")
    B, m = 3, 2
    n0 = np.full(B, 0.6)
    u = philox.source_bits(21, 0, B, qb.k)
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)
    t = c[:, g.tx_lo:g.tx_lo + g.e_tx]
    y = modem.awgn(modem.map_bits(t, m), n0, philox.normals(21, 0, B, g.e_tx // m))
    app, passes = ox.bicm_id(g, y, n0, m, "exact", outer=3, iters=5)
    for p in passes[1:]:
        assert np.allclose(p, passes[0], rtol=1e-9, atol=1e-9)


def test_stream1_real_normals_are_the_channel_normals():
    g = philox.normals(77, 5, 3, 10)
    r = philox.normals_real(77, 5, 3, 20, stream=1)
    assert np.allclose(r[:, 0::2], g.real, rtol=0, atol=1e-15)
    assert np.allclose(r[:, 1::2], g.imag, rtol=0, atol=1e-15)
    big = philox.normals_real(78, 0, 4, 50_000)
    assert abs(big.mean()) < 0.01 and abs(big.var() - 1.0) < 0.01
