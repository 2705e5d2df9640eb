"""Pins of the mapper, channel and demappers.

Closed forms: uncoded BPSK BER Q(sqrt(2 Eb/N0)); uncoded Gray 16-QAM BER
(3Q(d) + 2Q(3d) - Q(5d))/4 with d = sqrt(0.8 Eb/N0) (Cho & Yoon 2002);
64-QAM per-axis error from Gaussian interval probabilities.  Brute force:
Gray neighbours, per-axis separability of the exact and max-log LLRs,
max-log sign equals the nearest point's bit."""
import math
import os

import numpy as np
import pytest
from scipy import stats as sst

from inputs import rand
from oracle import modem, philox, stats

HERE = os.path.dirname(os.path.abspath(__file__))


def test_16qam_golden_table():
    rows = np.loadtxt(os.path.join(HERE, "golden", "qam16_gray_38211.txt"), comments="#")
    pts = modem.constellation(4)
    for row in rows:
        b = row[:4].astype(int)
        idx = int("".join(str(x) for x in b), 2)
        assert abs(pts[idx] * math.sqrt(10) - complex(row[4], row[5])) < 1e-12


@pytest.mark.parametrize("m", [1, 2, 4, 6])
def test_unit_energy_and_gray(m):
    pts = modem.constellation(m)
    assert abs(np.mean(np.abs(pts) ** 2) - 1.0) < 1e-12
    lab = modem.labels(m)
    if m == 1:
        return
    d = np.abs(pts[:, None] - pts[None, :])
    dmin = d[d > 1e-9].min()
    for a in range(len(pts)):
        for b in range(len(pts)):
            if abs(d[a, b] - dmin) < 1e-9:
                assert int((lab[a] != lab[b]).sum()) == 1


def _simulate_uncoded(m, ebn0_db, nsym, seed):
    B = 100
    S = nsym // B
    t = philox.source_bits(seed, 0, B, S * m)
    x = modem.map_bits(t, m)
    n0 = modem.ebn0_to_n0(ebn0_db, 1.0, m)
    y = modem.awgn(x, np.full(B, n0), philox.normals(seed, 0, B, S))
    L = modem.demap_bpsk(y, np.full(B, n0)) if m == 1 else \
        modem.demap_bruteforce(y, np.full(B, n0), m, "maxlog")
    return int(((L > 0).astype(np.uint8) != t).sum()), t.size


@pytest.mark.parametrize("ebn0", [0.0, 2.0, 4.0, 6.0])
def test_bpsk_ber_closed_form(ebn0):
    err, n = _simulate_uncoded(1, ebn0, 10_000_000, 1000 + int(ebn0))
    lo, hi = stats.wilson(err, n, z=3.29)
    assert lo <= stats.q_function(math.sqrt(2 * 10 ** (ebn0 / 10))) <= hi


@pytest.mark.parametrize("ebn0", [0.0, 4.0, 8.0])
def test_16qam_ber_closed_form(ebn0):
    err, n = _simulate_uncoded(4, ebn0, 400_000, 2000 + int(ebn0))
    d = math.sqrt(0.8 * 10 ** (ebn0 / 10))
    Q = stats.q_function
    p = (3 * Q(d) + 2 * Q(3 * d) - Q(5 * d)) / 4
    lo, hi = stats.wilson(err, n, z=3.29)
    assert lo <= p <= hi


def test_64qam_ber_interval_probabilities():
    ebn0 = 6.0
    err, n = _simulate_uncoded(6, ebn0, 300_000, 3000)
    n0 = modem.ebn0_to_n0(ebn0, 1.0, 6)
    sigma = math.sqrt(n0 / 2)
    scale = math.sqrt(42)
    levels = {}
    import itertools
    for bits in itertools.product((0, 1), repeat=3):
        levels[bits] = modem.pam_level(bits) / scale
    # per axis: bit error probability averaged over the 8 levels, decisions
    # by nearest level (max-log hard decisions are nearest-point decisions)
    srt = sorted(levels.items(), key=lambda kv: kv[1])
    vals = np.array([v for _, v in srt])
    mids = (vals[1:] + vals[:-1]) / 2
    edges = np.concatenate([[-np.inf], mids, [np.inf]])
    pe = 0.0
    for tb, tv in srt:
        for (rb, _), lo_, hi_ in zip(srt, edges[:-1], edges[1:]):
            pr = sst.norm.cdf((hi_ - tv) / sigma) - sst.norm.cdf((lo_ - tv) / sigma)
            pe += pr * sum(a != b for a, b in zip(tb, rb))
    p = pe / (8 * 3)
    lo, hi = stats.wilson(err, n, z=3.29)
    assert lo <= p <= hi


def test_bpsk_closed_form_equals_bruteforce():
    y = rand.gaussian(1, (20, 30)) + 1j * rand.gaussian(2, (20, 30))
    n0 = rand.uniform(3, 20, 0.05, 2.0)
    for meth in ("exact", "maxlog"):
        assert np.allclose(modem.demap_bruteforce(y, n0, 1, meth), modem.demap_bpsk(y, n0), rtol=1e-12, atol=1e-12)


def _axis_llr(v, n0, h, method, scale):
    """Per-axis LLRs from the 2^h PAM levels of one axis only."""
    import itertools
    labs = list(itertools.product((0, 1), repeat=h))
    lv = np.array([modem.pam_level(b) / scale for b in labs])
    d2 = (v[..., None] - lv) ** 2 / n0[..., None]
    out = []
    for i in range(h):
        one = np.array([b[i] == 1 for b in labs])
        if method == "maxlog":
            out.append(d2[..., ~one].min(-1) - d2[..., one].min(-1))
        else:
            a1, a0 = -d2[..., one], -d2[..., ~one]
            out.append(np.logaddexp.reduce(a1, -1) - np.logaddexp.reduce(a0, -1))
    return out


@pytest.mark.parametrize("m", [2, 4, 6])
@pytest.mark.parametrize("method", ["exact", "maxlog"])
def test_demapper_separates_per_axis(m, method):
    B, S = 16, 40
    y = 1.5 * (rand.gaussian(10 + m, (B, S)) + 1j * rand.gaussian(20 + m, (B, S)))
    n0 = rand.uniform(30 + m, B, 0.05, 2.0)
    L = modem.demap_bruteforce(y, n0, m, method).reshape(B, S, m)
    h = m // 2
    scale = math.sqrt(2 * (4 ** h - 1) / 3)
    n0b = np.broadcast_to(n0[:, None], (B, S))
    li = _axis_llr(y.real, n0b, h, method, scale)
    lq = _axis_llr(y.imag, n0b, h, method, scale)
    for i in range(h):
        assert np.allclose(L[:, :, 2 * i], li[i], rtol=1e-9, atol=1e-9)
        assert np.allclose(L[:, :, 2 * i + 1], lq[i], rtol=1e-9, atol=1e-9)


def test_qpsk_exact_equals_maxlog():
    y = rand.gaussian(5, (10, 50)) + 1j * rand.gaussian(6, (10, 50))
    n0 = rand.uniform(7, 10, 0.05, 2.0)
    assert np.allclose(modem.demap_bruteforce(y, n0, 2, "exact"),
                       modem.demap_bruteforce(y, n0, 2, "maxlog"), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m", [4, 6])
def test_exact_vs_maxlog_gap_and_sign(m):
    B, S = 8, 200
    y = 1.3 * (rand.gaussian(40 + m, (B, S)) + 1j * rand.gaussian(50 + m, (B, S)))
    n0 = rand.uniform(60 + m, B, 0.05, 2.0)
    Le = modem.demap_bruteforce(y, n0, m, "exact")
    Lm = modem.demap_bruteforce(y, n0, m, "maxlog")
    assert (np.abs(Le - Lm) <= math.log(2 ** (m // 2 - 1)) + 1e-9).all()
    pts = modem.constellation(m)
    near = np.argmin(np.abs(y[:, :, None] - pts) ** 2, axis=-1)
    bits = modem.labels(m)[near].reshape(B, S * m)
    assert np.array_equal((Lm > 0).astype(np.uint8), bits)


def test_awgn_variance():
    B, S = 200, 2000
    x = np.zeros((B, S), dtype=complex)
    n0 = np.full(B, 0.37)
    y = modem.awgn(x, n0, philox.normals(9, 0, B, S))
    v = np.mean(np.abs(y - x) ** 2)
    assert abs(v - 0.37) < 4.5 * 0.37 / math.sqrt(B * S)


def test_ebn0_to_n0_table():
    # 16-QAM, rate 1/3 at 0 dB: N0 = 1 / (1/3 * 4) = 0.75
    assert abs(modem.ebn0_to_n0(0.0, 1 / 3, 4) - 0.75) < 1e-15
    assert abs(modem.ebn0_to_n0(1.0, 0.5, 1) - 1.5887) < 1e-4


def test_quantizer_half_even_and_saturation():
    L = np.array([0.25, 0.75, -0.25, -0.75, 1.25, 100.0, -100.0, 15.25, 15.75], dtype=np.float32)
    assert modem.quantize(L).tolist() == [0, 2, 0, -2, 2, 31, -31, 30, 31]
