"""Pins of the Polar-code oracle.

* Transform = multiplication by the Kronecker power F^{(x)n}; it is its own
  inverse.
* Construction: on the BEC the Bhattacharyya recursion is exact, so the
  erasure probability of every synthetic channel, found by enumerating all
  erasure patterns and all inputs for N = 8, must equal it; the recursion
  conserves capacity.
* CRC: catalogue check values of CRC-16/XMODEM (0x1021) and CRC-8/SMBUS
  (0x07) on the ASCII string "123456789".
* SC with no frozen bit returns the inverse transform of the channel's hard
  decisions (the min-sum f keeps the sign of the exact one).
* SCL with a list large enough to keep every hypothesis is maximum
  likelihood: every final path metric equals the correlation discrepancy
  sum |lambda_j| [x_j != hard_j] of its codeword (enumerated by brute
  force) and the decision is the minimum.
* SCL with L = 1 is SC; SCL-CRC returns a path that passes the CRC when
  the list holds one.
"""
import itertools

import numpy as np
import pytest

from inputs import rand
from oracle import polar as P


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6])
def test_transform_is_kronecker_power_and_involution(n):
    N = 1 << n
    u = rand.bits(n, (7, N))
    x = P.transform(u)
    assert np.array_equal(x, (u.astype(np.int64) @ P.generator(n)) % 2)
    assert np.array_equal(P.transform(x), u)


def _bec_erasure_bruteforce(n, eps):
    """P(u_i undetermined by the unerased outputs and u_0..u_{i-1})."""
    N = 1 << n
    G = P.generator(n).astype(np.int64)
    U = np.array(list(itertools.product((0, 1), repeat=N)), dtype=np.int64)
    X = (U @ G) % 2
    pe = np.zeros(N)
    for E in itertools.product((0, 1), repeat=N):       # 1 = erased
        E = np.array(E, dtype=bool)
        w = eps ** E.sum() * (1 - eps) ** (N - E.sum())
        # u = 0 is sent (linear code): the candidates consistent with the
        # unerased outputs are the u whose x is 0 there
        ok = ~(X[:, ~E].any(axis=1))
        cand = U[ok]
        for i in range(N):
            c = cand[~(cand[:, :i].any(axis=1))] if i else cand
            if c[:, i].any():
                pe[i] += w
    return pe


def test_bhattacharyya_is_exact_on_the_bec():
    n, eps = 3, 0.4
    # the recursion starts from z0 = exp(-Es/N0); pick Es/N0 = -ln(eps)
    rate = 0.5
    ebn0_db = 10 * np.log10(-np.log(eps) / rate)
    z = P.bhattacharyya(n, ebn0_db, rate)
    assert np.allclose(z, _bec_erasure_bruteforce(n, eps), atol=1e-12)
    z10 = P.bhattacharyya(10, 1.0, 0.5)
    z0 = np.exp(-0.5 * 10 ** 0.1)
    assert abs((1 - z10).sum() - 1024 * (1 - z0)) < 1e-9


def test_info_mask_takes_the_k_best():
    n, K = 6, 20
    m = P.info_mask(n, K, 2.0)
    z = P.bhattacharyya(n, 2.0, K / 64)
    assert m.sum() == K and z[m == 1].max() <= z[m == 0].min()


def _ascii_bits(s):
    return np.array([(c >> (7 - j)) & 1 for c in s.encode() for j in range(8)], dtype=np.uint8)


def test_crc_catalogue_values():
    d = _ascii_bits("123456789")
    c16 = P.crc(d[None, :], 0x1021, 16)[0]
    assert int("".join(map(str, c16)), 2) == 0x31C3
    c8 = P.crc(d[None, :], 0x07, 8)[0]
    assert int("".join(map(str, c8)), 2) == 0xF4
    bits = rand.bits(3, (4, 40))
    full = np.concatenate([bits, P.crc(bits, 0x1021, 16)], axis=1)
    assert P.crc_ok(full, 0x1021, 16).all()
    full[1, 5] ^= 1
    assert not P.crc_ok(full, 0x1021, 16)[1]


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_sc_without_frozen_bits_inverts_hard_decisions(mode):
    n = 5
    N = 1 << n
    for seed in range(4):
        lam = rand.gaussian(10 + seed, N, scale=2.0)
        u = P.sc_decode(lam, np.ones(N, np.uint8), mode)
        assert np.array_equal(u, P.transform((lam < 0).astype(np.uint8)))


def test_noiseless_codewords_decode():
    n, K = 7, 50
    mask = P.info_mask(n, K, 1.0)
    data = rand.bits(20, (3, K - 8))
    x = P.encode(data, mask, 0x07, 8)
    lam = (1.0 - 2.0 * x) * 6.0
    for b in range(3):
        for L in (1, 4):
            u, _, _ = P.scl_decode(lam[b], mask, L, 0x07, 8)
            assert np.array_equal(P.data_bits(u, mask, 8), data[b])
        assert np.array_equal(P.data_bits(P.sc_decode(lam[b], mask), mask, 8), data[b])


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_scl_with_full_list_is_ml(mode):
    n, K = 4, 4
    N = 1 << n
    mask = P.info_mask(n, K, 0.0)
    info = np.flatnonzero(mask)
    allu = np.zeros((1 << K, N), np.uint8)
    allu[:, info] = np.array(list(itertools.product((0, 1), repeat=K)), dtype=np.uint8)
    X = P.transform(allu)
    for seed in range(6):
        lam = rand.gaussian(30 + seed, N, scale=1.5)
        if mode == "fp32":
            lam = lam.astype(np.float32)
        hard = (lam < 0).astype(np.uint8)
        disc = (np.abs(lam.astype(np.float64)) * (X != hard)).sum(1)
        u, pm, uh = P.scl_decode(lam, mask, 1 << K, mode=mode)
        # every hypothesis survives; each path's metric is its discrepancy
        for s in range(1 << K):
            j = int((uh[s][info] * (1 << np.arange(K - 1, -1, -1))).sum())
            assert abs(float(pm[s]) - disc[j]) <= 1e-5 * max(1.0, disc[j])
        best = int(np.argmin(disc))
        assert np.array_equal(u, allu[best])


def test_scl_list_one_is_sc():
    n, K = 6, 32
    mask = P.info_mask(n, K, 1.5)
    for seed in range(5):
        lam = rand.gaussian(40 + seed, 1 << n, scale=2.0) + 1.0
        for mode in ("fp64", "fp32"):
            u, _, _ = P.scl_decode(lam, mask, 1, mode=mode)
            assert np.array_equal(u, P.sc_decode(lam, mask, mode))


def test_scl_crc_picks_a_passing_path():
    n, K, r, poly = 6, 30, 8, 0x07
    mask = P.info_mask(n, K, 1.0)
    info = np.flatnonzero(mask)
    hits = 0
    for seed in range(40):
        data = rand.bits(50 + seed, (1, K - r))
        x = P.encode(data, mask, poly, r)[0]
        lam = (1.0 - 2.0 * x) * 1.2 + rand.gaussian(60 + seed, 1 << n, scale=1.3)
        u, pm, uh = P.scl_decode(lam, mask, 8, poly, r)
        passing = [s for s in range(8) if P.crc_ok(uh[s][info][None], poly, r)[0]]
        if passing:
            assert P.crc_ok(u[info][None], poly, r)[0]
            best = min(passing, key=lambda s: (pm[s], s))
            assert np.array_equal(u, uh[best])
            hits += int(not np.array_equal(uh[best], uh[min(range(8), key=lambda s: (pm[s], s))]))
    assert hits > 0          # the CRC changed the decision at least once


def test_non_finite_channel_values_stay_finite():
    """NaN reads as 0, +-inf as +-2^100; with opposite-sign infinities under
    one node (the right child's g would be inf - inf) every metric of every
    list size stays finite, and an all-NaN channel decodes as all zeros."""
    import numpy as np
    from oracle import polar as P
    lam = np.array([np.nan, np.inf, -np.inf, 1.0], dtype=np.float32)
    rc = P.read_channel(lam, np.float32)
    assert rc[0] == 0 and rc[1] == np.float32(2.0 ** 100) and rc[2] == -np.float32(2.0 ** 100)
    assert rc[3] == 1.0
    n, K = 5, 12
    mask = P.info_mask(n, K, 1.0)
    r = np.random.default_rng(7)
    for trial in range(8):
        lam = r.normal(1.0, 2.0, 1 << n)
        pos = r.choice(1 << n, 6, replace=False)
        lam[pos[:3]] = np.inf
        lam[pos[3:]] = -np.inf
        for L in (1, 4, 8):
            u, pm, _ = P.scl_decode(lam, mask, L, mode="fp32")
            assert np.isfinite(pm[:min(L, 1 << K)]).all(), (trial, L, pm)
    u = P.sc_decode(np.full(1 << n, np.nan), mask, "fp32")
    assert not u.any()
