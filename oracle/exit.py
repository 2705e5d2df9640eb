"""EXIT chart simulations and iterative demapping and decoding.

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this package.

The paper lists "Demapper with prior" and "EXIT chart simulations" among the
library's FEC features (Sec. III-B) and prints no formulas for them; what
follows is the textbook construction (ten Brink, "Convergence behavior of
iteratively decoded parallel concatenated codes", IEEE Trans. Commun. 2001),
in the LLR convention of the boundary (logit of bit 1):

* a-priori LLRs of mutual information I_A are consistent Gaussian LLRs,
  La = (2c - 1) sigma^2 / 2 + sigma n with n standard normal and
  sigma = J^-1(I_A);
* J(sigma) = 1 - E[log2(1 + e^{-X})], X ~ N(sigma^2/2, sigma^2), the mutual
  information between a bit and such an LLR;
* the mutual information between code bits c and LLRs L is estimated by
  the time average 1 - mean log2(1 + e^{-(2c-1) L});
* the decoder's extrinsic output on the transmitted bits is
  L_post - L_in with L_in as the decoder used it (clamped to +-20 by the
  sum-product decoders; zero for transmitted bits outside the decoded
  graph);
* iterative demapping and decoding (BICM-ID) feeds the decoder's extrinsic
  back to the demapper as its prior and the demapper's extrinsic to the
  decoder as its input.
"""
from __future__ import annotations

import numpy as np

from . import decoders, modem, philox, qc

LN2 = np.log(2.0)


def softplus(x):
    return np.logaddexp(0.0, x)


def apriori_llrs(t: np.ndarray, sigma: np.ndarray, nrm: np.ndarray) -> np.ndarray:
    """Consistent Gaussian LLRs ``float64[B][n]`` for bits ``t u8[B][n]`` with
    per-codeword ``sigma[B]`` and standard normals ``nrm[B][n]``."""
    s = np.asarray(sigma, dtype=np.float64).reshape(-1, 1)
    sgn = 2.0 * np.asarray(t, dtype=np.float64) - 1.0
    return sgn * s * s / 2.0 + s * np.asarray(nrm, dtype=np.float64)


def mutual_info(L: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Per-row estimate ``1 - mean_i log2(1 + exp(-(2 t_i - 1) L_i))``."""
    sgn = 2.0 * np.asarray(t, dtype=np.float64) - 1.0
    return 1.0 - softplus(-sgn * np.asarray(L, dtype=np.float64)).mean(-1) / LN2


def J(sigma: float) -> float:
    """Mutual information of a consistent Gaussian LLR with std sigma, by
    adaptive quadrature over the LLR's density."""
    from scipy.integrate import quad

    sigma = float(sigma)
    if sigma <= 0.0:
        return 0.0
    mu = sigma * sigma / 2.0

    def f(z):  # z standard normal, X = mu + sigma z
        return np.exp(-0.5 * z * z) / np.sqrt(2 * np.pi) * softplus(-(mu + sigma * z)) / LN2

    val, _ = quad(f, -40.0, 40.0, limit=400, epsabs=1e-13, epsrel=1e-12)
    return 1.0 - val


def J_inv(I: float, tol: float = 1e-12) -> float:
    """sigma with J(sigma) = I (bisection; J is increasing)."""
    if I <= 0.0:
        return 0.0
    lo, hi = 0.0, 1.0
    while J(hi) < I:
        hi *= 2.0
        if hi > 1e3:
            return hi
    while hi - lo > tol * max(1.0, hi):
        mid = 0.5 * (lo + hi)
        if J(mid) < I:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def decoder_extrinsic(g: qc.Graph, app: np.ndarray, L_in: np.ndarray,
                      llr_max: float | None = decoders.LLR_MAX) -> np.ndarray:
    """Extrinsic LLRs ``[B][e_tx]`` of the transmitted bits from the
    decoder's internal APP (``-L_post``, as returned by ``oracle.decoders``)
    and its input ``L_in[B][e_tx]``: L_post minus the input as the decoder
    used it (clamped to +-llr_max, as the sum-product decoders clamp their
    channel LLRs; None: no clamp)."""
    B = L_in.shape[0]
    out = np.zeros((B, g.e_tx))
    hi = min(g.tx_lo + g.e_tx, g.n_dec)
    n = hi - g.tx_lo
    lin = np.asarray(L_in, dtype=np.float64)[:, :n]
    if llr_max is not None:
        lin = np.clip(lin, -llr_max, llr_max)
    out[:, :n] = -np.asarray(app, dtype=np.float64)[:, g.tx_lo:hi] - lin
    return out


def demapper_exit(y, n0, t, m, method, sigma_a, nrm):
    """I_E of the demapper's extrinsic output given a-priori LLRs of std
    ``sigma_a`` (per codeword)."""
    La = apriori_llrs(t, sigma_a, nrm)
    Le = modem.demap_prior_bruteforce(y, n0, m, method, La, extrinsic=True)
    return mutual_info(Le, t), Le


def decoder_exit(g: qc.Graph, t, sigma_a, nrm, iters: int = 20):
    """I_E of the sum-product decoder's extrinsic output when its only
    input is a-priori LLRs of std ``sigma_a`` on the transmitted bits."""
    La = apriori_llrs(t, sigma_a, nrm)
    app = decoders.spa_flood(g, decoders.channel_lam(g, La), iters)
    Le = decoder_extrinsic(g, app, La)
    return mutual_info(Le, t), Le


def bicm_id(g: qc.Graph, y, n0, m: int, method: str, outer: int, iters: int = 20):
    """Iterative demapping and sum-product decoding: ``outer`` decoder runs
    of ``iters`` iterations.  Returns the decoder's internal APP of the last
    run and the demapper outputs of every pass."""
    B, S = y.shape
    prior = np.zeros((B, S * m))
    passes = []
    app = None
    for _ in range(outer):
        Le_dem = modem.demap_prior_bruteforce(y, n0, m, method, prior, extrinsic=True)
        passes.append(Le_dem)
        app = decoders.spa_flood(g, decoders.channel_lam(g, Le_dem), iters)
        prior = decoder_extrinsic(g, app, Le_dem)
    return app, passes


def normals_for_prior(seed: int, cw0: int, B: int, n: int) -> np.ndarray:
    return philox.normals_real(seed, cw0, B, n, 2)
