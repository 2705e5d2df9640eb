"""Belief-propagation decoders on a QC Tanner graph (FP64 unless stated).

The paper names a "belief propagation (BP) decoder and variants" among its
FEC features and the min-sum BP decoder as a custom-kernel candidate (Secs.
"Features" and "Custom CUDA kernels"); it prints no update rule.  The rules
below are textbook: the sum-product algorithm (Kschischang, Frey & Loeliger
2001; Richardson & Urbanke, Modern Coding Theory, 2008), offset and
normalized min-sum (Chen & Fossorier 2002) and layered scheduling (Mansour &
Shanbhag 2003; Hocevar 2004).

Internal convention: ``lam = -L = ln P(0)/P(1)``, ``b_hat = [APP < 0]``.
A decoder input ``lam`` is ``float64[B][n_dec]`` with zeros at punctured
and untransmitted variable nodes (``channel_lam``).  Messages are kept per
edge in canonical order: ``q`` (variable to check) and ``r`` (check to
variable), both ``[B][E]``.
"""
from __future__ import annotations

import numpy as np

from .qc import Graph

LLR_MAX = 20.0


def channel_lam(g: Graph, L: np.ndarray, dtype=np.float64) -> np.ndarray:
    """Place boundary LLRs ``L[B][e_tx]`` of transmitted VNs
    ``tx_lo .. tx_lo+e_tx-1`` at the decoder's VNs as ``lam = -L``; every
    other decoded VN (punctured or untransmitted) gets 0."""
    L = np.asarray(L)
    B = L.shape[0]
    lam = np.zeros((B, g.n_dec), dtype=dtype)
    lo = g.tx_lo
    hi = min(lo + g.e_tx, g.n_dec)
    lam[:, lo:hi] = -L[:, :hi - lo].astype(dtype)
    return lam


def _scatter_app(g: Graph, lam: np.ndarray, r: np.ndarray, w: np.ndarray | None = None) -> np.ndarray:
    """APP_v = lam_v + sum over edges e at v of (w_e) r_e."""
    Z = g.Z
    app = lam.astype(np.result_type(lam, r), copy=True)
    rr = np.arange(Z)
    for e, (_, j, s) in enumerate(g.entries):
        vn = j * Z + (rr + s) % Z
        val = r[:, e * Z:(e + 1) * Z]
        if w is not None:
            val = val * w[e * Z:(e + 1) * Z]
        app[:, vn] += val
    return app


# --------------------------------------------------------------------------
# Sum-product (flooding)
# --------------------------------------------------------------------------

def phi(x: np.ndarray) -> np.ndarray:
    """phi(x) = ln((e^x + 1)/(e^x - 1)) = log1p(2 / expm1(x)) for x >= 0,
    with phi(0) = +inf and phi(+inf) = 0."""
    with np.errstate(divide="ignore", over="ignore"):
        return np.log1p(2.0 / np.expm1(x))


def cn_spa_phi(q: np.ndarray) -> np.ndarray:
    """Sum-product check update on ``q[..., d, Z]`` (axis -2 runs over the
    check's edges): r_v = s_v phi(sum_{v' != v} phi(|q_v'|)), where s_v is
    the product of sgn(q_v') over v' != v with sgn(0) = +1.  The extrinsic
    sums are exclusive prefix plus exclusive suffix sums (no subtraction)."""
    f = phi(np.abs(q))
    zero = np.zeros_like(f[..., :1, :])
    pre = np.cumsum(np.concatenate([zero, f[..., :-1, :]], axis=-2), axis=-2)
    suf = np.flip(np.cumsum(np.flip(np.concatenate([f[..., 1:, :], zero], axis=-2), axis=-2), axis=-2), axis=-2)
    s = np.where(q < 0, -1.0, 1.0)
    s_ext = np.prod(s, axis=-2, keepdims=True) * s
    return s_ext * phi(pre + suf)


def cn_spa_tanh(q: np.ndarray) -> np.ndarray:
    """The same check update in the tanh form:
    r_v = 2 atanh(prod_{v' != v} tanh(q_v' / 2))."""
    t = np.tanh(q / 2.0)
    d = q.shape[-2]
    out = np.empty_like(q)
    for a in range(d):
        others = np.delete(t, a, axis=-2)
        out[..., a, :] = 2.0 * np.arctanh(np.prod(others, axis=-2))
    return out


def spa_iteration(g: Graph, lam: np.ndarray, q: np.ndarray, llr_max: float = LLR_MAX,
                  w: np.ndarray | None = None):
    """One flooding round from variable-to-check messages ``q``.

    r = clamp(CN_SPA(q), +-llr_max); APP = lam + sum_c (w) r;
    q' = clamp(APP - (w) r, +-llr_max).  ``w`` (per-edge weights) gives the
    weighted-BP round; ``None`` is plain SPA.  Returns (r, APP, q')."""
    B = q.shape[0]
    r = np.empty_like(q)
    for i in range(g.rows):
        ids = g.row_edge_ids(i)
        r[:, ids] = np.clip(cn_spa_phi(q[:, ids]), -llr_max, llr_max)
    app = _scatter_app(g, lam, r, w)
    vn = g.edge_vn()
    wr = r if w is None else r * w[None, :]
    qn = np.clip(app[:, vn] - wr, -llr_max, llr_max)
    return r, app, qn


def spa_flood(g: Graph, lam: np.ndarray, iters: int = 20, llr_max: float = LLR_MAX,
              trace: bool = False):
    """Flooding sum-product: lam <- clamp(lam, +-llr_max); q^(1) = lam on
    every edge; ``iters`` full check+variable rounds with no early stop.

    Returns the final APP (``float64[B][n_dec]``) and, with ``trace``, the
    lists of r^(t) and q^(t+1) per round."""
    lam = np.clip(np.asarray(lam, dtype=np.float64), -llr_max, llr_max)
    q = lam[:, g.edge_vn()]
    rs, qs = [], []
    app = lam.copy()
    for _ in range(iters):
        r, app, q = spa_iteration(g, lam, q, llr_max)
        if trace:
            rs.append(r)
            qs.append(q)
    return (app, rs, qs) if trace else app


# --------------------------------------------------------------------------
# Offset min-sum on integers (flooding)
# --------------------------------------------------------------------------

def _min1_min2(a: np.ndarray):
    """Over axis -2: first argmin i1, its value m1, and m2 = min over the
    other positions."""
    i1 = np.argmin(a, axis=-2)
    m1 = np.min(a, axis=-2)
    d = a.shape[-2]
    pos = np.arange(d).reshape((1,) * (a.ndim - 2) + (d, 1))
    big = np.iinfo(a.dtype).max if np.issubdtype(a.dtype, np.integer) else np.inf
    m2 = np.min(np.where(pos == i1[..., None, :], big, a), axis=-2)
    return i1, m1, m2, pos


def cn_oms(q: np.ndarray, offset: int = 1) -> np.ndarray:
    """Offset min-sum check update on integer ``q[..., d, Z]``:
    r_v = (S sgn q_v) max((v == i1 ? m2 : m1) - offset, 0), S the product of
    all signs (sgn(0) = +1), m1 = min |q|, i1 its first position, m2 the
    minimum over the other positions."""
    q = np.asarray(q, dtype=np.int64)
    a = np.abs(q)
    s = np.where(q < 0, -1, 1)
    S = np.prod(s, axis=-2, keepdims=True)
    i1, m1, m2, pos = _min1_min2(a)
    sel = np.where(pos == i1[..., None, :], m2[..., None, :], m1[..., None, :])
    return S * s * np.maximum(sel - offset, 0)


def oms_iteration(g: Graph, lam: np.ndarray, q: np.ndarray, offset: int = 1, sat: int = 31):
    """One flooding round: r = CN_OMS(q); APP = lam + sum_c r (exact
    integers); q' = clamp(APP - r, +-sat).  Returns (r, APP, q')."""
    r = np.empty_like(q)
    for i in range(g.rows):
        ids = g.row_edge_ids(i)
        r[:, ids] = cn_oms(q[:, ids], offset)
    app = _scatter_app(g, lam, r)
    qn = np.clip(app[:, g.edge_vn()] - r, -sat, sat)
    return r, app, qn


def oms_flood(g: Graph, lam: np.ndarray, iters: int = 20, offset: int = 1, sat: int = 31,
              trace: bool = False):
    """Offset min-sum on integer LLRs (``lam`` = minus the quantized channel
    LLR, already within +-sat); q^(1) = lam; ``iters`` rounds."""
    lam = np.asarray(lam, dtype=np.int64)
    q = lam[:, g.edge_vn()]
    rs, qs = [], []
    app = lam.copy()
    for _ in range(iters):
        r, app, q = oms_iteration(g, lam, q, offset, sat)
        if trace:
            rs.append(r)
            qs.append(q)
    return (app, rs, qs) if trace else app


# --------------------------------------------------------------------------
# Layered normalized min-sum
# --------------------------------------------------------------------------

def nms_layered(g: Graph, lam: np.ndarray, iters: int = 20, alpha: float = 0.75,
                mode: str = "fp64", trace: bool = False, order=None):
    """Layered normalized min-sum.

    State: APP (initially lam, no clamp) and per-edge r (initially 0).  Each
    iteration visits the decoded base rows in natural order (or in
    ``order``, a permutation of the rows); for all Z
    checks of row i at once (a QC row block meets each variable node at most
    once): t_v = APP_v - r_v, the variable-to-check message (channel value
    plus every other check's message); S, m1, i1, m2 from t with
    sgn(x) = -1 iff x < 0; r_v = (S sgn t_v) (alpha * (v == i1 ? m2 : m1));
    APP_v = t_v + r_v.  A variable node met by one check only has no other
    check message, so its t_v is the channel value lam_v itself (the same in
    exact arithmetic; in floating point APP_v - r_v would carry the rounding
    of the previous APP_v = t_v + r_v).

    ``mode="fp32"`` runs every array in IEEE single precision, each +, -, *
    rounded once (numpy does not contract), which is what a float32
    implementation without fused multiply-add computes.  ``mode="fp64"``
    runs in double.  Returns APP and, with ``trace``, (r, APP) after each
    iteration."""
    dt = np.float32 if mode == "fp32" else np.float64
    al = dt(alpha)
    ch = np.array(lam, dtype=dt, copy=True)
    app = ch.copy()
    B = app.shape[0]
    r = np.zeros((B, g.E), dtype=dt)
    vn_all = g.edge_vn()
    deg = np.bincount(g.entries[:, 1], minlength=g.cols)
    rows = []
    for i in range(g.rows):
        ids = g.row_edge_ids(i)
        one = (deg[g.entries[g.row_entries(i), 1]] == 1)[:, None]
        rows.append((ids, vn_all[ids], one))
    seq = range(g.rows) if order is None else [int(i) for i in order]
    if sorted(seq) != list(range(g.rows)):
        raise ValueError("order must be a permutation of the decoded rows")
    hist = []
    for _ in range(iters):
        for ids, vn, one in (rows[i] for i in seq):
            t = np.where(one, ch[:, vn], app[:, vn] - r[:, ids])
            a = np.abs(t)
            s = np.where(t < 0, dt(-1), dt(1))
            S = np.prod(s, axis=-2, keepdims=True)
            i1, m1, m2, pos = _min1_min2(a)
            sel = np.where(pos == i1[..., None, :], m2[..., None, :], m1[..., None, :])
            rn = (S * s) * (al * sel)
            app[:, vn] = t + rn
            r[:, ids] = rn
        if trace:
            hist.append((r.copy(), app.copy()))
    return (app, hist) if trace else app


def grouped_order(g: Graph) -> list:
    """A row order for the layered schedule that visits groups of rows with
    no common column one group after another.  Rows conflict when they meet
    a common column; groups are the colour classes of DSatur greedy
    colouring of that conflict graph (Brelaz, CACM 1979): repeatedly colour
    the uncoloured row with the most distinct colours among its neighbours,
    ties to the row with the most neighbours, then to the lowest index, with
    the smallest colour no neighbour has.  Groups in colour order, rows
    ascending within a group."""
    rows = [set(int(j) for j in g.entries[g.row_entries(i), 1]) for i in range(g.rows)]
    n = g.rows
    adj = [[b for b in range(n) if b != a and rows[a] & rows[b]] for a in range(n)]
    colour = [-1] * n
    for _ in range(n):
        best = None
        for i in range(n):
            if colour[i] >= 0:
                continue
            sat = len({colour[j] for j in adj[i] if colour[j] >= 0})
            key = (sat, len(adj[i]))
            if best is None or key > best[0]:
                best = (key, i)
        i = best[1]
        used = {colour[j] for j in adj[i]}
        c = 0
        while c in used:
            c += 1
        colour[i] = c
    return [i for c in range(max(colour) + 1) for i in range(n) if colour[i] == c]


def hard_bits(app: np.ndarray, k: int) -> np.ndarray:
    """b_hat_v = [APP_v < 0] for the information VNs 0..k-1."""
    return (np.asarray(app)[:, :k] < 0).astype(np.uint8)
