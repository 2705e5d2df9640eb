"""Weighted belief propagation, its loss and reference gradients.

The paper's premise is that gradients flow through the whole link so that
components can be trained end to end (Secs. "Why we decided to create
Sionna" and "Design principles"), and custom operations may register their
own gradients (Sec. "Custom CUDA kernels").  Weighted BP itself is textbook
(Nachmani, Be'ery & Burshtein 2016): sum-product with a learned weight on
every check-to-variable message of every iteration.

Forward (internal convention, T iterations, weights ``w[T][E]``):
q^(1) = lam; for t = 1..T: r^(t) = clamp(CN_SPA(q^(t)), +-20);
APP^(t) = lam + sum_c w^(t) r^(t); q^(t+1) = clamp(APP^(t) - w^(t) r^(t), +-20).
Output L_post = -APP^(T).  Loss = mean over (B x n_dec) of
BCE-with-logits(L_post, c) = softplus(L_post) - c L_post with the code bits
c as labels (Listing 2 uses the code bits as labels).

Two reference gradients, independent of each other and of any GPU code:
torch float64 autograd over a plain gather/scatter forward in the tanh form
(``grad_autograd``), and central finite differences of the numpy forward
(``loss_numpy``).
"""
from __future__ import annotations

import numpy as np

from .decoders import LLR_MAX, spa_iteration
from .qc import Graph


def forward_numpy(g: Graph, lam: np.ndarray, w: np.ndarray, llr_max: float = LLR_MAX) -> np.ndarray:
    lam = np.clip(np.asarray(lam, dtype=np.float64), -llr_max, llr_max)
    q = lam[:, g.edge_vn()]
    app = lam
    for t in range(w.shape[0]):
        _, app, q = spa_iteration(g, lam, q, llr_max, w=w[t])
    return app


def bce_with_logits(L: np.ndarray, c: np.ndarray) -> float:
    """mean(softplus(L) - c L)."""
    L = np.asarray(L, dtype=np.float64)
    return float(np.mean(np.logaddexp(0.0, L) - c * L))


def loss_numpy(g: Graph, L_ch: np.ndarray, w: np.ndarray, c: np.ndarray) -> float:
    """Loss as a function of the boundary channel LLRs ``L_ch[B][n_dec]``
    (zeros at untransmitted VNs) and the weights."""
    app = forward_numpy(g, -np.asarray(L_ch, dtype=np.float64), w)
    return bce_with_logits(-app, c)


def grad_autograd(g: Graph, L_ch: np.ndarray, w: np.ndarray, c: np.ndarray,
                  want_margin: bool = False):
    """(loss, dloss/dL_ch, dloss/dw, clamp_hits) by torch float64 autograd;
    with ``want_margin`` also, per codeword, the smallest distance of any
    clamped value (channel input, check output, variable output) to the
    clamp threshold -- where it is small, a single-precision forward may take
    the other side of the clamp, and with it a different derivative.

    The check update is written in the tanh form
    r_v = 2 atanh(prod_{v' != v} tanh(q_v'/2)), whose derivative is finite
    at q = 0 (punctured inputs), unlike the phi form."""
    import torch

    dt = torch.float64
    Z = g.Z
    Lt = torch.tensor(np.asarray(L_ch, dtype=np.float64), dtype=dt, requires_grad=True)
    wt = torch.tensor(np.asarray(w, dtype=np.float64), dtype=dt, requires_grad=True)
    ct = torch.tensor(np.asarray(c, dtype=np.float64), dtype=dt)
    vn = torch.tensor(g.edge_vn(), dtype=torch.long)
    rows = [torch.tensor(g.row_edge_ids(i), dtype=torch.long) for i in range(g.rows)]
    hits = 0
    margin = torch.full((Lt.shape[0],), float("inf"), dtype=dt)

    def near(x):
        return torch.minimum(margin, (x.detach().abs() - LLR_MAX).abs().amin(dim=1))

    lam_raw = -Lt
    hits += int((lam_raw.abs() > LLR_MAX).sum())
    margin = near(lam_raw)
    lam = torch.clamp(lam_raw, -LLR_MAX, LLR_MAX)
    q = lam[:, vn]
    app = lam
    for t in range(wt.shape[0]):
        tq = torch.tanh(q / 2)
        parts = []
        for ids in rows:
            th = tq[:, ids]                                  # (B, d, Z)
            d = th.shape[1]
            outs = []
            for a in range(d):
                keep = [b for b in range(d) if b != a]
                p = torch.prod(th[:, keep, :], dim=1)
                outs.append(2 * torch.atanh(p))
            parts.append((ids, torch.stack(outs, dim=1)))
        # rows hold consecutive canonical edge ids, so concatenation in row
        # order is the canonical order
        r_list = torch.cat([val.reshape(val.shape[0], -1) for _, val in parts], dim=1)
        hits += int((r_list.abs() > LLR_MAX).sum())
        margin = near(r_list)
        r = torch.clamp(r_list, -LLR_MAX, LLR_MAX)
        wr = r * wt[t][None, :]
        app = lam.index_add(1, vn, wr)
        qn = app[:, vn] - wr
        if t + 1 < wt.shape[0]:
            hits += int((qn.abs() > LLR_MAX).sum())
            margin = near(qn)
        q = torch.clamp(qn, -LLR_MAX, LLR_MAX)
    Lp = -app
    loss = torch.mean(torch.nn.functional.softplus(Lp) - ct * Lp)
    loss.backward()
    out = (float(loss.detach()), Lt.grad.numpy().copy(), wt.grad.numpy().copy(), hits)
    return out + (margin.numpy().copy(),) if want_margin else out


def fd_grad(fun, x: np.ndarray, idx: np.ndarray, h: float = 1e-6) -> np.ndarray:
    """Central finite differences of scalar ``fun`` at flat positions ``idx``."""
    out = np.empty(len(idx))
    flat = x.reshape(-1)
    for n, i in enumerate(idx):
        old = flat[i]
        flat[i] = old + h
        fp = fun(x)
        flat[i] = old - h
        fm = fun(x)
        flat[i] = old
        out[n] = (fp - fm) / (2 * h)
    return out
