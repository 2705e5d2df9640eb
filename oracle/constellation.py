"""Trainable constellation (end-to-end learning with the neural demapper).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this package.

The paper makes the constellation of the mapper trainable and replaces the
demapper by the neural demapper, then trains both jointly on the binary
cross-entropy between the coded bits and the demapper's LLRs, with the
gradient from automatic differentiation (Sec. III-C "Hello, World!",
Listings 2 and 3).  Here:

* points ``p[K][2]`` (real, imaginary), K = 2^m, indexed by the label of m
  coded bits read first-bit-most-significant, initialised with the Gray QAM
  of the mapper;
* the mapper uses the points scaled to unit average energy,
  ``x_k = p_k / sqrt(mean_j |p_j|^2)`` (reading: the paper fixes no
  normalisation; unit energy keeps Eb/N0 meaningful while training);
* ``y = x + sqrt(N0/2) g`` with the same standard normals as the AWGN
  channel, the neural demapper of ``oracle.ndm`` and the mean binary
  cross-entropy on logits.

Gradients come from float64 torch autograd.
"""
from __future__ import annotations

import numpy as np

from . import modem, ndm


def qam_points(m: int) -> np.ndarray:
    """``float64[2^m][2]``: the mapper's Gray QAM, by label."""
    c = modem.constellation(m)
    return np.stack([c.real, c.imag], axis=-1)


def labels_of(t: np.ndarray, m: int) -> np.ndarray:
    """Labels ``int64[B][S]`` of coded bits ``u8[B][S*m]`` (first bit MSB)."""
    t = np.asarray(t, dtype=np.int64)
    B, n = t.shape
    b = t.reshape(B, n // m, m)
    w = 1 << np.arange(m - 1, -1, -1)
    return (b * w).sum(-1)


def normalize(p: np.ndarray) -> np.ndarray:
    p = np.asarray(p, dtype=np.float64)
    return p / np.sqrt((p ** 2).sum() / p.shape[0])


def map_points(p: np.ndarray, t: np.ndarray, m: int) -> np.ndarray:
    """Symbols ``complex128[B][S]`` of coded bits with the (normalised) points."""
    x = normalize(p)[labels_of(t, m)]
    return x[..., 0] + 1j * x[..., 1]


def _torch_chain(p, params, t, m, n0, g):
    import torch

    K = p.shape[0]
    x = p / torch.sqrt((p ** 2).sum() / K)
    lab = torch.as_tensor(labels_of(t, m))
    xs = x[lab]                                              # (B, S, 2)
    sig = torch.sqrt(torch.as_tensor(np.asarray(n0, dtype=np.float64) / 2.0)).reshape(-1, 1)
    yr = xs[..., 0] + sig * torch.as_tensor(np.real(g))
    yi = xs[..., 1] + sig * torch.as_tensor(np.imag(g))
    return yr, yi


def loss_and_grads(p: np.ndarray, params: np.ndarray, t: np.ndarray, m: int, n0: np.ndarray,
                   g: np.ndarray, keep: np.ndarray | None = None):
    """(loss, d loss / d points ``[K][2]``, d loss / d params) of the mean BCE
    between coded bits ``t`` and the demapper LLRs; ``g`` complex standard
    normals ``[B][S]`` (E|g|^2 = 2).  Symbols where ``keep`` (bool ``[B][S]``)
    is False count in the loss but not in the gradients."""
    import torch

    pt = torch.tensor(np.asarray(p, dtype=np.float64), requires_grad=True)
    wt = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    yr, yi = _torch_chain(pt, wt, t, m, n0, g)
    llr = ndm.forward_torch_xy(wt, yr, yi, n0)
    tt = torch.as_tensor(np.asarray(t, dtype=np.float64))
    terms = torch.nn.functional.softplus(llr) - tt * llr
    loss = terms.mean()
    if keep is not None:
        B, S = np.shape(keep)
        w = torch.as_tensor(np.repeat(np.asarray(keep, dtype=np.float64), m, axis=1).reshape(B, S * m))
        (terms * w).sum().div(terms.numel()).backward()
    else:
        loss.backward()
    return float(loss.detach()), pt.grad.numpy(), wt.grad.numpy()


def points_vjp(p: np.ndarray, t: np.ndarray, m: int, gy: np.ndarray) -> np.ndarray:
    """d <gy, y(points)> / d points for ``gy[B][S][2]`` (the mapper's
    adjoint alone; the noise does not depend on the points)."""
    import torch

    pt = torch.tensor(np.asarray(p, dtype=np.float64), requires_grad=True)
    K = pt.shape[0]
    x = pt / torch.sqrt((pt ** 2).sum() / K)
    xs = x[torch.as_tensor(labels_of(t, m))]
    (xs * torch.as_tensor(np.asarray(gy, dtype=np.float64))).sum().backward()
    return pt.grad.numpy()


def ndm_input_vjp(params: np.ndarray, y: np.ndarray, n0: np.ndarray, gllr: np.ndarray) -> np.ndarray:
    """d <gllr, NDM(y)> / d (Re y, Im y) as ``float64[B][S][2]``."""
    import torch

    yr = torch.tensor(np.real(y).astype(np.float64), requires_grad=True)
    yi = torch.tensor(np.imag(y).astype(np.float64), requires_grad=True)
    out = ndm.forward_torch_xy(torch.as_tensor(np.asarray(params, dtype=np.float64)), yr, yi, n0)
    (out * torch.as_tensor(np.asarray(gllr, dtype=np.float64))).sum().backward()
    return np.stack([yr.grad.numpy(), yi.grad.numpy()], axis=-1)
