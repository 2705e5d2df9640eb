"""Neural demapper and its reference gradient (torch float64 on the CPU).

The paper's Listing 3 defines a neural demapper as a small dense network fed
[Re y, Im y, no] per symbol that outputs one LLR per bit, and Listing 2
trains it with a binary cross-entropy on logits against the code bits.  The
network here has the input [Re y, Im y, ln N0] and layers 3 -> 64 -> 64 -> 4
with ReLU, linear output.

Flat parameter layout (4676 floats): W1[64][3], b1[64], W2[64][64], b2[64],
W3[4][64], b3[4]; a layer computes W x + b.
"""
from __future__ import annotations

import numpy as np

SIZES = [(64, 3), (64,), (64, 64), (64,), (4, 64), (4,)]
N_PARAMS = sum(int(np.prod(s)) for s in SIZES)


def unpack(p):
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def forward_torch(params, y, n0):
    """LLRs ``[B][S*4]`` (float64 torch) from symbols ``y[B][S]`` complex."""
    import torch

    yr = torch.as_tensor(np.real(y), dtype=torch.float64)
    yi = torch.as_tensor(np.imag(y), dtype=torch.float64)
    return forward_torch_xy(params, yr, yi, n0)


def forward_torch_xy(params, yr, yi, n0):
    """As ``forward_torch`` with the symbol's real and imaginary parts given
    as float64 torch tensors (so gradients can flow into them)."""
    import torch

    W1, b1, W2, b2, W3, b3 = unpack(params)
    ln0 = torch.log(torch.as_tensor(np.asarray(n0, dtype=np.float64))).reshape(-1, 1).expand_as(yr)
    x = torch.stack([yr, yi, ln0], dim=-1)                   # (B, S, 3)
    h1 = torch.relu(x @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    out = h2 @ W3.T + b3                                     # (B, S, 4)
    return out.reshape(out.shape[0], -1)


def forward_numpy(params: np.ndarray, y: np.ndarray, n0: np.ndarray) -> np.ndarray:
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(params, dtype=np.float64))
    ln0 = np.broadcast_to(np.log(np.asarray(n0, dtype=np.float64)).reshape(-1, 1), y.shape)
    x = np.stack([y.real, y.imag, ln0], axis=-1)
    h1 = np.maximum(x @ W1.T + b1, 0)
    h2 = np.maximum(h1 @ W2.T + b2, 0)
    out = h2 @ W3.T + b3
    return out.reshape(out.shape[0], -1)


def grad_params(params: np.ndarray, y: np.ndarray, n0: np.ndarray, gllr: np.ndarray) -> np.ndarray:
    """Vector-Jacobian product d<gllr, NDM(y)>/dparams by autograd."""
    import torch

    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    out = forward_torch(p, y, n0)
    (out * torch.as_tensor(np.asarray(gllr, dtype=np.float64))).sum().backward()
    return p.grad.numpy().copy()
