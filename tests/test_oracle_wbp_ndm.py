"""Pins of weighted BP, its gradients and the neural demapper.

* Weighted BP with unit weights is flooding sum-product.
* The numpy forward (phi form) and the torch autograd forward (tanh form)
  are independent implementations; their losses agree.
* Autograd gradients equal central finite differences.
* On a tree code with enough iterations the posterior is bitwise MAP, so the
  gradient with respect to the channel LLRs equals the finite-difference
  gradient of the MAP loss.
* Neural demapper: numpy forward equals torch forward, autograd equals
  finite differences, BCE equals torch's binary_cross_entropy_with_logits.
"""
import numpy as np
import pytest
import torch

from inputs import rand
from inputs.workloads import SMALL
from oracle import decoders as D
from oracle import ndm, qc, wbp


def small_setup(T=3, B=2, seed=1):
    qb = SMALL.load()
    g = qc.graph_from_qcbase(qb, 648)
    u = rand.bits(seed, (B, g.k))
    c = qc.encode(qb.base, qb.kb, qb.Z, qb.family, u)[:, :g.n_dec].astype(np.float64)
    L = (2 * c - 1) * 1.2 + rand.gaussian(seed + 1, (B, g.n_dec), scale=1.0)
    w = rand.uniform(seed + 2, (T, g.E), 0.7, 1.3)
    return g, L, w, c


def test_unit_weights_is_spa():
    g, L, w, c = small_setup(T=4)
    a = wbp.forward_numpy(g, -L, np.ones_like(w))
    b = D.spa_flood(g, -L, 4)
    assert np.array_equal(a, b)


def test_numpy_and_autograd_losses_agree():
    g, L, w, c = small_setup(T=3)
    loss_t, _, _, hits = wbp.grad_autograd(g, L, w, c)
    assert hits == 0
    assert abs(loss_t - wbp.loss_numpy(g, L, w, c)) < 1e-10


def test_autograd_equals_finite_differences():
    g, L, w, c = small_setup(T=3)
    _, gL, gw, hits = wbp.grad_autograd(g, L, w, c)
    assert hits == 0
    r = rand.rng(5)
    iw = r.choice(w.size, 12, replace=False)
    iL = r.choice(L.size, 12, replace=False)
    fw = wbp.fd_grad(lambda x: wbp.loss_numpy(g, L, x, c), w.copy(), iw)
    fL = wbp.fd_grad(lambda x: wbp.loss_numpy(g, x, w, c), L.copy(), iL)
    assert np.allclose(gw.reshape(-1)[iw], fw, rtol=1e-5, atol=1e-9)
    assert np.allclose(gL.reshape(-1)[iL], fL, rtol=1e-5, atol=1e-9)


def test_tree_gradient_is_map_gradient():
    from tests.test_oracle_decoders import map_llr, tiny_graph
    g = tiny_graph([[3, 1, -1], [-1, 4, 2]], 5)
    L = rand.gaussian(21, (2, g.n_dec), scale=1.0)
    c = rand.bits(22, (2, g.n_dec)).astype(np.float64)
    w = np.ones((4, g.E))
    _, gL, _, _ = wbp.grad_autograd(g, L, w, c)

    def map_loss(x):
        return wbp.bce_with_logits(map_llr(g, x), c)

    idx = np.arange(L.size)
    fd = wbp.fd_grad(map_loss, L.copy(), idx)
    assert np.allclose(gL.reshape(-1), fd, rtol=1e-5, atol=1e-9)


def test_gradient_linear_in_upstream():
    params = rand.gaussian(30, ndm.N_PARAMS, scale=0.2)
    y = rand.gaussian(31, (3, 10)) + 1j * rand.gaussian(32, (3, 10))
    n0 = rand.uniform(33, 3, 0.2, 1.0)
    g1 = rand.gaussian(34, (3, 40))
    g2 = rand.gaussian(35, (3, 40))
    a = ndm.grad_params(params, y, n0, g1) * 2.0 + ndm.grad_params(params, y, n0, g2)
    b = ndm.grad_params(params, y, n0, 2.0 * g1 + g2)
    assert np.allclose(a, b, rtol=1e-10, atol=1e-12)


def test_ndm_numpy_equals_torch_and_fd():
    params = rand.gaussian(40, ndm.N_PARAMS, scale=0.3)
    y = rand.gaussian(41, (2, 8)) + 1j * rand.gaussian(42, (2, 8))
    n0 = rand.uniform(43, 2, 0.2, 1.0)
    a = ndm.forward_numpy(params, y, n0)
    b = ndm.forward_torch(torch.tensor(params), y, n0).numpy()
    assert np.allclose(a, b, rtol=1e-12, atol=1e-12)
    gl = rand.gaussian(44, a.shape)
    g = ndm.grad_params(params, y, n0, gl)
    idx = rand.rng(45).choice(ndm.N_PARAMS, 20, replace=False)
    fd = wbp.fd_grad(lambda p: float((ndm.forward_numpy(p, y, n0) * gl).sum()), params.copy(), idx)
    assert np.allclose(g[idx], fd, rtol=1e-5, atol=1e-8)


def test_bce_matches_torch():
    L = rand.gaussian(50, (4, 30), scale=5.0)
    c = rand.bits(51, (4, 30)).astype(np.float64)
    ref = torch.nn.functional.binary_cross_entropy_with_logits(torch.tensor(L), torch.tensor(c)).item()
    assert abs(wbp.bce_with_logits(L, c) - ref) < 1e-12
