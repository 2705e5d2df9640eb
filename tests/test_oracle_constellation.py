"""Pins of the trainable-constellation oracle: the initial points are the
mapper's pinned Gray QAM, normalisation is scale invariant, and the
autograd gradients agree with central finite differences."""
import numpy as np

from inputs import rand
from oracle import constellation as oc
from oracle import modem, ndm


def _glorot(seed):
    r = rand.rng(seed)
    out = []
    for fo, fi in ((64, 3), (64, 64), (4, 64)):
        lim = np.sqrt(6.0 / (fi + fo))
        out.append(r.uniform(-lim, lim, fo * fi))
        out.append(np.zeros(fo))
    return np.concatenate(out)


def test_initial_points_are_the_mapper():
    for m in (2, 4, 6):
        p = oc.qam_points(m)
        t = rand.bits(1, (3, 12 * m))
        got = oc.map_points(p, t, m)
        assert np.allclose(got, modem.map_bits(t, m), atol=1e-15)
        assert abs((p ** 2).sum() / len(p) - 1.0) < 1e-12


def test_labels_first_bit_most_significant():
    t = np.array([[1, 0, 0, 0, 0, 0, 1, 1]], dtype=np.uint8)
    assert oc.labels_of(t, 4).tolist() == [[8, 3]]


def test_normalisation_is_scale_invariant_and_gradient_orthogonal():
    m = 4
    p = oc.qam_points(m) + rand.gaussian(2, (16, 2), scale=0.2)
    t = rand.bits(3, (2, 40 * m))
    assert np.allclose(oc.map_points(p, t, m), oc.map_points(3.7 * p, t, m))
    gy = rand.gaussian(4, (2, 40, 2))
    g = oc.points_vjp(p, t, m, gy)
    # the map does not change along p, so the gradient has no radial part
    assert abs((g * p).sum()) < 1e-12 * max(1.0, np.abs(g).sum())


def _fd(f, x, h=1e-6):
    g = np.zeros_like(x)
    for i in np.ndindex(x.shape):
        d = np.zeros_like(x)
        d[i] = h
        g[i] = (f(x + d) - f(x - d)) / (2 * h)
    return g


def test_points_gradient_matches_finite_differences():
    m, B, S = 4, 2, 6
    params = _glorot(5)
    p = oc.qam_points(m) + rand.gaussian(6, (16, 2), scale=0.1)
    t = rand.bits(7, (B, S * m))
    n0 = np.array([0.3, 0.6])
    g = rand.gaussian(8, (B, S)) + 1j * rand.gaussian(9, (B, S))
    _, gp, gw = oc.loss_and_grads(p, params, t, m, n0, g)

    def loss_p(pp):
        return oc.loss_and_grads(pp, params, t, m, n0, g)[0]

    assert np.allclose(gp, _fd(loss_p, p), rtol=1e-5, atol=1e-8)
    # parameter gradient equals the demapper's own (pinned) autograd
    y = oc.map_points(p, t, m) + np.sqrt(n0[:, None] / 2) * g
    llr = ndm.forward_numpy(params, y, n0)
    gl = (1 / (1 + np.exp(-llr)) - t) / t.size
    assert np.allclose(gw, ndm.grad_params(params, y, n0, gl), rtol=1e-9, atol=1e-12)


def test_ndm_input_gradient_matches_finite_differences():
    params = _glorot(10)
    B, S = 2, 5
    y = rand.gaussian(11, (B, S)) + 1j * rand.gaussian(12, (B, S))
    n0 = np.array([0.2, 0.9])
    gl = rand.gaussian(13, (B, S * 4))
    gy = oc.ndm_input_vjp(params, y, n0, gl)

    def f_re(v):
        return float((ndm.forward_numpy(params, v.reshape(B, S) + 1j * y.imag, n0) * gl).sum())

    def f_im(v):
        return float((ndm.forward_numpy(params, y.real + 1j * v.reshape(B, S), n0) * gl).sum())

    assert np.allclose(gy[..., 0], _fd(f_re, y.real.copy()).reshape(B, S), rtol=1e-5, atol=1e-8)
    assert np.allclose(gy[..., 1], _fd(f_im, y.imag.copy()).reshape(B, S), rtol=1e-5, atol=1e-8)


def test_keep_mask_drops_symbols_from_the_gradient_only():
    m, B, S = 4, 2, 5
    params = _glorot(11)
    p = oc.qam_points(m)
    t = rand.bits(12, (B, S * m))
    n0 = np.array([0.4, 0.7])
    g = rand.gaussian(13, (B, S)) + 1j * rand.gaussian(14, (B, S))
    full = oc.loss_and_grads(p, params, t, m, n0, g)
    same = oc.loss_and_grads(p, params, t, m, n0, g, keep=np.ones((B, S), bool))
    none = oc.loss_and_grads(p, params, t, m, n0, g, keep=np.zeros((B, S), bool))
    assert same[0] == full[0] and np.array_equal(same[1], full[1]) and np.array_equal(same[2], full[2])
    assert none[0] == full[0] and not none[1].any() and not none[2].any()
    # dropping one symbol removes exactly its own contribution (linearity)
    keep = np.ones((B, S), bool)
    keep[1, 3] = False
    part = oc.loss_and_grads(p, params, t, m, n0, g, keep=keep)
    only = oc.loss_and_grads(p, params, t, m, n0, g, keep=~keep)
    assert np.allclose(part[2] + only[2], full[2], atol=1e-15)
    assert np.allclose(part[1] + only[1], full[1], atol=1e-15)
