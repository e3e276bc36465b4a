"""Pins for the reference network layers (the learned warm start's building
blocks): convolution against SciPy's correlation, gradients against central
finite differences, Adam against its closed form."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import net


def test_conv3d_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 5, 4, 6))
    w = rng.normal(size=(4, 3, 3, 3, 3))
    b = rng.normal(size=4)
    out = net.conv3d(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = sum(correlate(x[n, i], w[o, i], mode="same") for i in range(3)) + b[o]
            assert np.allclose(out[n, o], ref, rtol=1e-12, atol=1e-12)


def test_conv3d_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 2, 4, 3, 5))
    w = rng.normal(size=(3, 2, 3, 3, 3))
    b = rng.normal(size=3)
    g = rng.normal(size=(1, 3, 4, 3, 5))
    dx, dw, db = net.conv3d_backward(x, w, g)
    f = lambda x_, w_, b_: float((net.conv3d(x_, w_, b_) * g).sum())
    h = 1e-6
    for idx in [(0, 0, 1, 1, 2), (0, 1, 3, 2, 4), (0, 0, 0, 0, 0)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        assert dx[idx] == pytest.approx((f(xp, w, b) - f(xm, w, b)) / (2 * h), rel=1e-7, abs=1e-8)
    for idx in [(0, 0, 1, 1, 1), (2, 1, 0, 2, 1)]:
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        assert dw[idx] == pytest.approx((f(x, wp, b) - f(x, wm, b)) / (2 * h), rel=1e-7, abs=1e-8)
    assert np.allclose(db, g.sum(axis=(0, 2, 3, 4)))


def test_network_backward_finite_differences():
    rng = np.random.default_rng(2)
    params = net.init_params([2, 4, 4, 3], seed=3)
    x = rng.normal(size=(2, 2, 4, 4, 4))
    tgt = rng.normal(size=(2, 3, 4, 4, 4))
    mask = rng.random((2, 3, 4, 4, 4)) < 0.8

    def loss(ps):
        out, _ = net.forward(ps, x)
        return net.mse(out, tgt, mask)[0]

    out, acts = net.forward(params, x)
    _, dl = net.mse(out, tgt, mask)
    grads = net.backward(params, acts, dl)
    h = 1e-6
    for k, idx in [(0, (1, 0, 1, 2, 0)), (1, (3, 2, 0, 0, 1)), (2, (0, 3, 2, 1, 1))]:
        w, b = params[k]
        wp, wm = w.copy(), w.copy()
        wp[idx] += h
        wm[idx] -= h
        pp = [(wp, b) if j == k else params[j] for j in range(len(params))]
        pm = [(wm, b) if j == k else params[j] for j in range(len(params))]
        fd = (loss(pp) - loss(pm)) / (2 * h)
        assert grads[k][0][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_adam_first_step_is_signed_lr():
    """With zero moments, step 1 moves every parameter by lr * g / (|g| + eps')."""
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = net.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12)
