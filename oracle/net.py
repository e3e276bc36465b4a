"""Reference 3-D convolutional network for the learned warm start (test
infrastructure; nothing in the product path imports this module).

The learned part is not in the paper: a small fully convolutional network
maps per-cell inputs (density, previous displacement, coordinates) on a
regular grid to a displacement prediction.  Only the building blocks are
pinned here (forward and backward of every layer, the loss and the Adam
step); the quality of a trained network's outputs is PARITY UNPINNED - it is
judged through the plain FP64 solve it warm-starts (iterations and residual).

Layout: activations (B, C, Z, Y, X) float64; weights (Cout, Cin, 3, 3, 3);
every convolution is 3x3x3, stride 1, zero padding 1 ("same").
"""
from __future__ import annotations

import numpy as np


def conv3d(x, w, b):
    """out[n, o, z, y, x] = b[o] + sum_{i, dz, dy, dx} w[o, i, dz, dy, dx] x[n, i, z+dz-1, y+dy-1, x+dx-1]."""
    B, C, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    out = np.zeros((B, w.shape[0], Z, Y, X))
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sl = xp[:, :, dz:dz + Z, dy:dy + Y, dx:dx + X]
                out += np.einsum("oi,nizyx->nozyx", w[:, :, dz, dy, dx], sl)
    return out + b[None, :, None, None, None]


def conv3d_backward(x, w, dout):
    """Gradients of conv3d with respect to x, w and b."""
    B, C, Z, Y, X = x.shape
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sl = xp[:, :, dz:dz + Z, dy:dy + Y, dx:dx + X]
                dw[:, :, dz, dy, dx] = np.einsum("nozyx,nizyx->oi", dout, sl)
                dxp[:, :, dz:dz + Z, dy:dy + Y, dx:dx + X] += np.einsum("oi,nozyx->nizyx", w[:, :, dz, dy, dx], dout)
    return dxp[:, :, 1:-1, 1:-1, 1:-1], dw, dout.sum(axis=(0, 2, 3, 4))


def relu(x):
    return np.maximum(x, 0.0)


def init_params(channels, seed):
    """He-style init: w ~ N(0, 2 / (27 Cin)), b = 0 (numpy RNG; the library
    draws its own weights, tests copy them across)."""
    rng = np.random.default_rng(seed)
    params = []
    for ci, co in zip(channels[:-1], channels[1:]):
        w = rng.normal(0.0, np.sqrt(2.0 / (27 * ci)), size=(co, ci, 3, 3, 3))
        params.append((w, np.zeros(co)))
    return params


def forward(params, x, skip_from=None):
    """Conv layers with ReLU between them (none after the last); with
    skip_from, the output adds input channels [skip_from, skip_from + C_out).
    Returns the output and the per-layer inputs needed by backward."""
    acts = [x]
    h = x
    for k, (w, b) in enumerate(params):
        h = conv3d(h, w, b)
        if k + 1 < len(params):
            h = relu(h)
        acts.append(h)
    if skip_from is not None:
        h = h + x[:, skip_from:skip_from + h.shape[1]]
    return h, acts


def backward(params, acts, dout, skip_from=None, return_dx=False):
    """Parameter gradients (and, with return_dx, the input gradient)."""
    grads = [None] * len(params)
    g = dout
    for k in range(len(params) - 1, -1, -1):
        w, b = params[k]
        if k + 1 < len(params):
            g = g * (acts[k + 1] > 0)
        dx, dw, db = conv3d_backward(acts[k], w, g)
        grads[k] = (dw, db)
        g = dx
    if not return_dx:
        return grads
    if skip_from is not None:
        g = g.copy()
        g[:, skip_from:skip_from + dout.shape[1]] += dout
    return grads, g


def mse(pred, target, mask):
    """L = sum(mask (pred - target)^2) / sum(mask) and dL/dpred."""
    m = mask.astype(np.float64)
    d = (pred - target) * m
    n = max(m.sum(), 1.0)
    return float((d * d).sum() / n), 2.0 * d / n


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
