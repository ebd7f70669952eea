"""FP64 CPU reference of the surrogate's 3-D convolution network.

TEST INFRASTRUCTURE ONLY: the test-suite uses it to check the HIP conv3d
kernels; the product path never calls it.  It shares no code with them.

Conventions (the same ones the kernels document): activations are
channels-last arrays x[z, y, x, c]; a layer's weight is w[tap, ci, co] with
tap = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1) for offsets dz, dy, dx in
{-1, 0, 1}; zero padding ("same" size);

    out[v, co] = bias[co] + sum_{tap, ci} w[tap, ci, co] x[v + offset(tap), ci].

Everything is written as plain loops over the 27 taps with numpy slicing, in
float64.
"""
from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shifted(x, dz, dy, dx):
    """s[z, y, x] = x[z + dz, y + dy, x + dx], zero outside."""
    D, H, W = x.shape[:3]
    s = np.zeros_like(x)
    zs, ys, xs = slice(max(0, -dz), D - max(0, dz)), slice(max(0, -dy), H - max(0, dy)), \
        slice(max(0, -dx), W - max(0, dx))
    zt, yt, xt = slice(max(0, dz), D - max(0, -dz)), slice(max(0, dy), H - max(0, -dy)), \
        slice(max(0, dx), W - max(0, -dx))
    s[zs, ys, xs] = x[zt, yt, xt]
    return s


def conv3d(x, w, bias=None):
    """x [D,H,W,Ci], w [27,Ci,Co], bias [Co] -> [D,H,W,Co] (float64)."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    out = np.zeros(x.shape[:3] + (w.shape[2],))
    for t, (dz, dy, dx) in enumerate(OFFSETS):
        out += _shifted(x, dz, dy, dx) @ w[t]
    if bias is not None:
        out += np.asarray(bias, np.float64)
    return out


def conv3d_backward(x, w, g):
    """Gradients of L = sum(g * conv3d(x, w, b)): (dx, dw, db), float64."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    g = np.asarray(g, np.float64)
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dz, dy, dx_) in enumerate(OFFSETS):
        xs = _shifted(x, dz, dy, dx_)
        dw[t] = xs.reshape(-1, x.shape[3]).T @ g.reshape(-1, g.shape[3])
        dx += _shifted(g @ w[t].T, -dz, -dy, -dx_)
    db = g.reshape(-1, g.shape[3]).sum(axis=0)
    return dx, dw, db


def forward(x, layers):
    """The network: conv, ReLU after every layer but the last.
    layers: list of (w, b).  Returns the list of layer outputs (post-ReLU)."""
    outs = []
    h = np.asarray(x, np.float64)
    for i, (w, b) in enumerate(layers):
        h = conv3d(h, w, b)
        if i + 1 < len(layers):
            h = np.maximum(h, 0.0)
        outs.append(h)
    return outs


def loss_and_grads(x, layers, target):
    """MSE loss mean((y[..., 0] - target)^2) and the gradients of every layer."""
    outs = forward(x, layers)
    y = outs[-1][..., 0]
    n = y.size
    loss = float(np.mean((y - target) ** 2))
    g = np.zeros_like(outs[-1])
    g[..., 0] = 2.0 * (y - target) / n
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        xin = x if i == 0 else outs[i - 1]
        dx, dw, db = conv3d_backward(xin, layers[i][0], g)
        grads[i] = (dw, db)
        if i > 0:
            g = dx * (outs[i - 1] > 0.0)
    return loss, grads


def adamw(w, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    """One AdamW step (decoupled weight decay, bias-corrected moments), float64."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    w = w - lr * (mh / (np.sqrt(vh) + eps) + wd * w)
    return w, m, v
