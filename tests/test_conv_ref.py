"""Pins of the FP64 conv3d reference (the gradient oracle of the surrogate's
kernels): a direct per-voxel loop, finite differences, and adjointness."""
import numpy as np

from oracle import conv3d_ref as R


def _direct(x, w, b):
    D, H, W, Ci = x.shape
    out = np.zeros((D, H, W, w.shape[2]))
    for z in range(D):
        for y in range(H):
            for xx in range(W):
                acc = b.copy()
                for t, (dz, dy, dx) in enumerate(R.OFFSETS):
                    zz, yy, x2 = z + dz, y + dy, xx + dx
                    if 0 <= zz < D and 0 <= yy < H and 0 <= x2 < W:
                        acc = acc + x[zz, yy, x2] @ w[t]
                out[z, y, xx] = acc
    return out


def test_conv_matches_direct_loop():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 4, 5, 2))
    w = rng.normal(size=(27, 2, 3))
    b = rng.normal(size=3)
    np.testing.assert_allclose(R.conv3d(x, w, b), _direct(x, w, b), rtol=1e-13, atol=1e-13)


def test_backward_is_adjoint_and_matches_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 4, 4, 2))
    w = rng.normal(size=(27, 2, 3))
    b = rng.normal(size=3)
    g = rng.normal(size=(3, 4, 4, 3))
    dx, dw, db = R.conv3d_backward(x, w, g)
    # <g, conv(x)> = <dx, x> (linear in x without bias)
    assert abs(np.sum(g * R.conv3d(x, w)) - np.sum(dx * x)) < 1e-10
    f = lambda xx, ww, bb: np.sum(g * R.conv3d(xx, ww, bb))
    eps = 1e-6
    for idx in [(0, 1, 2, 1), (2, 3, 0, 0), (1, 0, 3, 1)]:
        e = np.zeros_like(x); e[idx] = eps
        assert abs((f(x + e, w, b) - f(x - e, w, b)) / (2 * eps) - dx[idx]) < 1e-6
    for idx in [(0, 0, 0), (13, 1, 2), (26, 0, 1), (4, 1, 0)]:
        e = np.zeros_like(w); e[idx] = eps
        assert abs((f(x, w + e, b) - f(x, w - e, b)) / (2 * eps) - dw[idx]) < 1e-6
    e = np.zeros_like(b); e[1] = eps
    assert abs((f(x, w, b + e) - f(x, w, b - e)) / (2 * eps) - db[1]) < 1e-6


def test_network_gradients_match_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 3, 4, 2))
    layers = [(rng.normal(size=(27, 2, 4)) * 0.3, rng.normal(size=4) * 0.1),
              (rng.normal(size=(27, 4, 4)) * 0.3, rng.normal(size=4) * 0.1),
              (rng.normal(size=(27, 4, 1)) * 0.3, rng.normal(size=1) * 0.1)]
    target = rng.normal(size=(3, 3, 4))
    loss, grads = R.loss_and_grads(x, layers, target)
    eps = 1e-6
    for li, idx in [(0, (5, 1, 2)), (1, (13, 3, 0)), (2, (20, 2, 0))]:
        w, b = layers[li]
        wp = w.copy(); wp[idx] += eps
        wm = w.copy(); wm[idx] -= eps
        Lp = R.loss_and_grads(x, [l if k != li else (wp, b) for k, l in enumerate(layers)], target)[0]
        Lm = R.loss_and_grads(x, [l if k != li else (wm, b) for k, l in enumerate(layers)], target)[0]
        assert abs((Lp - Lm) / (2 * eps) - grads[li][0][idx]) < 1e-6 * max(1.0, abs(grads[li][0][idx]))


def test_adamw_first_step_is_signed_lr():
    """With m = v = 0 the first bias-corrected step is lr * g / (|g| + eps)."""
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 0.0])
    w1, m, v = R.adamw(w, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-12)
    np.testing.assert_allclose(w1, w - 0.01 * np.sign(g), atol=1e-10)


def test_adamw_weight_decay_is_decoupled():
    """Decoupled weight decay (Loshchilov & Hutter): the decay term lr wd w is
    added to the step outside the adaptive moments.  With a constant gradient
    the bias-corrected moments are exactly g and g^2, so every step is
    w <- w (1 - lr wd) - lr g / (|g| + eps), a closed-form recurrence."""
    w0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -0.1, 0.0, 2.0])
    lr, wd, eps = 0.05, 0.4, 1e-12
    w, m, v = w0.copy(), np.zeros(4), np.zeros(4)
    expect = w0.copy()
    for step in range(1, 6):
        w, m, v = R.adamw(w, g, m, v, step, lr=lr, eps=eps, wd=wd)
        expect = expect * (1 - lr * wd) - lr * g / (np.abs(g) + eps)
        np.testing.assert_allclose(w, expect, rtol=1e-12, atol=1e-14)
    # the moments do not see the decay
    _, m0, v0 = R.adamw(w0, g, np.zeros(4), np.zeros(4), 1, lr=lr, eps=eps, wd=0.0)
    _, m1, v1 = R.adamw(w0, g, np.zeros(4), np.zeros(4), 1, lr=lr, eps=eps, wd=wd)
    np.testing.assert_array_equal(m0, m1)
    np.testing.assert_array_equal(v0, v1)
    # with zero gradient only the decay acts: w (1 - lr wd) exactly
    wz, _, _ = R.adamw(w0, np.zeros(4), np.zeros(4), np.zeros(4), 1, lr=lr, eps=1e-8, wd=wd)
    np.testing.assert_allclose(wz, w0 * (1 - lr * wd), rtol=1e-15)
