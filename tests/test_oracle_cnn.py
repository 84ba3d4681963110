"""Pins of the FP64 U-Net oracle (the learned warm start's reference)."""

import numpy as np

from oracle import cnn as C


def test_conv3_direct_loop():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 4, 5, 2))
    w = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(3)
    out = C.conv3(x, w, b)
    ref = np.zeros((3, 4, 5, 3))
    for z in range(3):
        for y in range(4):
            for xx in range(5):
                acc = b.copy()
                t = 0
                for dz in (-1, 0, 1):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            acc += x[(z + dz) % 3, (y + dy) % 4, (xx + dx) % 5] @ w[t]
                            t += 1
                ref[z, y, xx] = acc
    np.testing.assert_allclose(out, ref, atol=1e-12)


def test_pool_up_adjoint():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((4, 6, 8, 3))
    y = rng.standard_normal((2, 3, 4, 3))
    assert abs(np.sum(C.pool(x) * y) - np.sum(x * C.pool_backward(y))) < 1e-12
    assert abs(np.sum(C.up(y) * x) - np.sum(y * C.up_backward(x))) < 1e-12
    np.testing.assert_allclose(C.pool(np.ones((4, 4, 4, 2))), 1.0)


def test_network_gradient_finite_differences():
    rng = np.random.default_rng(2)
    c = (2, 3, 3, 4)
    p = C.init_params(c, seed=3)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((8, 8, 8, 2))
    target = rng.standard_normal((8, 8, 8, 3))
    loss, grads, _ = C.loss_and_grad(p, x, target, scale=0.7)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = C.loss_and_grad(p, x, target, scale=0.7)[0]
            flat[idx] = old - eps
            lm = C.loss_and_grad(p, x, target, scale=0.7)[0]
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            an = grads[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1e-8, abs(fd)) + 1e-10, (k, idx, fd, an)
