"""3-D U-Net for the learned warm start (oracle; test infrastructure only).

The network maps the template and reference, resampled to the velocity
grid, to a velocity that starts the Gauss-Newton solve.  This module is the
FP64 reference of its forward and backward passes, used to check the GPU's
hand-written kernels.  Tensors are channel-last, shape (Z, Y, X, C) in 3-D;
every convolution is 3x3x3 with periodic padding (the domain is periodic).

Architecture (channels c = (c0, c1, c2, c3), four resolution levels):
  enc0 = relu(conv(relu(conv(x, 2 -> c0)), c0 -> c0))          at full size
  enc1 = relu(conv(relu(conv(pool(enc0), c0 -> c1)), c1 -> c1)) at 1/2
  enc2 = relu(conv(relu(conv(pool(enc1), c1 -> c2)), c2 -> c2)) at 1/4
  mid  = relu(conv(relu(conv(pool(enc2), c2 -> c3)), c3 -> c3)) at 1/8
  dec2 = relu(conv(cat(up(mid), enc2), c3 + c2 -> c2))
  dec1 = relu(conv(cat(up(dec2), enc1), c2 + c1 -> c1))
  dec0 = relu(conv(cat(up(dec1), enc0), c1 + c0 -> c0))
  out  = scale * conv1x1(dec0, c0 -> 3)
pool = mean of 2x2x2 children; up = nearest-neighbour copy to the children.
Loss: 1/2 mean over voxels and components of (out - target)^2.

Precision: the GPU stores activations (ReLU and pooling outputs, hence all
convolution inputs) and convolution weights in bfloat16 and accumulates in
float32; the 1x1 head runs in float32.  ``quantize=True`` rounds exactly
those tensors to bfloat16 (round to nearest even on the 16 high bits of the
float32 pattern) where the GPU stores them, and treats rounding as the
identity in the backward pass (as the GPU does), so that a comparison
isolates accumulation order from the storage format.
"""

from __future__ import annotations

import numpy as np

OFFSETS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]

LAYERS = ["e0a", "e0b", "e1a", "e1b", "e2a", "e2b", "ma", "mb", "d2", "d1", "d0", "head"]


def layer_shapes(c):
    c0, c1, c2, c3 = c
    io = {"e0a": (2, c0), "e0b": (c0, c0), "e1a": (c0, c1), "e1b": (c1, c1),
          "e2a": (c1, c2), "e2b": (c2, c2), "ma": (c2, c3), "mb": (c3, c3),
          "d2": (c3 + c2, c2), "d1": (c2 + c1, c1), "d0": (c1 + c0, c0), "head": (c0, 3)}
    return {k: ((1 if k == "head" else 27), ci, co) for k, (ci, co) in io.items()}


def init_params(c, seed):
    """He-normal weights W[tap][cin][cout], zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for k, (taps, ci, co) in layer_shapes(c).items():
        std = np.sqrt(2.0 / (taps * ci)) if k != "head" else np.sqrt(1.0 / ci)
        p[k + ".w"] = rng.standard_normal((taps, ci, co)) * std
        p[k + ".b"] = np.zeros(co)
    return p


def bf16(a):
    """Round float64 values to bfloat16 (through float32), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _shift(x, off):
    """y[z, y, x] = x[z + dz, y + dy, x + dx] (periodic)."""
    return np.roll(x, shift=(-off[0], -off[1], -off[2]), axis=(0, 1, 2))


def conv3(x, w, b):
    """out[v] = b + sum_tap x[v + off(tap)] @ W[tap]."""
    out = np.broadcast_to(b, x.shape[:3] + (w.shape[2],)).copy()
    for t, off in enumerate(OFFSETS):
        out += _shift(x, off) @ w[t]
    return out


def conv3_backward(x, w, g):
    """Gradients of conv3 with respect to x, W and b for the output gradient g."""
    gx = np.zeros_like(x)
    gw = np.zeros_like(w)
    for t, off in enumerate(OFFSETS):
        xs = _shift(x, off)
        gw[t] = xs.reshape(-1, x.shape[3]).T @ g.reshape(-1, g.shape[3])
        gx += _shift(g @ w[t].T, (-off[0], -off[1], -off[2]))
    return gx, gw, g.reshape(-1, g.shape[3]).sum(axis=0)


def pool(x):
    Z, Y, X, C = x.shape
    return x.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).mean(axis=(1, 3, 5))


def pool_backward(g):
    return np.repeat(np.repeat(np.repeat(g, 2, axis=0), 2, axis=1), 2, axis=2) / 8.0


def up(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=0), 2, axis=1), 2, axis=2)


def up_backward(g):
    Z, Y, X, C = g.shape
    return g.reshape(Z // 2, 2, Y // 2, 2, X // 2, 2, C).sum(axis=(1, 3, 5))


def forward(params, x, scale=1.0, quantize=False):
    """Returns the output and a cache for backward."""
    P = params
    cache = {}
    q = bf16 if quantize else (lambda a: a)

    def cr(name, inp):
        inp = q(inp)
        pre = conv3(inp, q(P[name + ".w"]), P[name + ".b"])
        cache[name] = (inp, pre)
        return q(np.maximum(pre, 0.0))

    def qpool(a):
        return q(pool(a))

    e0 = cr("e0b", cr("e0a", x))
    e1 = cr("e1b", cr("e1a", qpool(e0)))
    e2 = cr("e2b", cr("e2a", qpool(e1)))
    m = cr("mb", cr("ma", qpool(e2)))
    d2 = cr("d2", np.concatenate([up(m), e2], axis=3))
    d1 = cr("d1", np.concatenate([up(d2), e1], axis=3))
    d0 = cr("d0", np.concatenate([up(d1), e0], axis=3))
    out = scale * (d0 @ P["head.w"][0] + P["head.b"])
    cache["head"] = (d0, None)
    cache["q"] = q
    cache["dims"] = (e0.shape[3], e1.shape[3], e2.shape[3], m.shape[3])
    return out, cache


def loss_and_grad(params, x, target, scale=1.0, quantize=False):
    """1/2 mean (out - target)^2 and its gradient with respect to every parameter.

    With ``quantize`` the backward convolutions also take bfloat16 operands
    (the rounded gradient of the pre-activation and the rounded weights)."""
    out, cache = forward(params, x, scale, quantize)
    q = cache["q"]
    diff = out - target
    loss = 0.5 * float(np.mean(diff * diff))
    g = diff / diff.size * scale
    grads = {}
    d0 = cache["head"][0]
    grads["head.w"] = (d0.reshape(-1, d0.shape[3]).T @ g.reshape(-1, 3))[None]
    grads["head.b"] = g.reshape(-1, 3).sum(axis=0)
    gd0 = g @ params["head.w"][0].T
    c0, c1, c2, c3 = cache["dims"]

    def back(name, gout):
        inp, pre = cache[name]
        gpre = gout * (pre > 0)
        gb_exact = gpre.reshape(-1, gpre.shape[3]).sum(axis=0)
        gx, gw, _ = conv3_backward(inp, q(params[name + ".w"]), q(gpre))
        gb = gb_exact
        grads[name + ".w"] = gw
        grads[name + ".b"] = gb
        return gx

    gcat = back("d0", gd0)
    gd1, ge0 = up_backward(gcat[..., :c1]), gcat[..., c1:]
    gcat = back("d1", gd1)
    gd2, ge1 = up_backward(gcat[..., :c2]), gcat[..., c2:]
    gcat = back("d2", gd2)
    gm, ge2 = up_backward(gcat[..., :c3]), gcat[..., c3:]
    g = back("ma", back("mb", gm))
    ge2 = ge2 + pool_backward(g)
    g = back("e2a", back("e2b", ge2))
    ge1 = ge1 + pool_backward(g)
    g = back("e1a", back("e1b", ge1))
    ge0 = ge0 + pool_backward(g)
    back("e0a", back("e0b", ge0))
    return loss, grads, out
