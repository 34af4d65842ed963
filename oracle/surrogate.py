"""FP64 forward/backward of the surrogate network (test infrastructure only).

The surrogate maps 21 Noll coefficients (waves) and a defocus z (nm) to a 64 x 64
intensity crop.  Features: x = (c_1..c_21 / 0.05, z / 1000).  Layers:

    h1 = relu(x W1 + b1)          22   -> 1024
    h2 = relu(h1 W2 + b2)         1024 -> 1024
    h3 = relu(h2 W3 + b3)         1024 -> 1024 = 16 x 8 x 8
    d1 = relu(T(h3; K1) + c1)     16 x 8 x 8   -> 16 x 16 x 16
    d2 = relu(T(d1; K2) + c2)     16 x 16 x 16 -> 8 x 32 x 32
    yd = T(d2; K3) + c3           8 x 32 x 32  -> 1 x 64 x 64
    a  = h3 Wa + ba               1024 -> 256          (linear)
    yb = a Wb + bb                256  -> 4096 = 64 x 64 (linear: a learned basis of crops)
    y  = yd + yb

T is the stride-2 transposed convolution with 4 x 4 kernels and one pixel of
padding: out[co, oy, ox] = sum_{ci, ky, kx} in[ci, iy, ix] K[ci, co, ky, kx] with
oy = 2 iy - 1 + ky, ox = 2 ix - 1 + kx.  Weights W are (in, out); K are
(in, out, 4, 4).  The loss is the mean squared error to the target crop.
This is a network of this project's design (the paper has none); the oracle is its
definition written out, layer by layer.
"""
from __future__ import annotations

import numpy as np

FEATURE_SCALE_C = 0.05
FEATURE_SCALE_Z = 1000.0
DENSE = [(22, 1024), (1024, 1024), (1024, 1024)]
DECONV = [(16, 16), (16, 8), (8, 1)]
BASIS = 256          # rank of the linear crop basis
KEYS = ("W1", "b1", "W2", "b2", "W3", "b3", "K1", "c1", "K2", "c2", "K3", "c3", "Wa", "ba", "Wb", "bb")


def features(coeffs, z):
    c = np.asarray(coeffs, dtype=np.float64)
    return np.concatenate([c[:, :21] / FEATURE_SCALE_C, (np.asarray(z, dtype=np.float64) / FEATURE_SCALE_Z)[:, None]],
                          axis=1)


def init_params(seed: int):
    rng = np.random.default_rng(seed)
    p = {}
    for i, (a, b) in enumerate(DENSE, start=1):
        p[f"W{i}"] = rng.normal(0.0, np.sqrt(2.0 / a), (a, b))
        p[f"b{i}"] = np.zeros(b)
    for i, (a, b) in enumerate(DECONV, start=1):
        p[f"K{i}"] = rng.normal(0.0, np.sqrt(2.0 / (a * 4)), (a, b, 4, 4))
        p[f"c{i}"] = np.zeros(b)
    p["Wa"] = rng.normal(0.0, np.sqrt(1.0 / 1024), (1024, BASIS))
    p["ba"] = np.zeros(BASIS)
    p["Wb"] = rng.normal(0.0, np.sqrt(1.0 / BASIS), (BASIS, 4096))
    p["bb"] = np.zeros(4096)
    return p


def deconv(x, K, bias):
    """Stride-2 transposed convolution, kernel 4, padding 1: (B, Ci, H, W) -> (B, Co, 2H, 2W)."""
    B, Ci, H, W = x.shape
    Co = K.shape[1]
    full = np.zeros((B, Co, 2 * H + 2, 2 * W + 2))           # output with a 1-pixel border
    for ky in range(4):
        for kx in range(4):
            contrib = np.einsum("bihw,io->bohw", x, K[:, :, ky, kx])
            full[:, :, ky:ky + 2 * H:2, kx:kx + 2 * W:2] += contrib
    return full[:, :, 1:2 * H + 1, 1:2 * W + 1] + bias[None, :, None, None]


def deconv_backward(x, K, dout):
    """Gradients (dx, dK, dbias) of deconv for the upstream gradient dout (B, Co, 2H, 2W)."""
    B, Ci, H, W = x.shape
    Co = K.shape[1]
    dfull = np.zeros((B, Co, 2 * H + 2, 2 * W + 2))
    dfull[:, :, 1:2 * H + 1, 1:2 * W + 1] = dout
    dx = np.zeros_like(x)
    dK = np.zeros_like(K)
    for ky in range(4):
        for kx in range(4):
            g = dfull[:, :, ky:ky + 2 * H:2, kx:kx + 2 * W:2]   # (B, Co, H, W)
            dx += np.einsum("bohw,io->bihw", g, K[:, :, ky, kx])
            dK[:, :, ky, kx] = np.einsum("bihw,bohw->io", x, g)
    return dx, dK, dout.sum(axis=(0, 2, 3))


def forward(p, x):
    """Output (B, 64, 64) and the cache for backward."""
    cache = {"x": x}
    h = x
    for i in range(1, 4):
        pre = h @ p[f"W{i}"] + p[f"b{i}"]
        cache[f"pre{i}"] = pre
        h = np.maximum(pre, 0.0)
        cache[f"h{i}"] = h
    d = h.reshape(-1, 16, 8, 8)
    cache["d0"] = d
    for i in range(1, 4):
        pre = deconv(d, p[f"K{i}"], p[f"c{i}"])
        cache[f"dpre{i}"] = pre
        d = np.maximum(pre, 0.0) if i < 3 else pre
        cache[f"d{i}"] = d
    a = cache["h3"] @ p["Wa"] + p["ba"]
    cache["a"] = a
    yb = a @ p["Wb"] + p["bb"]
    return d[:, 0] + yb.reshape(-1, 64, 64), cache


def loss_and_grads(p, x, target):
    """Mean squared error and its gradient with respect to every parameter."""
    y, cache = forward(p, x)
    r = y - target
    loss = float(np.mean(r * r))
    g = {}
    dd = (2.0 * r / r.size)[:, None]
    # basis branch: y = ... + (h3 Wa + ba) Wb + bb
    dy = dd.reshape(x.shape[0], 4096)
    g["Wb"] = cache["a"].T @ dy
    g["bb"] = dy.sum(axis=0)
    da = dy @ p["Wb"].T
    g["Wa"] = cache["h3"].T @ da
    g["ba"] = da.sum(axis=0)
    dh3_basis = da @ p["Wa"].T
    for i in range(3, 0, -1):
        if i < 3:
            dd = dd * (cache[f"dpre{i}"] > 0)
        din, g[f"K{i}"], g[f"c{i}"] = deconv_backward(cache[f"d{i - 1}"], p[f"K{i}"], dd)
        dd = din
    dh = dd.reshape(x.shape[0], -1) + dh3_basis      # h3 feeds both branches
    for i in range(3, 0, -1):
        dh = dh * (cache[f"pre{i}"] > 0)
        hin = cache[f"h{i - 1}"] if i > 1 else cache["x"]
        g[f"W{i}"] = hin.T @ dh
        g[f"b{i}"] = dh.sum(axis=0)
        dh = dh @ p[f"W{i}"].T
    return loss, g


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of every parameter, in place; t counts from 1."""
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
