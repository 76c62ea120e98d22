"""Reference of the learned correction's network (numpy).

TEST INFRASTRUCTURE ONLY.  A 64 -> 64 -> 64 -> 1 ReLU network predicting the
log of a host's cardinality from its 64 occupancy features, trained with the
mean squared error on ln n and Adam.  Two forms:

- `forward64` / `backward64`: plain FP64, no rounding (checked by finite
  differences);
- `forward_bf16` / `backward_bf16`: the rounding points of the device
  kernels: features, weights and hidden activations rounded to bfloat16
  (round to nearest even), products accumulated in (at least) FP32, biases
  and the output in FP32.

Parameter vector layout (8385 floats): W1[64x64] (row = output unit), b1[64],
W2[64x64], b2[64], w3[64], b3[1].
"""
from __future__ import annotations

import numpy as np

D = 64
NPARAM = D * D + D + D * D + D + D + 1
OFF_W1, OFF_B1 = 0, D * D
OFF_W2, OFF_B2 = D * D + D, 2 * D * D + D
OFF_W3, OFF_B3 = 2 * D * D + 2 * D, 2 * D * D + 3 * D


def unpack(p: np.ndarray):
    W1 = p[OFF_W1:OFF_B1].reshape(D, D)
    b1 = p[OFF_B1:OFF_W2]
    W2 = p[OFF_W2:OFF_B2].reshape(D, D)
    b2 = p[OFF_B2:OFF_W3]
    w3 = p[OFF_W3:OFF_B3]
    b3 = p[OFF_B3]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, np.atleast_1d(b3)]).astype(np.float64)


def bf16(x) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).reshape(a.shape)


def init_params(seed: int) -> np.ndarray:
    """He-uniform initialisation (float32 values)."""
    rng = np.random.default_rng(seed)
    lim = np.sqrt(6.0 / D)
    W1 = rng.uniform(-lim, lim, (D, D))
    W2 = rng.uniform(-lim, lim, (D, D))
    w3 = rng.uniform(-lim, lim, D) * 0.1
    b1 = np.zeros(D)
    b2 = np.zeros(D)
    b3 = 7.0
    return pack(W1, b1, W2, b2, w3, b3).astype(np.float32).astype(np.float64)


# ------------------------------------------------------------------ FP64

def forward64(p, X):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(p, np.float64))
    X = np.asarray(X, np.float64)
    z1 = X @ W1.T + b1
    h1 = np.maximum(z1, 0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0)
    y = h2 @ w3 + b3
    return y, (X, z1, h1, z2, h2)


def loss64(p, X, t):
    y, _ = forward64(p, X)
    return float(np.mean((y - t) ** 2))


def backward64(p, X, t):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(p, np.float64))
    y, (X, z1, h1, z2, h2) = forward64(p, X)
    B = X.shape[0]
    dy = 2.0 * (y - t) / B
    dh2 = np.outer(dy, w3) * (z2 > 0)
    dh1 = (dh2 @ W2) * (z1 > 0)
    g = pack(dh1.T @ X, dh1.sum(0), dh2.T @ h1, dh2.sum(0), h2.T @ dy, dy.sum())
    return g, float(np.mean((y - t) ** 2))


# ------------------------------------------------------------------ BF16 points

def forward_bf16(p, X):
    W1, b1, W2, b2, w3, b3 = unpack(np.asarray(p, np.float64))
    f32 = np.float32
    Xb = bf16(X).astype(np.float64)
    W1b, W2b, w3b = (bf16(W).astype(np.float64) for W in (W1, W2, w3))
    z1 = (Xb @ W1b.T).astype(f32) + b1.astype(f32)
    h1b = bf16(np.maximum(z1, 0)).astype(np.float64)
    z2 = (h1b @ W2b.T).astype(f32) + b2.astype(f32)
    h2b = bf16(np.maximum(z2, 0)).astype(np.float64)
    y = (h2b @ w3b).astype(f32) + f32(b3)
    return y, (Xb, z1, h1b, z2, h2b, W2b, w3b)


def backward_bf16(p, X, t):
    y, (Xb, z1, h1b, z2, h2b, W2b, w3b) = forward_bf16(p, X)
    f32 = np.float32
    B = Xb.shape[0]
    dy = (f32(2.0 / B) * (y - np.asarray(t, f32))).astype(f32)
    dh2 = (dy[:, None] * w3b[None, :].astype(f32)).astype(f32) * (h2b > 0)
    dh2b = bf16(dh2).astype(np.float64)
    dh1 = (dh2b @ W2b).astype(f32) * (h1b > 0)
    dh1b = bf16(dh1).astype(np.float64)
    g = pack(dh1b.T @ Xb, dh1b.sum(0), dh2b.T @ h1b, dh2b.sum(0), h2b.T @ dy.astype(np.float64),
             dy.astype(np.float64).sum())
    loss = float(np.mean((y.astype(np.float64) - np.asarray(t, np.float64)) ** 2))
    return g.astype(np.float32).astype(np.float64), loss


def adam(p, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in float32 arithmetic, in the device's operation order."""
    f32 = np.float32
    p, m, v, g = (np.asarray(a, f32).copy() for a in (p, m, v, g))
    c1 = f32(1.0 - b1 ** step)
    c2 = f32(1.0 - b2 ** step)
    m = f32(b1) * m + f32(1.0 - b1) * g
    v = f32(b2) * v + f32(1.0 - b2) * (g * g)
    mh = m / c1
    vh = v / c2
    p = p - f32(lr) * (mh / (np.sqrt(vh) + f32(eps)))
    return p, m, v
