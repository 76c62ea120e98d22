"""Pins of the learned correction's reference network (CPU)."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 20000),
                        np.array([1.0, 1 + 2**-8, 1 + 3 * 2**-8, 1 + 2**-9, -1 - 2**-8, 0.0, 65504.0], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(np.float32(1 + 2**-8)) == 1.0          # tie -> even
    assert mlp.bf16(np.float32(1 + 3 * 2**-8)) == np.float32(1 + 2**-6)


def test_backward64_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3) + rng.normal(0, 0.05, mlp.NPARAM)
    X = rng.random((40, 64))
    t = rng.uniform(3, 12, 40)
    g, _ = mlp.backward64(p, X, t)
    idx = np.concatenate([rng.integers(0, mlp.NPARAM, 200), [mlp.OFF_B3, mlp.OFF_W3, mlp.OFF_B1, mlp.OFF_B2]])
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd = (mlp.loss64(p + e, X, t) - mlp.loss64(p - e, X, t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_bf16_form_tracks_fp64():
    rng = np.random.default_rng(2)
    p = mlp.init_params(4)
    X = rng.random((256, 64))
    t = rng.uniform(3, 12, 256)
    y64, _ = mlp.forward64(p, X)
    yb, _ = mlp.forward_bf16(p, X)
    assert np.max(np.abs(yb - y64)) < 0.05 * (1 + np.max(np.abs(y64)))
    g64, _ = mlp.backward64(p, X, t)
    gb, _ = mlp.backward_bf16(p, X, t)
    assert np.linalg.norm(gb - g64) < 0.05 * np.linalg.norm(g64)


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2, so each weight moves
    by lr * g / (|g| + eps), i.e. lr * sign(g) for |g| >> eps."""
    rng = np.random.default_rng(3)
    p = rng.standard_normal(mlp.NPARAM).astype(np.float32)
    g = rng.standard_normal(mlp.NPARAM).astype(np.float32)
    z = np.zeros(mlp.NPARAM, np.float32)
    p1, m1, v1 = mlp.adam(p, z, z, g, 1, 1e-3)
    assert np.allclose(p - p1, 1e-3 * np.sign(g), rtol=1e-4, atol=1e-9)
    assert np.allclose(m1, 0.1 * g, rtol=1e-6) and np.allclose(v1, 0.001 * g * g, rtol=1e-5)


def _fp32_shuffled_forward(p, X, seed):
    """The bf16 rounding points of the device with FP32 sums taken in a
    shuffled order (one product at a time), as another accumulation order."""
    W1, b1, W2, b2, w3, b3 = mlp.unpack(np.asarray(p, np.float64))
    f32 = np.float32
    rng = np.random.default_rng(seed)
    Xb, W1b, W2b, w3b = mlp.bf16(X), mlp.bf16(W1), mlp.bf16(W2), mlp.bf16(w3)

    def dot(A, B):  # A[n,64] @ B[64,m] in float32, shuffled order
        z = np.zeros((A.shape[0], B.shape[1]), f32)
        for k in rng.permutation(A.shape[1]):
            z = (z + A[:, k:k + 1] * B[k:k + 1, :]).astype(f32)
        return z

    h1 = mlp.bf16(np.maximum(dot(Xb, W1b.T) + b1.astype(f32), 0))
    h2 = mlp.bf16(np.maximum(dot(h1, W2b.T) + b2.astype(f32), 0))
    return dot(h2, w3b[:, None])[:, 0] + f32(b3)


def test_forward_bound_covers_another_summation_order():
    """The per-row bound the GPU forward test uses holds for FP32 sums in
    other orders, and is far below the output scale."""
    from .test_gpu_mlp import _forward_bound, _rand_problem
    for seed in range(3):
        p, X, _ = _rand_problem(seed, 1500)
        y_r, _ = mlp.forward_bf16(p, X)
        y_s = _fp32_shuffled_forward(p, X, seed)
        d = np.abs(y_s.astype(np.float64) - y_r)
        b = _forward_bound(p, X)
        assert (d <= b).all()
        assert np.median(b) < 1e-2 and b.max() < 0.1
