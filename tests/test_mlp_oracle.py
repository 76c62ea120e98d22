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
