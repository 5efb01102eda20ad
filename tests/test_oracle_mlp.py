"""Pins of the model oracle (oracle/mlp.py) against independent references:
torch's float64 GELU and autograd, torch's bfloat16 conversion, closed forms."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp


def test_gelu_closed_forms():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    x = np.array([-3.0, -1.0, 0.5, 2.0, 8.0])
    ref = torch.nn.functional.gelu(torch.tensor(x, dtype=torch.float64), approximate="none").numpy()
    assert np.allclose(mlp.gelu(x), ref, rtol=0, atol=1e-15)
    assert abs(mlp.gelu(np.array([8.0]))[0] - 8.0) < 1e-12


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=5000), rng.normal(size=100) * 1e-30, [1.00390625, 1.01171875, -0.0, 3e38]])
    x = x.astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def _random_blob(rng):
    b = np.zeros(mlp.BLOB)
    b[:mlp.PARAMS] = rng.normal(size=mlp.PARAMS) * 0.3
    b[mlp.PARAMS:mlp.PARAMS + 8] = rng.normal(size=8)
    b[mlp.PARAMS + 8:mlp.PARAMS + 16] = rng.uniform(0.5, 2.0, size=8)
    b[-1] = 1.0
    return b


def test_forward_matches_torch():
    rng = np.random.default_rng(1)
    blob = _random_blob(rng)
    X = rng.normal(size=(50, 8))
    W1, b1, W2, b2, w3, b3, mu, sd, _ = [torch.tensor(a, dtype=torch.float64) for a in mlp.unpack(blob)[:8]] + [None]
    x = (torch.tensor(X) - mu) / sd
    G = lambda z: torch.nn.functional.gelu(z, approximate="none")
    ref = (G(G(x @ W1 + b1) @ W2 + b2) @ w3 + b3).numpy()
    assert np.allclose(mlp.forward(blob, X), ref, rtol=1e-13, atol=1e-13)


def test_finite_differences_match_autograd():
    rng = np.random.default_rng(2)
    blob = _random_blob(rng)
    X = rng.normal(size=(20, 8))
    Y = rng.normal(size=20)
    g_fd = mlp.grad_fd(blob, X, Y)
    base = torch.tensor(mlp.rounded(blob)[:mlp.PARAMS], dtype=torch.float64, requires_grad=True)
    o = 0
    def take(n):
        nonlocal o
        t = base[o:o + n]
        o += n
        return t
    W1 = take(8 * 64).reshape(8, 64); b1 = take(64); W2 = take(64 * 64).reshape(64, 64); b2 = take(64)
    w3 = take(64); b3 = take(1)
    mu = torch.tensor(blob[mlp.PARAMS:mlp.PARAMS + 8]); sd = torch.tensor(blob[mlp.PARAMS + 8:mlp.PARAMS + 16])
    G = lambda z: torch.nn.functional.gelu(z, approximate="none")
    y = G(G(((torch.tensor(X) - mu) / sd) @ W1 + b1) @ W2 + b2) @ w3 + b3
    L = torch.mean((y - torch.tensor(Y)) ** 2)
    L.backward()
    assert np.allclose(g_fd, base.grad.numpy(), rtol=1e-5, atol=1e-8)


def test_zero_waste_label():
    INF = np.uint64(0xFFFFFFFFFFFFFFFF)
    dist = np.array([5, 7, 9, 2], np.uint64)
    assert mlp.zero_waste_label(np.array([5, 7, 10, 2], np.uint64), [0, 1, 2, 3], dist) == 1.0
    assert mlp.zero_waste_label(np.array([5, 7, 9, 2], np.uint64), [0, 1, 2, 3], dist) == 2.0
    assert mlp.zero_waste_label(np.array([6, 7], np.uint64), [0, 1], dist) == 0.0   # at least 1
    assert mlp.zero_waste_label(np.array([5, 7, 9, INF], np.uint64), [0, 1, 2, 0], dist) == math.log2(3)
