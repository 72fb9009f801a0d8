"""Pins of the oracle's learned-seed network (forward, gradient, Adam)."""
import numpy as np
import pytest
import torch

import oracle as O

NP = O.N_PARAMS


def init_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(NP)
    p[0:128] = rng.normal(0, np.sqrt(2 / 2), 128) * scale
    p[128:192] = rng.normal(0, 0.1, 64)
    p[192:4288] = rng.normal(0, np.sqrt(2 / 64), 4096) * scale
    p[4288:4352] = rng.normal(0, 0.1, 64)
    p[4352:4416] = rng.normal(0, np.sqrt(2 / 64), 64)
    p[4416] = 0.05
    return p


def test_parameter_count():
    assert NP == 64 * 2 + 64 + 64 * 64 + 64 + 64 + 1 == 4417


def test_gradient_matches_central_differences():
    """FP64 network (no rounding): analytic gradient = central differences."""
    p = init_params(1)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (64, 2))
    t = rng.uniform(-1, 1, 64)
    loss, g = O.mlp_loss_grad(p, x, t, round_bf16=False)
    idx = np.concatenate([np.arange(0, 128, 7), np.arange(128, 192, 5), np.arange(192, 4288, 97),
                          np.arange(4288, 4352, 5), np.arange(4352, 4416, 5), [4416]])
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (O.mlp_loss_grad(pp, x, t, False)[0] - O.mlp_loss_grad(pm, x, t, False)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_bf16_rounding_points_match_library_bfloat16():
    """A one-path network y = w3 * r(w2 * r(w1 * r(x))) (all other weights 0)
    shows where the oracle rounds; torch's bfloat16 conversion is the reference."""
    def r(v):
        return float(torch.tensor(v, dtype=torch.float32).to(torch.bfloat16).to(torch.float32))
    p = np.zeros(NP)
    w1, w2, w3 = 1.2345678, 0.87654321, 1.1111111
    p[0] = w1              # W1[0][0]
    p[192] = w2            # W2[0][0]
    p[4352] = w3           # W3[0]
    for x0 in (0.3333333, 0.7777777, -0.5, 0.123456789):
        y = O.mlp_forward(p, np.array([[x0, 0.25]]), round_bf16=True)[0]
        h1 = r(max(r(w1) * r(x0), 0.0))
        h2 = r(max(r(w2) * h1, 0.0))
        assert y == pytest.approx(r(w3) * h2, rel=1e-15, abs=0)
    y0 = O.mlp_forward(p, np.array([[0.3333333, 0.25]]), round_bf16=False)[0]
    assert y0 == pytest.approx(w3 * w2 * w1 * 0.3333333, rel=1e-14)


def test_adam_first_step_closed_form():
    """At step 1 the bias-corrected moments are g and g^2: w -= lr g / (|g| + eps)."""
    w = np.array([1.0, -2.0, 0.5])
    m = np.zeros(3)
    v = np.zeros(3)
    g = np.array([0.3, -4.0, 1e-3])
    O.mlp_adam(w, m, v, g, 1, 1e-2)
    expect = np.array([1.0, -2.0, 0.5]) - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.allclose(w, expect, rtol=1e-14, atol=0)


def test_training_reduces_loss():
    rng = np.random.default_rng(3)
    x = rng.uniform(-1, 1, (512, 2))
    t = 0.5 * np.sin(2 * x[:, 0]) + 0.3 * x[:, 1] ** 2 - 0.2
    p = init_params(4)
    m = np.zeros(NP)
    v = np.zeros(NP)
    l0 = O.mlp_loss_grad(p, x, t, True)[0]
    for s in range(1, 201):
        loss, g = O.mlp_loss_grad(p, x, t, True)
        O.mlp_adam(p, m, v, g, s, 3e-3)
    assert O.mlp_loss_grad(p, x, t, True)[0] < 0.1 * l0
