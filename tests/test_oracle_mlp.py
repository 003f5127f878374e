"""Pins for the network oracle: gradients against central finite differences,
GELU against its erf definition, Adam against its constant-gradient closed
form, and the bfloat16 rounding against the format's definition."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_matches_erf_definition_and_derivative():
    for z in (-3.0, -0.5, 0.0, 0.7, 2.5):
        assert mlp.gelu(np.array(z)) == pytest.approx(0.5 * z * (1 + math.erf(z / math.sqrt(2))), abs=1e-15)
        h = 1e-6
        fd = (mlp.gelu(np.array(z + h)) - mlp.gelu(np.array(z - h))) / (2 * h)
        assert mlp.gelu_prime(np.array(z)) == pytest.approx(fd, abs=1e-8)


def test_gradients_match_central_finite_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(64, 32, 64, seed=1)
    X = rng.standard_normal((8, 64))
    T = rng.standard_normal((8, 64))
    _, g, _ = mlp.loss_and_grads(p, X, T)
    h = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            q = {kk: vv.copy() for kk, vv in p.items()}
            q[k].reshape(-1)[idx] += h
            lp, _, _ = mlp.loss_and_grads(q, X, T)
            q[k].reshape(-1)[idx] -= 2 * h
            lm, _, _ = mlp.loss_and_grads(q, X, T)
            fd = (lp - lm) / (2 * h)
            assert g[k].reshape(-1)[idx] == pytest.approx(fd, rel=1e-5, abs=1e-10), (k, idx)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are g and g^2, so each
    step moves a weight by lr * g / (|g| + eps)."""
    p = {"w": np.array([1.0, -2.0, 0.5])}
    g = {"w": np.array([0.3, -1e-3, 4.0])}
    st = {}
    q = p
    for t in range(1, 6):
        q = mlp.adam_update(q, g, st, t, lr=1e-2)
    expect = p["w"] - 5 * 1e-2 * g["w"] / (np.abs(g["w"]) + 1e-8)
    assert np.allclose(q["w"], expect, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_definition():
    # exactly representable values are unchanged; halfway cases round to even
    vals = np.array([1.0, -2.5, 3.140625, 0.0], dtype=np.float32)
    assert np.array_equal(mlp.bf16_round(vals), vals.astype(np.float64))
    one = np.float32(1.0).view(np.uint32)
    up_half = np.array([one + 0x8000], dtype=np.uint32).view(np.float32)      # 1 + 2^-8: tie -> even (1.0)
    above = np.array([one + 0x8001], dtype=np.uint32).view(np.float32)        # just above the tie -> up
    odd_half = np.array([one + 0x18000], dtype=np.uint32).view(np.float32)    # tie with odd lsb -> up
    assert mlp.bf16_round(up_half)[0] == 1.0
    assert mlp.bf16_round(above)[0] == 1.0 + 2 ** -7
    assert mlp.bf16_round(odd_half)[0] == 1.0 + 2 * 2 ** -7
    x = np.random.default_rng(2).standard_normal(1000)
    assert np.max(np.abs(mlp.bf16_round(x) - x) / np.abs(x)) <= 2 ** -8
