"""Pins of the FP64 loss-predictor reference (oracle/mlp.py): BF16 rounding
against the bit-level definition of round-to-nearest-even, gradients against
central finite differences, the loss and its gradient at known points, and
the first Adam step against its closed form."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_bf16_round_to_nearest_even():
    f32 = lambda bits: np.array([bits], dtype=np.uint32).view(np.float32)[0]
    one = 1.0
    assert mlp.bf16(one)[()] == 1.0
    # halfway between 1 and 1 + 2^-7 -> even (1); halfway above an odd value -> up
    assert mlp.bf16(1 + 2.0 ** -8)[()] == 1.0
    assert mlp.bf16(1 + 3 * 2.0 ** -8)[()] == 1 + 2.0 ** -6
    assert mlp.bf16(1 + 2.0 ** -8 + 2.0 ** -20)[()] == 1 + 2.0 ** -7
    assert mlp.bf16(-(1 + 3 * 2.0 ** -8))[()] == -(1 + 2.0 ** -6)
    # exactly representable values are unchanged; bf16 keeps the FP32 exponent range
    for v in (0.0, -0.0, 2.0 ** -126, 3.0 * 2.0 ** 100, float("inf")):
        assert mlp.bf16(v)[()] == v
    assert np.isnan(mlp.bf16(float("nan"))[()])
    # largest finite FP32 rounds up to infinity (past the largest bf16)
    assert mlp.bf16(f32(0x7F7FFFFF))[()] == float("inf")
    # relative rounding error is at most 2^-8
    x = np.random.default_rng(1).normal(size=10000) * 10.0 ** np.random.default_rng(2).integers(-5, 5, 10000)
    assert np.max(np.abs(mlp.bf16(x) / x.astype(np.float32) - 1)) <= 2.0 ** -8


def _net(seed=3):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.2, mlp.N_PARAMS)
    x = rng.normal(0, 1, (64, 16))
    y = (rng.random(64) < 0.3).astype(float)
    return theta, x, y


def test_backward_matches_finite_differences_unrounded():
    theta, x, y = _net()
    w = 2.5
    L, g = mlp.backward(theta, x, y, w, rounding=False)
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(mlp.N_PARAMS, 60, replace=False), [mlp.N_PARAMS - 1]])
    h = 1e-6
    for j in idx:
        tp = theta.copy(); tp[j] += h
        tm = theta.copy(); tm[j] -= h
        fd = (mlp.loss(mlp.forward(tp, x, False)["z3"], y, w) -
              mlp.loss(mlp.forward(tm, x, False)["z3"], y, w)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-7 * max(1.0, abs(g[j])), j
    assert abs(L - mlp.loss(mlp.forward(theta, x, False)["z3"], y, w)) < 1e-15


def test_rounded_backward_close_to_unrounded():
    theta, x, y = _net(5)
    _, g0 = mlp.backward(theta, x, y, 2.0, rounding=False)
    _, g1 = mlp.backward(theta, x, y, 2.0, rounding=True)
    cos = g0 @ g1 / np.linalg.norm(g0) / np.linalg.norm(g1)
    assert cos > 0.999
    assert np.linalg.norm(g1 - g0) / np.linalg.norm(g0) < 2e-2


def test_loss_and_gradient_at_zero_logit():
    w = 3.0
    y = np.array([1.0, 0.0, 1.0, 0.0])
    z = np.zeros(4)
    assert math.isclose(mlp.loss(z, y, w), (2 * w + 2) * math.log(2) / 4, rel_tol=1e-15)
    theta = np.zeros(mlp.N_PARAMS)          # all-zero net: logit 0 for any input
    _, g = mlp.backward(theta, np.ones((4, 16)), y, w)
    # dL/db3 = mean(s(0)(w y + 1 - y) - w y) = mean(0.5 (w+1 - ... ))
    expect = np.mean(0.5 * (w * y + 1 - y) - w * y)
    assert math.isclose(g[-1], expect, rel_tol=1e-15)
    # very confident logits stay finite
    assert np.isfinite(mlp.loss(np.array([800.0, -800.0]), np.array([0.0, 1.0]), 1.0))


def test_first_adam_step_closed_form():
    rng = np.random.default_rng(0)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, lr=1e-3)
    # bias-corrected m/sqrt(v) = g/|g| on the first step
    assert np.allclose(new - theta, -1e-3 * np.sign(g) * (np.abs(g) / (np.abs(g) + 1e-8)),
                       rtol=1e-12, atol=1e-18)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_forward_shapes_and_relu():
    theta, x, _ = _net(9)
    f = mlp.forward(theta, x)
    assert f["z3"].shape == (64,)
    assert np.all(f["H1"] >= 0) and np.all(f["H2"] >= 0)
    assert np.array_equal(f["H1"], mlp.bf16(np.maximum(f["z1"], 0.0)))
    assert np.array_equal(f["H2"], mlp.bf16(np.maximum(f["z2"], 0.0)))
