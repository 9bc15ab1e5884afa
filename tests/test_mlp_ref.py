"""Pins of the FP64 reference MLP of the learned proposal (CPU)."""
import math

import numpy as np

from oracle import mlp_ref as M


def _params(rng, scale=0.1):
    n = M.IN * M.HID + M.HID + M.HID * M.HID + M.HID + M.HID * M.OUT + M.OUT
    return rng.normal(size=n) * scale


def test_zero_parameters_give_uniform_softmax_loss():
    rng = np.random.default_rng(0)
    p = np.zeros(M.IN * M.HID + M.HID + M.HID * M.HID + M.HID + M.HID * M.OUT + M.OUT)
    x = rng.normal(size=(5, M.IN))
    cls = rng.integers(0, M.NR, size=5)
    hist = rng.random(size=(5, M.NB))
    hist /= hist.sum(axis=1, keepdims=True)
    loss, _ = M.loss_and_grad(p, x, cls, hist)
    assert abs(loss - (math.log(M.NR) + math.log(M.NB))) < 1e-12


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params(rng)
    x = rng.normal(size=(4, M.IN))
    cls = rng.integers(0, M.NR, size=4)
    hist = rng.random(size=(4, M.NB))
    hist /= hist.sum(axis=1, keepdims=True)
    _, g = M.loss_and_grad(p, x, cls, hist)
    idx = rng.choice(p.size, size=60, replace=False)
    h = 1e-6
    num = []
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        num.append((M.loss_and_grad(p + e, x, cls, hist)[0] - M.loss_and_grad(p - e, x, cls, hist)[0]) / (2 * h))
    num = np.array(num)
    assert np.linalg.norm(num - g[idx]) <= 1e-6 * max(np.linalg.norm(g[idx]), 1e-12) + 1e-9


def test_bf16_rounding_and_inference():
    """BF16 rounding keeps 8 significant bits with ties to even (hand values), and BF16
    inference equals the FP64 forward when every operand is a BF16 value already."""
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -7 + 2.0 ** -9, -3.5, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2.0 ** -6, 1.0 + 2.0 ** -7, -3.5, 0.0])
    assert np.array_equal(M.bf16(vals), want)
    rng = np.random.default_rng(3)
    n = M.IN * M.HID + M.HID + M.HID * M.HID + M.HID + M.HID * M.OUT + M.OUT
    # sparse weights of few bits: every operand and every activation is a BF16 value
    p = rng.integers(-1, 2, size=n) * (rng.random(n) < 0.03) / 4.0
    x = rng.integers(-1, 2, size=(5, M.IN)).astype(np.float64)
    h1, h2, y = M.forward(p, x)
    assert np.all(np.abs(h1 - M.bf16(h1)) == 0) and np.all(np.abs(h2 - M.bf16(h2)) == 0)
    assert np.array_equal(M.forward_bf16(p, x)[2], y)
