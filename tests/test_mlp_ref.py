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
