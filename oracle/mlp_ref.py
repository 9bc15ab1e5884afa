"""FP64 reference of the learned-proposal MLP (test infrastructure only).

Same parameter layout and loss as the HIP kernels: W1[IN][HID], b1, W2[HID][HID], b2,
W3[HID][OUT], b3; ReLU; loss = CE(rank logits, class) + CE(bin logits, target histogram),
mean over the batch. Gradients by hand-derived backpropagation.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT, NR, NB = 96, 128, 81, 17, 64


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    shapes = [(IN, HID), (HID,), (HID, HID), (HID,), (HID, OUT), (OUT,)]
    out = []
    for s in shapes:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    assert o == p.size
    return out


def forward(p, x):
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = np.maximum(x @ W1 + b1, 0.0)
    h2 = np.maximum(h1 @ W2 + b2, 0.0)
    return h1, h2, h2 @ W3 + b3


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64: the upper 16 bits of
    the FP32 encoding after adding half an ulp of the bits dropped."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def forward_bf16(p, x):
    """BF16 inference: every layer's operands (input or previous activation as FP32, weights,
    biases) rounded to BF16, products and sums exact (FP64)."""
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1 = np.maximum(bf16(x) @ bf16(W1) + bf16(b1), 0.0).astype(np.float32)
    h2 = np.maximum(bf16(h1) @ bf16(W2) + bf16(b2), 0.0).astype(np.float32)
    return h1, h2, bf16(h2) @ bf16(W3) + bf16(b3)


def _logsumexp(z):
    m = z.max(axis=1, keepdims=True)
    return m[:, 0] + np.log(np.exp(z - m).sum(axis=1))


def loss_and_grad(p, x, cls, hist):
    x = np.asarray(x, dtype=np.float64)
    hist = np.asarray(hist, dtype=np.float64)
    B = x.shape[0]
    W1, b1, W2, b2, W3, b3 = unpack(p)
    h1, h2, y = forward(p, x)
    yr, yh = y[:, :NR], y[:, NR:]
    lr, lh = _logsumexp(yr), _logsumexp(yh)
    loss = (lr - yr[np.arange(B), cls]).sum() + (hist * (lh[:, None] - yh)).sum()
    loss /= B
    dy = np.zeros_like(y)
    dy[:, :NR] = np.exp(yr - lr[:, None])
    dy[np.arange(B), cls] -= 1.0
    dy[:, NR:] = hist.sum(axis=1, keepdims=True) * np.exp(yh - lh[:, None]) - hist
    dy /= B
    gW3, gb3 = h2.T @ dy, dy.sum(axis=0)
    dh2 = (dy @ W3.T) * (h2 > 0)
    gW2, gb2 = h1.T @ dh2, dh2.sum(axis=0)
    dh1 = (dh2 @ W2.T) * (h1 > 0)
    gW1, gb1 = x.T @ dh1, dh1.sum(axis=0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g
