"""Training of the learned cross proposal on the library's own pivot logs.

Logs come from plain WENO-TT runs (wenott_set_cross_logging): one sample per TT bond of every
stage cross, features of the previous cross and targets of the current one (rank change class,
histogram of the right indices its pivots used). Training runs on the GPU with the library's
FP32 forward/backward/Adam kernels; torch only provides the device buffers.
"""
from __future__ import annotations

import numpy as np

from . import wenott as W


def collect_logs(flows, steps: int, opts=None):
    """Run each flow for `steps` SSP-RK3 steps with logging on; return (x, cls, hist) arrays."""
    xs, cs, hs = [], [], []
    for f in flows:
        s = W.Solver(f, opts if opts is not None else W.default_opts(eps_mode=1, eps0=f.eps0))
        try:
            W.wenott_set_cross_logging(s.ctx, True)
            h = min(f.h)
            for _ in range(steps):
                s.step(f.cfl * h / s.max_wavespeed())
            x, c, hh = W.wenott_get_cross_log(s.ctx)
            xs.append(x), cs.append(c), hs.append(hh)
        finally:
            s.close()
    return np.concatenate(xs), np.concatenate(cs), np.concatenate(hs)


def train(x, cls, hist, iters: int = 400, batch: int = 256, lr: float = 2e-3, seed: int = 1):
    """Adam on the GPU; returns (device params tensor, per-iteration losses)."""
    import torch
    dev = torch.device("cuda")
    n = x.shape[0]
    P = torch.empty(W.wenott_mlp_nparams(), dtype=torch.float32, device=dev)
    W.wenott_mlp_init_params(P, seed)
    g = torch.zeros_like(P)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    X = torch.from_numpy(x.astype(np.float32)).to(dev)
    C = torch.from_numpy(cls.astype(np.int32)).to(dev)
    H = torch.from_numpy(hist.astype(np.float32)).to(dev)
    b = min(batch, n)
    work = torch.empty(W.wenott_mlp_workspace(b), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(seed)
    losses = []
    for t in range(1, iters + 1):
        idx = torch.from_numpy(rng.choice(n, size=b, replace=False)).to(dev)
        xb, cb, hb = X[idx].contiguous(), C[idx].contiguous(), H[idx].contiguous()
        W.wenott_mlp_loss_grad(P, xb, cb, hb, g, loss, work)
        W.wenott_mlp_adam_step(P, g, m, v, t, lr)
        if t % 20 == 0 or t == 1:
            losses.append(float(loss.item()))
    return P, losses
