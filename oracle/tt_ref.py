"""Tensor-train reference definitions in NumPy FP64.

TEST INFRASTRUCTURE ONLY (part of the oracle).

* ``tt_full``: the TT value X(i1..id) = G1(i1) G2(i2) ... Gd(id) written out as a chain
  of contractions (Sec. 3.1, eqs. TT_def and TT_def_2). Cores are (R_{k-1}, N_k, R_k).
* ``tt_svd``: TT-SVD, the sequence of truncated SVDs of the unfoldings of a full tensor
  (Sec. 3.3 first paragraph), each truncated to the smallest rank whose discarded tail is
  at most delta = eps ||X||_F / sqrt(d-1), so that ||X - X_TT||_F <= eps ||X||_F.
  Its ranks are the reference for what a rounding to the same tolerance may keep.
* ``maxvol_dominant``: the maximum-volume condition (Sec. 3.3) checked by brute force.
"""
from __future__ import annotations

import itertools

import numpy as np


def tt_full(cores) -> np.ndarray:
    """Dense tensor of a TT given as a list of (R_{k-1}, N_k, R_k) cores."""
    out = np.asarray(cores[0], dtype=np.float64)
    if out.shape[0] != 1:
        raise ValueError("first rank must be 1")
    res = out.reshape(out.shape[1], out.shape[2])
    shape = [out.shape[1]]
    for g in cores[1:]:
        g = np.asarray(g, dtype=np.float64)
        if g.shape[0] != res.shape[1]:
            raise ValueError("rank mismatch")
        res = res @ g.reshape(g.shape[0], -1)
        shape.append(g.shape[1])
        res = res.reshape(-1, g.shape[2])
    if res.shape[1] != 1:
        raise ValueError("last rank must be 1")
    return res.reshape(shape)


def tt_svd(x: np.ndarray, eps: float, rank_cap: int | None = None):
    """TT-SVD of a full tensor with relative Frobenius accuracy eps (and an optional cap)."""
    x = np.asarray(x, dtype=np.float64)
    d = x.ndim
    nrm = np.linalg.norm(x)
    delta = eps * nrm / np.sqrt(max(d - 1, 1))
    cores = []
    r = 1
    c = x.reshape(1, -1)
    for k in range(d - 1):
        c = c.reshape(r * x.shape[k], -1)
        u, s, vt = np.linalg.svd(c, full_matrices=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]  # tail[j] = ||s[j:]||
        rk = int(np.sum(tail > delta)) if s.size else 0
        rk = max(rk, 1)
        if rank_cap is not None:
            rk = min(rk, rank_cap)
        cores.append(u[:, :rk].reshape(r, x.shape[k], rk))
        c = s[:rk, None] * vt[:rk]
        r = rk
    cores.append(c.reshape(r, x.shape[-1], 1))
    return cores


def tt_ranks(cores):
    return [1] + [int(g.shape[2]) for g in cores[:-1]] + [1]


def maxvol_dominant(a: np.ndarray, rows, tol: float = 1e-12) -> bool:
    """True iff the r rows `rows` of the n x r matrix a form a dominant submatrix:
    every entry of B = a a[rows]^{-1} is at most 1 in modulus (up to tol)."""
    sub = a[list(rows)]
    b = np.linalg.solve(sub.T, a.T).T
    return bool(np.max(np.abs(b)) <= 1.0 + tol)


def max_volume_rows(a: np.ndarray):
    """Brute force: the r-row subset of an n x r matrix with the largest |det|."""
    n, r = a.shape
    best, arg = -1.0, None
    for rows in itertools.combinations(range(n), r):
        v = abs(np.linalg.det(a[list(rows)]))
        if v > best:
            best, arg = v, rows
    return arg, best


def full_pivot_lu(a: np.ndarray, rel_tol2: float, rmax: int):
    """Greedy maximum-volume pivots by complete pivoting (the cross's pivot rule, Sec. 3.3):
    at each step the residual entry of largest magnitude (the first in row-major order among
    equals) is the pivot; its row and column are recorded, L's column is the residual column
    divided by the pivot (1 at the pivot row) and the rank-one term is subtracted. The search
    stops when the residual's squared Frobenius norm is <= rel_tol2 times the block's, after rmax
    pivots, or at a zero residual; a nonzero block always gives at least one pivot, an all-zero
    block gives rank 1 with pivot (0, 0). Returns (rank, rows, cols, L (m x rank), residual^2)."""
    r = np.array(a, dtype=np.float64, copy=True)
    m, n = r.shape
    tol2 = rel_tol2 * float(np.sum(r * r))
    rows, cols, lcols = [], [], []
    for t in range(rmax + 1):
        s2 = float(np.sum(r * r))
        e = int(np.argmax(np.abs(r)))
        pmax = abs(r.flat[e])
        if t == 0 and pmax <= 0.0:
            l0 = np.zeros(m)
            l0[0] = 1.0
            return 1, [0], [0], l0[:, None], 0.0
        if t > 0 and (t >= rmax or pmax <= 0.0 or s2 <= tol2):
            return t, rows, cols, np.stack(lcols, axis=1), s2
        i, j = divmod(e, n)
        lcol = r[:, j] / r[i, j]
        lcol[i] = 1.0
        urow = r[i, :].copy()
        r -= np.outer(lcol, urow)
        r[i, :] = 0.0
        r[:, j] = 0.0
        rows.append(i)
        cols.append(j)
        lcols.append(lcol)
    raise AssertionError("unreachable")
