"""The pivot selection of the cross (complete pivoting: the greedy maximum-volume rule of
Sec. 3.3) on its own, against the oracle's step-by-step definition, in every layout the library
uses (one workgroup in registers; stripes over many workgroups stepped one launch per pivot, or
in one persistent launch with the stripes in registers, in registers and LDS, or streamed), on
blocks shaped like the cross blocks of the 512^3 workload (needs a GPU)."""
import sys

import numpy as np
import pytest

import oracle
from oracle import tt_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    from paper_2405_12301_amd import wenott
    wenott.load()
    oracle.build(force=False)
    return wenott


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _block(m, n, rank, seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(m, rank)) @ rng.normal(size=(rank, n))
    A *= np.exp(rng.normal(size=(1, n)))  # columns of unequal scale
    return A + 1e-7 * rng.normal(size=(m, n))


@pytest.mark.parametrize("m,n,rank,persistent", [
    (60, 40, 12, True),          # one workgroup, register tiles
    (900, 120, 20, True),        # stripes, small persistent launch
    (900, 120, 20, False),       # the same stepped
    (6000, 200, 30, True),       # long stripes in registers
    (22528, 240, 44, True),      # 16 rows per thread
    (30208, 315, 48, True),      # 20 rows per thread (4 in LDS)
    (30208, 315, 48, False),     # stepped, long stripes
    (61440, 300, 40, True),      # rows streamed through the block
    (22528, 660, 100, True),     # the widest cross blocks of the 512^3 workload
    (40000, 9, 5, True),         # narrow: two threads per row
    (38000, 255, 60, True),      # 16 rows per thread in registers, 3 in LDS
    (90000, 200, 20, True),      # 16 in registers, 10 in LDS, 10 streamed
    (5000, 2048, 30, True),      # the widest block the layout takes: one row per 256 threads
])
def test_pivot_search_matches_the_definition(W, m, n, rank, persistent):
    import torch
    layout = W.wenott_pivot_layout(m, n)
    _say(f"case: pivots {m} x {n}, rank {rank}, persistent allowed {persistent}, layout {layout}")
    A = _block(m, n, rank, seed=m + n)
    rmax = min(m, n, 128)
    rel_tol2 = 1e-12
    r_o, rows_o, cols_o, L_o, s2_o = tt_ref.full_pivot_lu(A, rel_tol2, rmax)
    r, rows, cols, L, s2, tol2 = W.wenott_pivot_search(torch.from_numpy(A).cuda(), rmax, rel_tol2, persistent)
    _say(f"  rank {r} (oracle {r_o}), residual^2 {s2:.3e} (oracle {s2_o:.3e}, threshold {tol2:.3e})")
    assert r == r_o
    assert list(rows) == list(rows_o) and list(cols) == list(cols_o)
    Lg = L[:, :r].cpu().numpy()
    assert np.max(np.abs(Lg - L_o)) <= 1e-9
    assert abs(s2 - s2_o) <= 1e-6 * max(s2_o, 1e-300) + 1e-20 * float(np.sum(A * A))
