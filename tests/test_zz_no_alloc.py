"""wenott_max_wavespeed_noalloc: the entry point that allocates nothing (needs a GPU; collected
last, after every other test has run in the same process).

Its result is compared with wenott_max_wavespeed's on twin contexts (same state, same options,
so the same seeded search): equal bit for bit, on two calls in a row (the second on a smaller
state, in the same static workspace), for the line search (3D and 2D) and the exact 2D maximum,
which is also checked against the oracle's maximum over every cell. A request beyond the static
workspace is rejected with EINVAL.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import dense_of_cores, oracle_problem

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


def _pair(W, flows, alpha_mode):
    """alpha of each flow from the allocating entry point and from the no-alloc one, called on
    twin contexts one after the other (each list in call order). The steps after the calls are
    compared bit for bit, so both take the same contraction tiles: the tile table is fixed
    while they run (a bucket still being tuned gives successive calls different candidate
    shapes, which agree only to rounding)."""
    ref, got = [], []
    W.wenott_gemm_autotune(0)
    try:
        _pair_steps(W, flows, alpha_mode, ref, got)
    finally:
        W.wenott_gemm_autotune(1)
    return ref, got


def _pair_steps(W, flows, alpha_mode, ref, got):
    for f in flows:
        a = W.Solver(f, W.default_opts(alpha_mode=alpha_mode))
        b = W.Solver(f, W.default_opts(alpha_mode=alpha_mode))
        try:
            ref.append(a.max_wavespeed())
            got.append(W.wenott_max_wavespeed_noalloc(b.ctx))
            # the value is cached for the next step exactly like the allocating call's
            dt = 0.4 * min(f.h) / got[-1]
            a.step(dt)
            b.step(dt)
            assert np.array_equal(a.dense(), b.dense())
        finally:
            a.close()
            b.close()


@pytest.mark.parametrize("case", ["search3d", "search2d", "exact2d"])
def test_noalloc_matches_allocating_entry_point(W, case):
    if case == "search3d":
        flows = [workloads.config5_tilted_sod_3d(96, seed=0), workloads.config5_tilted_sod_3d(48, seed=4)]
        mode = 1
    elif case == "search2d":
        flows = [workloads.config2_quadrants_2d(256, seed=0), workloads.config2_quadrants_2d(64, seed=3)]
        mode = 1
    else:
        flows = [workloads.config2_quadrants_2d(512, seed=0), workloads.config1_smooth_wave_2d(40)]
        mode = 0
    _say("case: no-alloc alpha,", case, [f.n for f in flows])
    ref, got = _pair(W, flows, mode)
    _say("  allocating", ref, "no-alloc", got)
    assert got == ref  # bit for bit, both calls
    if mode == 0:
        for f, g in zip(flows, got):
            want = oracle_problem(f).alpha(dense_of_cores(f.cores))
            assert abs(g - want) <= 1e-12 * want


def test_noalloc_rejects_what_does_not_fit(W):
    f = workloads.config3_wave_3d(24, seed=0, modes=2)
    s = W.Solver(f, W.default_opts(alpha_mode=0))
    try:
        with pytest.raises(W.WenottError) as ei:
            W.wenott_max_wavespeed_noalloc(s.ctx)
        assert ei.value.status == W.EINVAL
        assert s.max_wavespeed() > 0  # the allocating entry point still serves it
    finally:
        s.close()
