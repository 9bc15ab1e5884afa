"""The benchmark workload at its full size and launch configuration (needs a GPU).

The four-quadrant Riemann problem on 512 x 512 cells with eps_TT dynamic from 1e-8 is the
workload the benchmark times. Its ranks grow from 2 to about 20 within the first twenty steps,
and from a bond rank of about 17 on the cross blocks (512 x 4 (r + 4)) no longer fit one
workgroup's registers, so the later steps run the multi-workgroup pivot search (one persistent
launch per factorisation). The oracle steps the full grid (about 0.1 s per step), so every step
is checked against it from the same densified state with the alphas the step used: the
per-step bound of the parity tests, 10 eps_TT in the relative Frobenius norm.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import EpsTracker, oracle_problem, rel_err

pytestmark = pytest.mark.gpu

STEPS = 24


@pytest.fixture(scope="module")
def W():
    from paper_2405_12301_amd import wenott
    wenott.load()
    oracle.build(force=False)
    return wenott


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_quadrants_512_every_step_vs_oracle(W):
    _say("case: quadrants 512^2, dynamic eps from 1e-8,", STEPS, "steps, each against the oracle")
    f = workloads.config2_quadrants_2d(512, seed=0)
    s = W.Solver(f, W.default_opts(eps_mode=1, eps0=f.eps0))
    P = oracle_problem(f)
    try:
        worst = 0.0
        eps_of = EpsTracker(f, s.dense(), eps0=f.eps0)
        for step in range(STEPS):
            u = s.dense()
            e_step = eps_of(u)
            dt = f.cfl * min(f.h) / s.max_wavespeed()
            s.step(dt)
            info = s.info()
            assert abs(info.eps - e_step) <= 1e-10 * e_step, (step, info.eps, e_step)
            P.ssprk3(u, dt, alphas=[info.alpha[j] for j in range(3)])
            err = rel_err(s.dense(), u)
            worst = max(worst, err / e_step)
            if step % 4 == 3 or step == STEPS - 1:
                _say(f"  step {step} ranks={list(info.ranks)[:3]} eps={e_step:.3e} err={err:.3e}")
            assert err <= 10 * e_step, (step, err, e_step)
        assert max(list(s.info().ranks)[:3]) >= 17  # the later crosses took the multi-workgroup search
        _say(f"  worst err / eps = {worst:.2f}")
    finally:
        s.close()


def test_quadrants_512_batch_matches_single_and_oracle(W):
    _say("case: quadrants 512^2, two states in lock-step against single steps and the oracle")
    flows = [workloads.config2_quadrants_2d(512, seed=sd) for sd in (0, 3)]
    opts = W.default_opts(eps_mode=1, eps0=flows[0].eps0)
    batch = [W.Solver(f, opts) for f in flows]
    single = [W.Solver(f, opts) for f in flows]
    P = oracle_problem(flows[0])
    try:
        eps_of = EpsTracker(flows[0], batch[0].dense(), eps0=flows[0].eps0)
        for step in range(STEPS):
            check = step >= STEPS - 2
            u0 = batch[0].dense() if check else None
            e_step = eps_of(u0) if check else None
            dts = [f.cfl * min(f.h) / s.max_wavespeed() for f, s in zip(flows, batch)]
            W.wenott_batch_rk3_step([s.ctx for s in batch], dts)
            for s1, dt in zip(single, dts):
                s1.step(dt)
            if check:
                info = batch[0].info()
                P.ssprk3(u0, dt=dts[0], alphas=[info.alpha[j] for j in range(3)])
                err = rel_err(batch[0].dense(), u0)
                _say(f"  step {step} ranks={list(info.ranks)[:3]} err vs oracle={err:.3e} eps={e_step:.3e}")
                assert abs(info.eps - e_step) <= 1e-10 * e_step, (step, info.eps, e_step)
                assert err <= 10 * e_step, (step, err)
        for i, (b, s1) in enumerate(zip(batch, single)):
            d = rel_err(b.dense(), s1.dense())
            _say(f"  state {i}: batched vs single after {STEPS} steps {d:.3e}")
            assert d <= 10 * STEPS * flows[i].eps0 * 2, (i, d)
        assert max(list(batch[0].info().ranks)[:3]) >= 17
    finally:
        for s in batch + single:
            s.close()


def test_blast_full_size_single_state_steps_vs_oracle(W):
    """One spherical blast of the batched workload at its full size (256 x 192 x 128, seed 0,
    dynamic eps from 1e-6), stepped on its own: its ranks reach ~120 in the first step, so the
    cross blocks (10^6-10^7 entries) take the multi-workgroup pivot search one launch per step
    and the TSQR of the wide unfoldings; the step against the oracle on the full grid (observed
    2.7 eps; a second step, not run here, gave 7.8 eps)."""
    _say("case: blast 256 x 192 x 128 (seed 0), a single-state step against the oracle")
    f = workloads.config4_blast_3d(seed=0)
    # the stage crosses of this state need joint ranks beyond the cross-rank limit of 128 (the
    # five components stacked on the column side): they stop there with sampled residuals of a few
    # eps after max_sweeps sweeps, which the explicit slack accepts; the step itself is still held
    # to 10 eps against the oracle
    s = W.Solver(f, W.default_opts(eps_mode=1, eps0=f.eps0, conv_slack=100.0))
    P = oracle_problem(f)
    try:
        u = s.dense()
        e_step = EpsTracker(f, u, eps0=f.eps0)(u)
        dt = f.cfl * min(f.h) / s.max_wavespeed()
        s.step(dt)
        info = s.info()
        assert abs(info.eps - e_step) <= 1e-10 * e_step, (info.eps, e_step)
        P.ssprk3(u, dt, alphas=[info.alpha[j] for j in range(3)])
        err = rel_err(s.dense(), u)
        _say(f"  ranks={list(info.ranks)[:4]} eps={e_step:.2e} err={err:.3e}")
        assert err <= 10 * e_step, (err, e_step)
    finally:
        s.close()
