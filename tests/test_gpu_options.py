"""Options of the boundary and their failure outcomes, through the C ABI (needs a GPU).

* rounds_per_stage = 2: eq. tt-ssprk3 literally (the forward Euler value X + dt L(X) rounded,
  then the combination with U^n rounded again in stages 2 and 3), step parity with the oracle.
* A cross that cannot reach its tolerance within max_sweeps fails the step with ENOCONV and
  leaves the state as it was.
* The single-launch pivot search whose waits for the other workgroups give up (forced from the
  host by a zero poll bound, so every kernel still ends) falls back to one launch per pivot step
  from a freshly evaluated block; the step still matches the oracle.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import EpsTracker, oracle_problem, rel_err

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


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("case", ["quadrants2d", "wave3d"])
def test_two_roundings_per_stage(W, case, scheme):
    f = workloads.config2_quadrants_2d(64, seed=2) if case == "quadrants2d" else \
        workloads.config3_wave_3d(24, seed=0, modes=2)
    eps = 1e-8
    _say("case: rounds_per_stage = 2,", case, "scheme", scheme)
    s = W.Solver(f, W.default_opts(eps_mode=0, eps0=eps, scheme=scheme, rounds_per_stage=2))
    P = oracle_problem(f)
    try:
        for step in range(2):
            u = s.dense()
            dt = 0.5 * min(P.h) / P.alpha(u)
            s.step(dt)
            info = s.info()
            P.ssprk3(u, dt, alphas=[info.alpha[i] for i in range(3)])
            err = rel_err(s.dense(), u)
            _say(f"  step {step} err {err:.3e} ranks {list(info.ranks)[:f.ndim + 1]}")
            # one more rounding per stage than the default: the per-step budget of 10 eps holds
            assert err <= 10 * eps
    finally:
        s.close()


def test_nonconvergence_raises_and_keeps_state(W):
    f = workloads.config2_quadrants_2d(48, seed=1)
    _say("case: forced non-convergence (one sweep, no enrichment, eps 1e-13)")
    s = W.Solver(f, W.default_opts(eps_mode=0, eps0=1e-13, max_sweeps=1, kick_rank=0))
    try:
        before = s.dense()
        P = oracle_problem(f)
        dt = 0.5 * min(P.h) / P.alpha(before)
        with pytest.raises(W.WenottError) as ei:
            s.step(dt)
        _say("  raised:", ei.value)
        assert ei.value.status == W.ENOCONV
        after = s.dense()
        assert np.array_equal(before, after)
    finally:
        s.close()


def test_conv_slack_accepts_what_strict_rejects(W):
    """The same forced case with a huge slack is accepted (the slack is an explicit option); the
    default slack (1) rejects it."""
    f = workloads.config2_quadrants_2d(48, seed=1)
    s = W.Solver(f, W.default_opts(eps_mode=0, eps0=1e-13, max_sweeps=1, kick_rank=0, conv_slack=1e30))
    try:
        u = s.dense()
        dt = 0.5 * min(oracle_problem(f).h) / oracle_problem(f).alpha(u)
        s.step(dt)
        info = s.info()
        _say("  accepted with residuals", [info.residual[i][0] for i in range(3)])
        assert max(info.residual[i][0] for i in range(3)) > 1e-13
    finally:
        s.close()


def test_persistent_pivot_fallback(W):
    """Tilted Sod 128^3: the cross blocks are stripes for the single-launch pivot search. With the
    poll bound set to zero every such launch gives up at its first wait; the driver evaluates the
    block again and runs the one-launch-per-step form. Two steps against the oracle, then the
    default bound is restored."""
    f = workloads.config5_tilted_sod_3d(128, seed=0)
    _say("case: pivot fallback, tilted Sod 128^3")
    s = W.Solver(f, W.default_opts(eps_mode=1, eps0=f.eps0))
    P = oracle_problem(f)
    W.wenott_set_pivot_wait_limit(0)
    try:
        u = s.dense()
        eps_of = EpsTracker(f, u, eps0=f.eps0)
        falls = 0
        for step in range(2):
            u = s.dense()
            e_step = eps_of(u)
            dt = f.cfl * min(f.h) / s.max_wavespeed()
            s.step(dt)
            info = s.info()
            falls += info.pivot_fallbacks
            P.ssprk3(u, dt, alphas=[info.alpha[i] for i in range(3)])
            err = rel_err(s.dense(), u)
            _say(f"  step {step} err {err:.3e} eps {e_step:.3e} fallbacks {info.pivot_fallbacks} "
                 f"ranks {list(info.ranks)[:4]}")
            assert err <= 10 * e_step
        assert falls >= 1
    finally:
        W.wenott_set_pivot_wait_limit(-1)
        s.close()


def test_batched_pivot_fallback(W):
    """The same forced give-up in lock-step batched stepping: each failed job's block is evaluated
    again and searched one launch per step; the batched states match the oracle."""
    flows = [workloads.config5_tilted_sod_3d(96, seed=sd) for sd in (0, 4)]
    _say("case: batched pivot fallback, two tilted Sod states 96^3")
    solvers = [W.Solver(f, W.default_opts(eps_mode=1, eps0=f.eps0)) for f in flows]
    W.wenott_set_pivot_wait_limit(0)
    try:
        us = [s.dense() for s in solvers]
        e_steps = [EpsTracker(f, u, eps0=f.eps0)(u) for f, u in zip(flows, us)]
        dts = [f.cfl * min(f.h) / s.max_wavespeed() for f, s in zip(flows, solvers)]
        W.wenott_batch_rk3_step([s.ctx for s in solvers], dts)
        falls = 0
        for f, s, u, dt, e_step in zip(flows, solvers, us, dts, e_steps):
            info = s.info()
            falls += info.pivot_fallbacks
            oracle_problem(f).ssprk3(u, dt, alphas=[info.alpha[i] for i in range(3)])
            err = rel_err(s.dense(), u)
            _say(f"  {f.note}: err {err:.3e} eps {e_step:.3e} fallbacks {info.pivot_fallbacks}")
            assert err <= 10 * e_step
        assert falls >= 1
    finally:
        W.wenott_set_pivot_wait_limit(-1)
        for s in solvers:
            s.close()
