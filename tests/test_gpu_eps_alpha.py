"""The dynamic eps_TT, the Lax-Friedrichs alpha and the densification, each against a value
computed here from the densified state (needs a GPU).

* eq. eps-tt-formula (Sec. 4.6) in d dimensions: eps = C_eps V^{1/2} h^{5 - d/2} / max_q ||q||_F,
  on grids with unequal cell sizes (h is their geometric mean) and boxes of volume != 1, with
  C_eps given and with C_eps fixed by eps(0) = eps0.
* alpha (eq. lax-friedrichs, Sec. 4.2): the exact mode against the oracle's maximum over every
  cell; the line-search estimate (the tt_max_abs role of eq. cfl-other) is a lower bound of it.
* to_dense in 3D against the oracle's chain product of the cores (eq. TT_def_2), element by
  element.
"""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import EpsTracker, dense_of_cores, eps_formula, oracle_problem

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


def _aniso(ndim):
    """A random positive state on a box with unequal sides and cells (transmissive)."""
    if ndim == 2:
        f = workloads.random_positive_tt((48, 40), rank=4, seed=11, amp=0.3, bc=(1, 1))
        return dataclasses.replace(f, lo=(0.0, -1.0), hi=(1.5, 1.0))
    f = workloads.random_positive_tt((24, 20, 16), rank=3, seed=12, amp=0.3, bc=(1, 1, 1))
    return dataclasses.replace(f, lo=(0.0, 0.0, 0.0), hi=(1.0, 2.0, 0.5))


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("given", ["c_eps", "eps0"])
def test_dynamic_eps_formula(W, ndim, given):
    f = _aniso(ndim)
    u0 = dense_of_cores(f.cores)
    c_eps = 3.0e-4
    if given == "c_eps":
        opts = W.default_opts(eps_mode=1, eps0=0.0, c_eps=c_eps)
        want = EpsTracker(f, u0, c_eps=c_eps)
    else:
        opts = W.default_opts(eps_mode=1, eps0=2e-9)
        want = EpsTracker(f, u0, eps0=2e-9)
    _say(f"case: dynamic eps, {ndim}D {f.n} on {f.lo}..{f.hi}, {given}")
    s = W.Solver(f, opts)
    try:
        e0 = s.eps()
        _say(f"  t=0: library {e0!r} formula {want(u0)!r}")
        assert abs(e0 - want(u0)) <= 1e-12 * want(u0)
        if given == "eps0":
            assert abs(e0 - 2e-9) <= 1e-12 * 2e-9
        P = oracle_problem(f)
        for step in range(3):
            u = s.dense()
            dt = 0.4 * min(P.h) / P.alpha(u)
            s.step(dt)
            info = s.info()
            # the eps of the step is the formula on the state before it
            assert abs(info.eps - want(u)) <= 1e-12 * want(u), (step, info.eps, want(u))
            u1 = s.dense()
            _say(f"  step {step}: eps used {info.eps!r} formula {want(u):.15e}; now {s.eps()!r} "
                 f"formula {want(u1)!r} C_eps {info.c_eps!r}")
            assert abs(s.eps() - want(u1)) <= 1e-12 * want(u1)
            assert abs(info.c_eps - want.c_eps) <= 1e-12 * want.c_eps
        # the formula itself, once more spelled out with the grid of the flow
        d = len(f.n)
        h = float(np.prod(f.h)) ** (1.0 / d)
        vol = float(np.prod(np.array(f.hi) - np.array(f.lo)))
        u1 = s.dense()
        direct = want.c_eps * np.sqrt(vol) * h ** (5 - d / 2) / max(np.linalg.norm(u1[c]) for c in range(d + 2))
        assert abs(direct - eps_formula(f, u1, want.c_eps)) <= 1e-14 * direct
    finally:
        s.close()


@pytest.mark.parametrize("which", ["wave24", "random"])
def test_to_dense_3d_elementwise(W, which):
    f = workloads.config3_wave_3d(24, seed=0, modes=4) if which == "wave24" else \
        workloads.random_positive_tt((13, 17, 11), rank=6, seed=5, rough=True)
    _say("case: to_dense 3D", which, f.n)
    s = W.Solver(f)
    try:
        got = s.dense()
        ref = dense_of_cores(f.cores)
        err = np.max(np.abs(got - ref))
        _say(f"  max |to_dense - tt_full| = {err:.3e}")
        assert err <= 1e-13 * max(1.0, np.max(np.abs(ref)))
        dev = s.dense(device=True).cpu().numpy()
        assert np.array_equal(dev, got)
    finally:
        s.close()


@pytest.mark.parametrize("case", ["quadrants2d", "wave3d", "tilted_sod3d", "blast3d"])
def test_alpha_line_search_is_a_tight_lower_bound(W, case):
    """The estimate never exceeds the exact maximum (it is the maximum over visited cells) and on
    these workloads reaches it to within 1 % (printed)."""
    if case == "quadrants2d":
        f = workloads.config2_quadrants_2d(128, seed=3)
    elif case == "wave3d":
        f = workloads.config3_wave_3d(48, seed=1, modes=8)
    elif case == "tilted_sod3d":
        f = workloads.config5_tilted_sod_3d(64, seed=4)
    else:
        f = workloads.config4_blast_3d(seed=2, n=(48, 40, 56))
    _say("case: alpha line search,", case, f.n)
    # each flow at its own eps_TT; the blast's crosses stop at the cross-rank limit (explicit slack)
    est = W.Solver(f, W.default_opts(alpha_mode=1, eps_mode=f.eps_mode, eps0=f.eps0,
                                     conv_slack=100.0 if case == "blast3d" else 1.0))
    ex = W.Solver(f, W.default_opts(alpha_mode=0))
    try:
        ref = oracle_problem(f).alpha(dense_of_cores(f.cores))
        a1, a0 = est.max_wavespeed(), ex.max_wavespeed()
        _say(f"  estimate {a1!r} exact {a0!r} oracle {ref!r} ratio {a1 / ref:.6f}")
        assert abs(a0 - ref) <= 1e-12 * ref
        assert a1 <= ref * (1 + 1e-12)
        assert a1 >= 0.99 * ref
        # after a step the stages' alphas are estimates of the stage inputs (reported)
        dt = 0.4 * min(f.h) / a1
        est.step(dt)
        info = est.info()
        _say("  stage alphas", [info.alpha[i] for i in range(3)])
        assert all(info.alpha[i] > 0 for i in range(3))
    finally:
        est.close()
        ex.close()
