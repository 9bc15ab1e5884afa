"""The two scalar laws of Sec. 5.1 and 5.2 through the TT path (one component, unit velocity along
every axis): 3D linear advection (f = u, alpha = 1) and 3D Burgers (f = u^2 / 2, alpha = max |u|).

* Step parity: steps of the library from the densified state against the oracle's scalar modes
  with the alphas the step used, each within 10 eps_TT, the eps computed here from eq.
  eps-tt-formula with the C_eps the paper gives for the problem.
* Tables 1 and 2: the TT solver run to T with dt = h^{5/3} and C_eps = 500 (linear advection) or
  10 (Burgers), its L2 error against the exact solution compared with the paper's tensor-train
  column and with the dense oracle on the same grid.
(needs a GPU)
"""
import dataclasses
import math
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_util import EpsTracker, dense_of_cores, oracle_problem, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def W():
    from paper_2405_12301_amd import wenott
    wenott.load()
    oracle.build(force=False)
    return wenott


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _golden(name):
    rows = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                n, ft, tt = line.split()
                rows[int(n)] = (float(ft), float(tt))
    return rows


def _l2(v):
    return float(np.sqrt(np.mean(v * v)))  # h^{3/2} ||v||_F on the unit cube


def _flow(law, n):
    return workloads.scalar_linadv_3d(n) if law == "linadv" else workloads.scalar_burgers_3d(n)


def _scalar_2d(law):
    """A ragged 2D transmissive case: the density of a random positive state as the scalar."""
    f = workloads.random_positive_tt((37, 29), rank=4, seed=21, amp=0.3, bc=(1, 1))
    return dataclasses.replace(f, cores=[f.cores[0]], law=1 if law == "linadv" else 2, c_eps=0.0,
                               eps_mode=0, eps0=1e-9)


# The Burgers solution under C_eps = 10 needs TT ranks close to N on these grids, grown from the
# rank-3 initial state within the first step: one column per index tuple (one component) lets a
# sweep add only kick_rank pivots, so its crosses take kick 8 and up to 8 sweeps.
BURGERS_CROSS = dict(kick_rank=8, max_sweeps=8)


def _opts(W, f, **kw):
    extra = BURGERS_CROSS if f.law == 2 else {}
    return W.default_opts(eps_mode=1, eps0=0.0, c_eps=f.c_eps, **extra, **kw)


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("law", ["linadv", "burgers"])
def test_scalar_3d_steps_vs_oracle(W, law, scheme):
    f = _flow(law, 24)
    _say(f"case: {law} 3D 24^3 scheme {scheme}, C_eps {f.c_eps}, 4 steps of dt = h^(5/3) against the oracle")
    s = W.Solver(f, _opts(W, f, scheme=scheme))
    P = oracle_problem(f)
    try:
        eps_of = EpsTracker(f, s.dense(), c_eps=f.c_eps)
        for step in range(4):
            u = s.dense()
            e_step = eps_of(u)
            s.step(f.fixed_dt)
            info = s.info()
            assert abs(info.eps - e_step) <= 1e-10 * e_step, (info.eps, e_step)
            alphas = [info.alpha[j] for j in range(3)]
            if law == "linadv":
                assert alphas == [1.0, 1.0, 1.0]
            P.ssprk3(u, f.fixed_dt, alphas=alphas)
            err = rel_err(s.dense(), u)
            _say(f"  step {step} ranks {list(info.ranks)[:4]} alphas {alphas} eps {e_step:.3e} err {err:.3e}")
            assert err <= 10 * e_step, (step, err, e_step)
    finally:
        s.close()


@pytest.mark.parametrize("law", ["linadv", "burgers"])
def test_scalar_2d_ragged_transmissive_step(W, law):
    f = _scalar_2d(law)
    _say(f"case: {law} 2D {f.n} transmissive, fixed eps 1e-9, 3 steps against the oracle")
    s = W.Solver(f, W.default_opts(eps_mode=0, eps0=1e-9, alpha_mode=0))
    P = oracle_problem(f)
    try:
        for step in range(3):
            u = s.dense()
            a = s.max_wavespeed()
            ref_a = P.alpha(u)
            assert abs(a - ref_a) <= 1e-13 * ref_a, (a, ref_a)
            dt = 0.4 * min(f.h) / a
            s.step(dt)
            info = s.info()
            P.ssprk3(u, dt, alphas=[info.alpha[j] for j in range(3)])
            err = rel_err(s.dense(), u)
            _say(f"  step {step} alpha {a!r} ranks {list(info.ranks)[:3]} err {err:.3e}")
            assert err <= 10 * 1e-9, (step, err)
    finally:
        s.close()


def test_burgers_alpha_line_search(W):
    f = workloads.scalar_burgers_3d(48)
    s = W.Solver(f, W.default_opts(alpha_mode=1, eps_mode=1, eps0=0.0, c_eps=f.c_eps))
    try:
        a = s.max_wavespeed()
        ref = oracle_problem(f).alpha(dense_of_cores(f.cores))
        _say(f"case: Burgers alpha line search 48^3: {a!r} exact {ref!r}")
        assert a <= ref * (1 + 1e-12) and a >= 0.99 * ref
    finally:
        s.close()


def test_scalar_law_options_rejected(W):
    """The proposal is built for the Euler law; a state whose component count is not the law's and
    an unknown law are rejected at init."""
    f = _flow("linadv", 12)
    with pytest.raises(W.WenottError) as e:
        W.Solver(f, W.default_opts(eps_mode=1, eps0=0.0, c_eps=f.c_eps, use_proposal=1))
    assert e.value.status == W.EINVAL
    euler = workloads.config3_wave_3d(12, seed=0, modes=2)
    for bad in (dataclasses.replace(euler, law=1), dataclasses.replace(f, law=0), dataclasses.replace(f, law=3)):
        o = W.default_opts()
        o.law = bad.law
        with pytest.raises(W.WenottError) as e:
            W.wenott_init(bad.cores, bad.n, bad.lo, bad.hi, bad.gamma, bad.bc, o)
        assert e.value.status == W.EINVAL


def _run_to_T(W, f, scheme):
    s = W.Solver(f, _opts(W, f, scheme=scheme))
    try:
        t, k, rmax = 0.0, 0, 0
        while t < f.t_end * (1.0 - 1e-14):
            dt = min(f.fixed_dt, f.t_end - t)
            s.step(dt)
            t += dt
            k += 1
            rmax = max(rmax, max(list(s.info().ranks)[:4]))
        return s.dense(), k, rmax, list(s.info().ranks)[:4]
    finally:
        s.close()


def _columns(W, law, scheme, sizes):
    ref = _golden("table1_linear_advection.txt" if law == "linadv" else "table2_burgers.txt")
    errs, ft = {}, {}
    for N in sizes:
        f = _flow(law, N)
        u, steps, rmax, ranks = _run_to_T(W, f, scheme)
        errs[N] = _l2(u[0] - f.exact(f.t_end)[0])
        U = dense_of_cores(f.cores)
        oracle_problem(f).run(U, f.t_end, fixed_dt=f.fixed_dt)
        ft[N] = _l2(U[0] - f.exact(f.t_end)[0])
        _say(f"  {law} scheme {scheme} N={N}: {steps} steps, final ranks {ranks} (max {rmax}); TT L2 {errs[N]:.3e} "
             f"(paper TT {ref[N][1]:.3e}, ratio {errs[N] / ref[N][1]:.3f}); oracle FT L2 {ft[N]:.3e} "
             f"(paper FT {ref[N][0]:.3e}); TT / FT {errs[N] / ft[N]:.3f}")
    pairs = list(zip(sizes[:-1], sizes[1:]))
    orders = [math.log2(errs[a] / errs[b]) / math.log2(b / a) for a, b in pairs]
    porders = [math.log2(ref[a][1] / ref[b][1]) / math.log2(b / a) for a, b in pairs]
    _say(f"  {law} scheme {scheme} orders {[round(o, 3) for o in orders]} (paper TT {[round(o, 3) for o in porders]})")
    return ref, errs, ft, orders, porders


@pytest.mark.parametrize("law", ["linadv", "burgers"])
def test_table_tt_column(W, law):
    """Table 1 (Sec. 5.1) or Table 2 (Sec. 5.2), tensor-train column at 10^3 to 80^3, with the
    paper's pipeline: per direction a cross of the numerical flux, the shift difference, the TT sum
    of the stage terms and one rounding (scheme 1)."""
    ref, errs, ft, orders, porders = _columns(W, law, 1, (10, 20, 40, 80))
    for N in errs:
        # the TT solution carries the scheme's own error: within 25 % of the dense oracle's
        assert abs(errs[N] / ft[N] - 1.0) <= 0.25, (N, errs[N], ft[N])
    assert orders[-1] >= 4.5
    if law == "linadv":
        # the oracle reproduces Table 1's full-tensor column to 1 %, and the TT column is held to
        # 25 % of the printed tensor-train values; the orders from 20^3 on to 0.15 of the printed
        # ones (at 10^3 eps_TT is 7e-3 and the truncation lowers the error below the dense one)
        for N in errs:
            assert abs(errs[N] / ref[N][1] - 1.0) <= 0.25, (N, errs[N], ref[N][1])
        for o, po in list(zip(orders, porders))[1:]:
            assert abs(o - po) <= 0.15, (orders, porders)
    else:
        # Table 2 prints larger full-tensor errors than the oracle gives (2.3x at 20^3, 3.5x at
        # 40^3); the TT column shares that offset, so only the factor 4 of the oracle's pin holds
        for N in errs:
            assert ref[N][1] / 4 < errs[N] < ref[N][1] * 4, (N, errs[N], ref[N][1])


def test_table1_stage_cross_column(W):
    """Table 1 with the stage cross (scheme 0): one cross of the whole stage value, whose
    interpolation error is relative to the state rather than to dt times the flux difference.
    Reported against the dense oracle; its error stays within 3x of the dense one."""
    ref, errs, ft, orders, porders = _columns(W, "linadv", 0, (20, 40, 80))
    for N in errs:
        assert errs[N] <= 3.0 * ft[N], (N, errs[N], ft[N])
