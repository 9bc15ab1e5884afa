"""Parity of the HIP WENO-TT path against the oracle, through the C ABI (needs a GPU)."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import tt_ref
from tests.gpu_util import EpsTracker, dense_of_cores, eps_formula, oracle_problem, rel_err

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


def assert_rhs_parity(got, Lref, u, P, alpha, eps):
    """Each flux cross is accurate to eps relative to the flux tensor (the cross bound of
    Sec. 3.3), the shift difference (T - 1)/h has norm <= 2/h, and the sum is rounded at eps:
    max_c ||L_TT - L||_F <= 10 eps (sum_d 2 max_c ||Fhat_d,c||_F / h_d + max_c ||L_c||_F)."""
    scale = sum(2.0 * max(np.linalg.norm(F[c]) for c in range(F.shape[0])) / P.h[d]
                for d, F in enumerate(P.interface_flux(u, alpha, d) for d in range(P.ndim)))
    scale += max(np.linalg.norm(Lref[c]) for c in range(Lref.shape[0]))
    err = max(np.linalg.norm(got[c] - Lref[c]) for c in range(got.shape[0]))
    assert err <= 10 * eps * scale, (err, eps * scale)


def test_to_dense_and_alpha_config1(W):
    _say("case: to_dense / alpha, smooth wave 2D 64^2")
    f = workloads.config1_smooth_wave_2d(64)
    s = W.Solver(f, W.default_opts(alpha_mode=0))
    try:
        got = s.dense()
        ref = dense_of_cores(f.cores)
        assert np.max(np.abs(got - ref)) < 1e-13
        a = s.max_wavespeed()
        assert abs(a - oracle_problem(f).alpha(ref)) < 1e-12
    finally:
        s.close()


# The rough cases keep their ranks (eps 1e-9): ~25 per bond re-orthonormalises on the matrix-core
# Gram kernel with two 16-column blocks, ~41 on the one-wave Cholesky of a split-K Gram.
@pytest.mark.parametrize("shape,rank,rough,eps", [((40, 33), 7, False, 1e-3), ((12, 10, 9), 5, False, 1e-3),
                                                  ((40, 33), 24, True, 1e-9), ((70, 60), 40, True, 1e-9),
                                                  ((20, 24, 18), 12, True, 1e-9)])
def test_round_error_bound_and_ranks(W, shape, rank, rough, eps):
    _say("case: round", shape, rank, "rough" if rough else "smooth", eps)
    f = workloads.random_positive_tt(shape, rank, seed=3, rough=rough)
    ref = dense_of_cores(f.cores)
    s = W.Solver(f)
    try:
        s.round(eps)
        cores = s.state_cores()
        got = dense_of_cores(cores)
        for c in range(ref.shape[0]):
            err = np.linalg.norm(got[c] - ref[c])
            assert err <= eps * np.linalg.norm(ref[c]) * (1 + 1e-9) + 1e-14, (c, err)
            want = tt_ref.tt_ranks(tt_ref.tt_svd(ref[c], eps))
            # common padded ranks: the largest component rank at each bond
        want_max = np.max([tt_ref.tt_ranks(tt_ref.tt_svd(ref[c], eps)) for c in range(ref.shape[0])], axis=0)
        got_r = tt_ref.tt_ranks(cores[0])
        _say("  ranks", got_r, "oracle", list(want_max))
        assert all(g <= w for g, w in zip(got_r, want_max)), (got_r, want_max)
    finally:
        s.close()


SCHEMES = [0, 1]


@pytest.mark.parametrize("n", [96, 128])
def test_exact_alpha_3d_register_path(W, n):
    """The exact alpha at 96^3 and 128^3 (9216 and 16384 rows of the left part, so each thread of
    the alpha kernel sweeps 4 and 8 rows with its column of the last core in registers) against
    the oracle's alpha of the densified state."""
    _say("case: exact alpha 3D smooth wave", n)
    f = workloads.config3_wave_3d(n, seed=0)
    s = W.Solver(f, W.default_opts(alpha_mode=0))
    try:
        ref = dense_of_cores(f.cores)
        a = s.max_wavespeed()
        want = oracle_problem(f).alpha(ref)
        _say(f"  alpha {a!r} oracle {want!r}")
        assert abs(a - want) <= 1e-12 * want
    finally:
        s.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_rhs_matches_oracle_config1(W, scheme):
    _say("case: rhs, smooth wave 2D 64^2, scheme", scheme)
    f = workloads.config1_smooth_wave_2d(64)
    eps = 1e-10
    s = W.Solver(f, W.default_opts(eps0=eps, scheme=scheme))
    try:
        ref_u = dense_of_cores(f.cores)
        P = oracle_problem(f)
        a = P.alpha(ref_u)
        Lref = P.rhs(ref_u, a)
        got = dense_of_cores(s.rhs_cores(a))
        info = s.info()
        _say("rhs rel err", rel_err(got, Lref), "cross residuals", info.residual[0][0], info.residual[0][1])
        if scheme == 0:
            # the cross of L(U) itself is accurate to eps relative to L(U); one rounding at eps
            assert rel_err(got, Lref) <= 10 * eps
        else:
            assert_rhs_parity(got, Lref, ref_u, P, a, eps)
    finally:
        s.close()


@pytest.mark.parametrize("scheme", SCHEMES)
def test_rk3_step_matches_oracle_config1(W, scheme):
    _say("case: rk3 step, smooth wave 2D 64^2, scheme", scheme)
    f = workloads.config1_smooth_wave_2d(64)
    eps = 1e-10
    s = W.Solver(f, W.default_opts(eps0=eps, scheme=scheme))
    try:
        u = dense_of_cores(f.cores)
        P = oracle_problem(f)
        dt = 0.5 * min(P.h) / P.alpha(u)
        s.step(dt)
        info = s.info()
        al = [info.alpha[i] for i in range(3)]
        P.ssprk3(u, dt, alphas=al)
        got = s.dense()
        e = rel_err(got, u)
        _say("step rel err", e, "ranks", list(info.ranks), "alphas", al)
        assert e <= 10 * eps
    finally:
        s.close()


@pytest.mark.parametrize("which", ["wave", "quadrants"])
def test_dense_comparator_matches_oracle(W, which):
    import torch
    _say("case: dense comparator", which)
    f = workloads.config1_smooth_wave_2d(64) if which == "wave" else workloads.config2_quadrants_2d(64, seed=1)
    u = dense_of_cores(f.cores)
    P = oracle_problem(f)
    ctx = W.wenott_dense_init(f.n, f.lo, f.hi, f.gamma, f.bc)
    try:
        U = torch.from_numpy(u.copy()).cuda()
        a = W.wenott_dense_max_wavespeed(ctx, U)
        assert abs(a - P.alpha(u)) <= 1e-14 * a
        dt = 0.5 * min(P.h) / a
        for _ in range(3):
            al = W.wenott_dense_rk3_step(ctx, U, dt)
            P.ssprk3(u, dt, alphas=al)
        got = U.cpu().numpy()
        assert rel_err(got, u) < 1e-13
    finally:
        W.wenott_dense_destroy(ctx)


def step_eps(o, f, u0):
    """eps_TT of each step computed here, not read from the library: the fixed eps0, or eq.
    eps-tt-formula on the densified state before the step with C_eps fixed by eps0 on u0 (or the
    given C_eps)."""
    if o.eps_mode == 0:
        return lambda u: o.eps0
    if o.eps0 > 0:
        return EpsTracker(f, u0, eps0=o.eps0)
    return EpsTracker(f, u0, c_eps=o.c_eps)


def _step_parity(W, f, eps, nsteps=1, opts=None, tol_factor=10.0, scheme=0, sweeps_out=None):
    """Advance the TT path and the oracle from the same densified state with the same dt and
    the alphas the TT path used; per-step error in the max_c ||.||_F / max_c ||.||_F norm,
    bounded by tol_factor times the eps_TT this test computes itself (and the library's eps is
    checked against it). sweeps_out, if given, receives each step's per-stage sweep counts."""
    o = opts if opts is not None else W.default_opts(eps0=eps, scheme=scheme)
    s = W.Solver(f, o)
    try:
        P = oracle_problem(f)
        errs = []
        eps_of = None
        for _ in range(nsteps):
            u = s.dense()
            if eps_of is None:
                eps_of = step_eps(o, f, u)
            e_ind = eps_of(u)
            dt = 0.5 * min(P.h) / P.alpha(u)
            s.step(dt)
            info = s.info()
            al = [info.alpha[i] for i in range(3)]
            P.ssprk3(u, dt, alphas=al)
            e = rel_err(s.dense(), u)
            errs.append(e)
            if sweeps_out is not None:
                sweeps_out.append([info.sweeps[j][0] for j in range(3)])
            _say("  step err", e, "eps", e_ind, "ranks", list(info.ranks), "sweeps",
                 [list(r) for r in info.sweeps], "sum ranks", list(info.sum_rank))
            assert abs(info.eps - e_ind) <= 1e-10 * e_ind, (info.eps, e_ind)
            assert e <= tol_factor * e_ind, (e, e_ind)
        return errs
    finally:
        s.close()


def test_stage_cross_rejected_warm_sweep(W):
    """A stage cross whose first (warm-started) sweep misses eps: the TT-rounding queued behind
    that sweep's residual check is dropped, the refresh and second sweep run, and the step still
    matches the oracle. Without the random kick the warm index sets cannot grow in the first
    sweep, so the rank growth of the four-quadrant problem at eps 1e-10 forces such a stage."""
    _say("case: rejected warm sweep, four-quadrant 2D 48^2, eps 1e-10, no kick")
    f = workloads.config2_quadrants_2d(48, seed=1)
    sw = []
    _step_parity(W, f, 1e-10, nsteps=4, opts=W.default_opts(eps0=1e-10, eps_mode=0, kick_rank=0), sweeps_out=sw)
    assert any(n >= 2 for st in sw[1:] for n in st), sw


@pytest.mark.parametrize("mode", [7, 8, 9])
def test_resident_operand_contractions_3d(W, mode):
    """The resident-operand matrix-core contraction shapes (5: A resident; 6, 7: B resident in
    64- and 32-column groups) forced on every product they fit, through 3D steps whose gathers
    have other row, column and reduction counts than the 2D ones (ranks of a wave with 8 modes,
    K on both sides of 32): each step within 10 eps of the oracle."""
    _say("case: forced contraction shape", mode - 2, "on a 3D wave 24^3 with 8 modes")
    f = workloads.config3_wave_3d(24, seed=0, modes=8)
    W.wenott_gemm_autotune(mode)
    try:
        _step_parity(W, f, 1e-9, nsteps=2)
    finally:
        W.wenott_gemm_autotune(1)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_step_parity_3d_smooth(W, scheme):
    _say("case: rk3 step, 3D smooth wave 24^3 with 2 Fourier modes, scheme", scheme)
    f = workloads.config3_wave_3d(24, seed=0, modes=2)
    _step_parity(W, f, 1e-9, nsteps=2, scheme=scheme)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("n", [(64, 64), (37, 29)])
def test_step_parity_quadrants_shocks(W, n, scheme):
    _say("case: rk3 steps, four-quadrant Riemann problem", n, "scheme", scheme)
    f = workloads.config2_quadrants_2d(64, seed=2)
    if n != (64, 64):
        import dataclasses
        g = workloads.config2_quadrants_2d(max(n), seed=2)
        # ragged grid: resample the quadrant cores on an n0 x n1 grid
        cores = []
        for comp in g.cores:
            c0 = np.zeros((1, n[0], 2)); c0[0, :, 0] = np.arange(n[0]) < n[0] // 2; c0[0, :, 1] = 1 - c0[0, :, 0]
            vals = comp[1][:, [0, -1], 0]  # (2 quadrants in x) x (low/high y)
            c1 = np.zeros((2, n[1], 1))
            for a in range(2):
                c1[a, :, 0] = np.where(np.arange(n[1]) < n[1] // 2, vals[a, 0], vals[a, 1])
            cores.append([c0, c1])
        f = dataclasses.replace(g, n=n, cores=cores)
    _step_parity(W, f, 1e-8, nsteps=3, scheme=scheme)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("ndim", [2, 3])
def test_full_rank_exactness_8d(W, ndim, scheme):
    _say("case: full-rank exactness on 8^d, random smooth state, d =", ndim, "scheme", scheme)
    f = workloads.random_positive_tt((8,) * ndim, rank=8, seed=7, amp=0.3)
    _step_parity(W, f, 1e-13, nsteps=1, tol_factor=10, scheme=scheme)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_sod_stays_rank_one_and_matches(W, scheme):
    _say("case: axis-aligned Sod in 3D stays rank 1, scheme", scheme)
    f = workloads.sod_1d_like(3, 32)
    s = W.Solver(f, W.default_opts(eps_mode=0, eps0=1e-8, scheme=scheme))
    try:
        P = oracle_problem(f)
        u = s.dense()
        for _ in range(3):
            dt = 0.5 * min(P.h) / P.alpha(u)
            s.step(dt)
            info = s.info()
            P.ssprk3(u, dt, alphas=[info.alpha[i] for i in range(3)])
        ranks = list(info.ranks)[:4]
        _say(f"  ranks {ranks} err {rel_err(s.dense(), u):.3e}")
        if scheme == 0:
            assert ranks == [1, 1, 1, 1]
        else:
            # the per-direction flux crosses are accurate to eps relative to the fluxes; the
            # y and z fluxes are constant along their own direction and their shift differences
            # cancel only to that accuracy, which leaves singular values at the truncation
            # threshold (eps ||X|| / sqrt(d - 1)): one of them may survive the rounding
            assert max(ranks) <= 3
        assert rel_err(s.dense(), u) <= 1e-7
    finally:
        s.close()


@pytest.mark.parametrize("case", ["wave3d", "quadrants"])
def test_fp32_fiber_path_error(W, case):
    """Reduced-precision path: gathers on the FP32 matrix cores and FP32 LF + WENO5 in the
    fiber kernel; pivots, rounding and the error estimator in FP64. The error against the FP64
    oracle is reported and bounded by 10 eps_cross + 1e-7 per step."""
    _say("case: FP32 fiber path,", case)
    if case == "wave3d":
        f = workloads.config3_wave_3d(24, seed=0, modes=8)
        eps = 1e-6
    else:
        f = workloads.config2_quadrants_2d(64, seed=2)
        eps = 1e-8
    res = {}
    for prec in (0, 1):
        s = W.Solver(f, W.default_opts(eps0=eps, precision=prec))
        try:
            P = oracle_problem(f)
            u = s.dense()
            dt = 0.5 * min(P.h) / P.alpha(u)
            s.step(dt)
            info = s.info()
            P.ssprk3(u, dt, alphas=[info.alpha[i] for i in range(3)])
            got = s.dense()
            res[prec] = (rel_err(got, u), got, list(info.ranks))
        finally:
            s.close()
    e64, e32 = res[0][0], res[1][0]
    d = rel_err(res[1][1], res[0][1])
    _say(f"  FP64 path err {e64:.3e}  FP32 path err {e32:.3e}  FP32 vs FP64 path {d:.3e}  ranks {res[0][2]} {res[1][2]}")
    assert e32 <= 10 * max(eps, 1e-6)
