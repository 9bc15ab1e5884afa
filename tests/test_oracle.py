"""Pins of the oracle against what the paper and the mathematics fix (CPU only).

Every check here compares the dense FP64 oracle with something other than itself:
printed paper values, exact solutions, closed forms, invariants, or brute force.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import riemann, tt_ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def _cube(N, model):
    return oracle.Problem((N, N, N), (0, 0, 0), (1, 1, 1), (0, 0, 0), model=model)


def _l2(v):
    return float(np.sqrt(np.mean(v * v)))  # h^{3/2} ||v||_F on the unit cube


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# --- Table 1 (Sec. 5.1): 3D linear advection, full-tensor column ---------------------
@pytest.mark.parametrize("N", [10, 20, 40])
def test_table1_linear_advection_full_tensor(N):
    ref = {int(r[0]): float(r[1]) for r in _golden("table1_linear_advection.txt")}
    P = _cube(N, oracle.LINADV)
    x = P.centers(0)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    U = np.sin(2 * np.pi * (X + Y + Z))[None].copy()
    P.run(U, 0.1, fixed_dt=(1.0 / N) ** (5.0 / 3.0))
    err = _l2(U[0] - np.sin(2 * np.pi * (X + Y + Z - 0.3)))
    # the printed values carry three digits
    assert abs(err / ref[N] - 1.0) < 0.01, (N, err, ref[N])


# --- Sec. 5.2: 3D Burgers, against the exact solution by characteristics -------------
def _burgers_exact(xi, t):
    u = 0.5 + 0.5 * np.sin(2 * np.pi * xi)
    for _ in range(100):  # u = u0(xi - 3 u t), Newton
        a = 2 * np.pi * (xi - 3 * u * t)
        g = u - (0.5 + 0.5 * np.sin(a))
        u = u - g / (1 + 3 * np.pi * t * np.cos(a))
    return u


def test_burgers_exact_and_table2_magnitude():
    T = 1.0 / (12.0 * np.pi)
    errs = []
    for N in (20, 40):
        P = _cube(N, oracle.BURGERS)
        x = P.centers(0)
        X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
        U = (0.5 + 0.5 * np.sin(2 * np.pi * (X + Y + Z)))[None].copy()
        P.run(U, T, fixed_dt=(1.0 / N) ** (5.0 / 3.0))
        errs.append(_l2(U[0] - _burgers_exact(X + Y + Z, T)))
    order = math.log2(errs[0] / errs[1])
    assert order > 4.5, errs
    # Table 2 prints larger errors (by 2.3x at 20^3 and 3.5x at 40^3) than this reading of
    # the scheme gives; both must at least agree within a factor of 4.
    ref = {int(r[0]): float(r[1]) for r in _golden("table2_burgers.txt")}
    for N, e in zip((20, 40), errs):
        assert ref[N] / 4 < e < ref[N] * 4, (N, e, ref[N])


# --- Sec. 5.5: Sod shock tube against the exact Riemann solution ---------------------
def test_exact_riemann_solver_self_consistent():
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    ps, us = riemann.star_state(L, R)
    assert riemann.pressure_function_residual(L, R, ps) < 1e-14
    # Rankine-Hugoniot across the right shock: mass and momentum fluxes continuous
    g = 1.4
    rs = R[0] * (ps / R[2] + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / R[2] + 1)
    S = (rs * us - R[0] * R[1]) / (rs - R[0])
    mom_l = rs * us * (us - S) + ps
    mom_r = R[0] * R[1] * (R[1] - S) + R[2]
    assert abs(mom_l - mom_r) < 1e-13
    # energy flux continuity
    El = ps / (g - 1) + 0.5 * rs * us * us
    Er = R[2] / (g - 1)
    assert abs((El + ps) * us - S * El - ((Er + R[2]) * R[1] - S * Er)) < 1e-13
    # the rarefaction's tail state lies on the left isentrope with the left Riemann invariant
    rl_star = L[0] * (ps / L[2]) ** (1 / g)
    a_l, a_star = math.sqrt(g * L[2] / L[0]), math.sqrt(g * ps / rl_star)
    assert abs((L[1] + 2 * a_l / (g - 1)) - (us + 2 * a_star / (g - 1))) < 1e-13


def test_sod_converges_to_exact():
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    errs = []
    for N in (100, 200, 400, 800):
        P = oracle.Problem((N,), (0.0,), (1.0,), (oracle.BC_TRANSMISSIVE,))
        x = P.centers(0)
        left = x < 0.5
        U = np.stack([np.where(left, 1.0, 0.125), 0 * x, np.where(left, 1.0, 0.1) / 0.4]).copy()
        P.run(U, 0.2, cfl=0.5)
        rho_ex, _, _ = riemann.sample(L, R, (x - 0.5) / 0.2)
        errs.append(float(np.mean(np.abs(U[0] - rho_ex))))
        # ENO: no over/undershoot beyond 1% of the largest jump
        assert U[0].max() < 1.0 + 0.01 * 0.875 and U[0].min() > 0.125 - 0.01 * 0.875
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1.2e-3


# --- smooth order (Sec. 2.2: fifth order) --------------------------------------------
def test_fifth_order_smooth_density_wave_2d():
    errs = []
    for N in (32, 64, 128):
        P = oracle.Problem((N, N), (0, 0), (2, 2), (0, 0))
        x, y = P.centers(0), P.centers(1)
        X, Y = np.meshgrid(x, y, indexing="ij")
        rho = 1 + 0.2 * np.sin(np.pi * (X + Y))
        U = np.stack([rho, rho, rho, 2.5 + rho]).copy()
        T = 0.1
        P.run(U, T, fixed_dt=0.5 * (2.0 / N) ** (5 / 3))
        errs.append(float(np.sqrt(np.mean((U[0] - (1 + 0.2 * np.sin(np.pi * (X + Y - 2 * T)))) ** 2))))
    orders = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert orders[-1] > 4.8, (errs, orders)


# --- conservation with periodic boundaries --------------------------------------------
def _random_state(shape, rng):
    ndim = len(shape)
    rho = 1 + 0.3 * rng.uniform(-1, 1, size=shape)
    mom = [0.4 * rng.uniform(-1, 1, size=shape) for _ in range(ndim)]
    p = 1 + 0.3 * rng.uniform(-1, 1, size=shape)
    E = p / 0.4 + 0.5 * sum(m * m for m in mom) / rho
    return np.stack([rho] + mom + [E]).copy()


@pytest.mark.parametrize("n", [(12, 10), (8, 10, 6)])
def test_conservation_periodic(n):
    rng = np.random.default_rng(3)
    P = oracle.Problem(n, (0,) * len(n), (1,) * len(n), (0,) * len(n))
    U = _random_state(n, rng)
    tot0 = U.reshape(U.shape[0], -1).sum(axis=1)
    for _ in range(10):
        a = P.alpha(U)
        P.ssprk3(U, 0.3 * min(P.h) / a)
    tot = U.reshape(U.shape[0], -1).sum(axis=1)
    scale = np.abs(U).reshape(U.shape[0], -1).sum(axis=1)
    assert np.all(np.abs(tot - tot0) <= 1e-12 * scale), (tot - tot0) / scale


# --- brute force: naive per-point twin on 8^d grids -----------------------------------
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("bc", [oracle.BC_PERIODIC, oracle.BC_TRANSMISSIVE])
def test_naive_twin(ndim, bc):
    rng = np.random.default_rng(ndim * 10 + bc)
    n = (8,) * ndim
    P = oracle.Problem(n, (0,) * ndim, (1.3,) * ndim, (bc,) * ndim)
    U = _random_state(n, rng)
    a = P.alpha(U)
    L1 = P.rhs(U, a)
    L2 = P.rhs(U, a, naive=True)
    assert np.max(np.abs(L1 - L2)) <= 1e-14 * np.max(np.abs(L1))


# --- closed forms of the reconstruction ----------------------------------------------
def test_weno_reproduces_linear_data_exactly():
    # linear advection: f = u, alpha = 1 -> f^+ = u, f^- = 0; WENO5 of linear data is exact
    N = 20
    P = oracle.Problem((N,), (0.0,), (1.0,), (oracle.BC_TRANSMISSIVE,), model=oracle.LINADV)
    x = P.centers(0)
    U = (2.0 + 3.0 * x)[None].copy()
    F = P.interface_flux(U, 1.0, 0)[0]
    faces = np.arange(N + 1) * P.h[0]
    inner = slice(3, N - 2)  # faces whose stencils avoid the boundary extrapolation
    assert np.max(np.abs(F[inner] - (2.0 + 3.0 * faces[inner]))) < 1e-13


def test_weno_eno_at_a_step():
    # a unit step between cells 9 and 10: the face 3 cells away sees only one side, and the
    # face on the step takes (nearly) the upwind value
    N = 20
    P = oracle.Problem((N,), (0.0,), (1.0,), (oracle.BC_TRANSMISSIVE,), model=oracle.LINADV)
    U = (np.arange(N) >= 10).astype(float)[None].copy()
    F = P.interface_flux(U, 1.0, 0)[0]
    assert F[6] == 0.0 and abs(F[14] - 1.0) < 1e-15
    assert abs(F[10]) < 1e-3  # upwind side of the step for f^+ (left cell value 0)


def test_alpha_closed_form():
    P = oracle.Problem((4, 4), (0, 0), (1, 1), (0, 0))
    rho, u, v, p = 1.3, 0.4, -0.3, 0.9
    U = np.stack([np.full((4, 4), q) for q in (rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v))]).copy()
    assert abs(P.alpha(U) - (math.hypot(u, v) + math.sqrt(1.4 * p / rho))) < 1e-14


def test_nonphysical_state_is_an_error():
    P = oracle.Problem((8,), (0.0,), (1.0,), (oracle.BC_PERIODIC,))
    U = np.stack([np.ones(8), np.zeros(8), np.full(8, 2.5)]).copy()
    U[2, 3] = -1.0
    with pytest.raises(oracle.OracleError) as e:
        P.alpha(U)
    assert e.value.status == oracle.ENONPHYS
    with pytest.raises(oracle.OracleError):
        P.rhs(U, 2.0)


# --- invariants -----------------------------------------------------------------------
def test_x_only_data_matches_1d_bitwise():
    rng = np.random.default_rng(7)
    N = 16
    u1 = _random_state((N,), rng)
    P1 = oracle.Problem((N,), (0.0,), (1.0,), (oracle.BC_TRANSMISSIVE,))
    P2 = oracle.Problem((N, 5), (0, 0), (1, 5 / 16), (oracle.BC_TRANSMISSIVE, oracle.BC_PERIODIC))
    U2 = np.zeros((4, N, 5))
    U2[0] = u1[0][:, None]
    U2[1] = u1[1][:, None]
    U2[3] = u1[2][:, None]
    a = P1.alpha(u1)
    assert P2.alpha(U2) == a
    L1 = P1.rhs(u1, a)
    L2 = P2.rhs(U2, a)
    for j in range(5):
        assert np.array_equal(L2[0][:, j], L1[0]) and np.array_equal(L2[1][:, j], L1[1])
        assert np.array_equal(L2[3][:, j], L1[2]) and np.all(L2[2][:, j] == 0.0)


def test_axis_permutation_symmetry_3d():
    rng = np.random.default_rng(11)
    n = (6, 8, 7)
    P = oracle.Problem(n, (0, 0, 0), (0.6, 0.8, 0.7), (0, 1, 0))
    U = _random_state(n, rng)
    a = P.alpha(U)
    L = P.rhs(U, a)
    perm = (2, 0, 1)  # new axis k is old axis perm[k]
    Pp = oracle.Problem(tuple(n[i] for i in perm), (0, 0, 0), tuple((0.6, 0.8, 0.7)[i] for i in perm),
                        tuple((0, 1, 0)[i] for i in perm))
    Up = np.stack([U[0].transpose(perm)] + [U[1 + i].transpose(perm) for i in perm] + [U[4].transpose(perm)]).copy()
    Lp = Pp.rhs(Up, a)
    Lref = np.stack([L[0].transpose(perm)] + [L[1 + i].transpose(perm) for i in perm] + [L[4].transpose(perm)])
    assert np.max(np.abs(Lp - Lref)) <= 1e-13 * np.max(np.abs(L))


def test_reflection_symmetry_pins_the_minus_side():
    # mirror x -> -x with u -> -u: the f^- reconstruction must be the mirror of f^+
    rng = np.random.default_rng(5)
    N = 24
    P = oracle.Problem((N,), (0.0,), (1.0,), (oracle.BC_TRANSMISSIVE,))
    U = _random_state((N,), rng)
    a = P.alpha(U)
    L = P.rhs(U, a)
    Um = np.stack([U[0][::-1], -U[1][::-1], U[2][::-1]]).copy()
    Lm = P.rhs(Um, a)
    ref = np.stack([L[0][::-1], -L[1][::-1], L[2][::-1]])
    assert np.max(np.abs(Lm - ref)) <= 1e-13 * np.max(np.abs(L))


# --- tensor-train reference ------------------------------------------------------------
def test_tt_full_matches_separable_closed_form():
    x = np.linspace(0, 1, 7)
    y = np.linspace(0, 2, 5)
    z = np.linspace(-1, 1, 6)
    a, b, c = 1.3 * x, 0.7 * y, 2.1 * z
    g1 = np.stack([np.sin(a), np.cos(a)], -1)[None]
    g2 = np.empty((2, 5, 2))
    g2[0, :, 0], g2[0, :, 1], g2[1, :, 0], g2[1, :, 1] = np.cos(b), -np.sin(b), np.sin(b), np.cos(b)
    g3 = np.stack([np.cos(c), np.sin(c)], 0)[:, :, None]
    full = tt_ref.tt_full([g1, g2, g3])
    ref = np.sin(a[:, None, None] + b[None, :, None] + c[None, None, :])
    assert np.max(np.abs(full - ref)) < 1e-14
    # rank-1 TT is an outer product
    assert np.allclose(tt_ref.tt_full([x[None, :, None], y[None, :, None], z[None, :, None]]),
                       np.multiply.outer(np.multiply.outer(x, y), z), rtol=0, atol=1e-15)


def test_manufactured_solution_exact_ranks():
    want = {r[0]: int(r[1]) for r in _golden("manufactured_ranks.txt")}
    n = 20
    s = (np.arange(n) + 0.5) / n
    X, Y, Z = np.meshgrid(s, s, s, indexing="ij")
    th = 2 * np.pi * (X + Y + Z)
    rho = 1 + 0.1 * np.sin(th)
    u, v, w, e = 1 + 0.1 * np.sin(th), 1 + 0.1 * np.cos(th), 1 + 0.1 * np.cos(th), 1 + 0.1 * np.cos(th)
    fields = {"rho": rho, "rhou": rho * u, "rhov": rho * v, "rhow": rho * w,
              "rhoE": rho * (e + 0.5 * (u * u + v * v + w * w))}
    for k, f in fields.items():
        ranks = tt_ref.tt_ranks(tt_ref.tt_svd(f, 1e-12))
        assert ranks[1] == ranks[2] == want[k], (k, ranks)


def test_tt_svd_error_bound_and_exact_rank3_wave():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(6, 7, 8))
    for eps in (1e-1, 3e-2, 1e-3):
        cores = tt_ref.tt_svd(x, eps)
        assert np.linalg.norm(tt_ref.tt_full(cores) - x) <= eps * np.linalg.norm(x) * (1 + 1e-12)
    n = 64
    s = (np.arange(n) + 0.5) * (2.0 / n)
    rho = 1 + 0.2 * np.sin(np.pi * (s[:, None] + s[None, :]))
    assert tt_ref.tt_ranks(tt_ref.tt_svd(rho, 1e-12)) == [1, 3, 1]


def test_maxvol_brute_force_is_dominant():
    rng = np.random.default_rng(1)
    for n, r in ((6, 2), (8, 3), (10, 4)):
        a = rng.normal(size=(n, r))
        rows, vol = tt_ref.max_volume_rows(a)
        assert tt_ref.maxvol_dominant(a, rows)
        # a different subset with a smaller volume is not dominant in general
        assert vol > 0


# --- transmissive boundary after a wave has left the domain (reading C8) --------------
@pytest.mark.parametrize("side", ["high", "low"])
def test_transmissive_outflow_after_the_shock_leaves(side):
    """Sod run to t = 0.32: the right-moving shock (speed 1.752) left x = 1 at t = 0.285, the
    rarefaction head (speed -1.183) has not reached x = 0. Zero-order extrapolation lets the
    shock out: the whole domain stays within first-order discretisation error of the exact
    solution on the infinite line, also next to the boundary it crossed. A periodic ghost map
    would bring the other side's state in at t = 0 and a reflecting one would send a reflected
    shock back (an O(0.5) density error next to the wall). side = "low" mirrors the problem."""
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    N, t = 400, 0.32
    P = oracle.Problem((N,), (0.0,), (1.0,), (oracle.BC_TRANSMISSIVE,))
    x = P.centers(0)
    high = side == "high"
    left = x < 0.5 if high else x >= 0.5
    U = np.stack([np.where(left, 1.0, 0.125), 0 * x, np.where(left, 1.0, 0.1) / 0.4]).copy()
    P.run(U, t, cfl=0.5)
    xi = (x - 0.5) / t if high else (0.5 - x) / t
    rho_ex = riemann.sample(L, R, xi)[0]
    near = x >= 0.95 if high else x <= 0.05
    assert riemann.star_state(L, R)[1] > 0 and 0.5 + 1.7522 * 0.285 > 1.0 - 1e-3
    assert float(np.mean(np.abs(U[0] - rho_ex))) < 2.5e-3
    assert float(np.max(np.abs(U[0] - rho_ex)[near])) < 1e-2
    # the outflow state next to the boundary is the post-shock one (rho* = 0.2656)
    assert abs(U[0][-1 if high else 0] - 0.2656) < 5e-3


# --- the independent eps_TT of the GPU tests (eq. eps-tt-formula) ----------------------
def test_eps_formula_helper_hand_values():
    """eps = C V^{1/2} h^{5 - d/2} / max_q ||q||_F on a constant state, worked by hand:
    3D ones on 8^3 cells of [0,2]^3: V = 8, h = 1/4, ||q|| = sqrt(512), so eps = C sqrt(8) 2^-7 /
    sqrt(512) = C / 1024; 2D ones on 16 x 4 cells of [0,1] x [0,4]: h = (1/16 * 1)^(1/2) = 1/4,
    V = 4, ||q|| = 8, eps = C * 2 * 4^-4 / 8 = C / 1024."""
    import dataclasses

    import workloads
    from tests.gpu_util import EpsTracker, eps_formula
    f3 = dataclasses.replace(workloads.random_positive_tt((8, 8, 8), 2, seed=0), lo=(0.0,) * 3, hi=(2.0,) * 3)
    u3 = np.ones((5, 8, 8, 8))
    assert abs(eps_formula(f3, u3, 3.0) - 3.0 / 1024) < 1e-17
    f2 = dataclasses.replace(workloads.random_positive_tt((16, 4), 2, seed=0), lo=(0.0, 0.0), hi=(1.0, 4.0))
    u2 = np.ones((4, 16, 4))
    u2[3] *= 0.5  # the largest component norm counts
    assert abs(eps_formula(f2, u2, 5.0) - 5.0 / 1024) < 1e-17
    tr = EpsTracker(f2, u2, eps0=1e-6)
    assert abs(tr(u2) - 1e-6) < 1e-21 and abs(tr(2.0 * u2) - 0.5e-6) < 1e-21


# --- the tilted Sod workload: its exact solution and its initial TT ---------------------
def test_workload_exact_sod_matches_the_oracle_riemann_solver():
    """The benchmark's L1 reference (workloads.sod_exact_rho, its own wave-curve solver) against
    the oracle's exact Riemann solver on the same similarity variable, through all five regions."""
    import workloads
    s = np.linspace(-0.6, 0.6, 4801)
    for t in (0.05, 0.2):
        a = workloads.sod_exact_rho(s, t)
        b = riemann.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), s / t)[0]
        assert np.max(np.abs(a - b)) < 1e-13


@pytest.mark.parametrize("seed", [0, 2, 4])
def test_tilted_sod_initial_tt_is_exact(seed):
    """The initial TT of the tilted Sod workload equals the sampled step field cell by cell, and
    its ranks are the number of distinct step rows, about N tan(theta) + 1."""
    import workloads
    n = 64
    f = workloads.config5_tilted_sod_3d(n, seed=seed)
    rho = tt_ref.tt_full(f.cores[0])
    ene = tt_ref.tt_full(f.cores[4])
    ex = f.exact_rho(1e-12)  # t -> 0: the initial step
    assert np.array_equal(np.unique(rho.round(12)), np.array([0.125, 1.0]))
    assert np.max(np.abs(rho - ex)) < 1e-12
    assert np.max(np.abs(ene - np.where(rho > 0.5, 2.5, 0.25))) < 1e-12
    for c in (1, 2, 3):
        assert np.max(np.abs(tt_ref.tt_full(f.cores[c]))) == 0.0
    theta = math.radians(float(f.note.split("theta ")[1].split(" deg")[0]))
    r = max(g.shape[2] for g in f.cores[0][:-1])
    assert r <= n * math.tan(theta) + 2


# --- the cross's pivot rule (complete pivoting, Sec. 3.3) -------------------------------
@pytest.mark.parametrize("shape,rank", [((12, 9), 3), ((40, 25), 7), ((30, 30), 30)])
def test_full_pivot_lu_recovers_low_rank_and_bounds_l(shape, rank):
    """The oracle's pivot rule on exactly low-rank matrices: it stops at the exact rank, the
    skeleton A(:, J) A(I, J)^{-1} A(I, :) reproduces A, every entry of L is at most 1 in
    magnitude (complete pivoting), and the first pivot is the largest entry of A."""
    rng = np.random.default_rng(rank)
    A = rng.normal(size=(shape[0], rank)) @ rng.normal(size=(rank, shape[1]))
    r, rows, cols, L, s2 = tt_ref.full_pivot_lu(A, 1e-26, min(shape))
    assert r == rank
    skel = A[:, cols] @ np.linalg.solve(A[np.ix_(rows, cols)], A[rows, :])
    assert np.max(np.abs(skel - A)) <= 1e-10 * np.max(np.abs(A))
    assert np.max(np.abs(L)) <= 1.0 + 1e-12
    assert divmod(int(np.argmax(np.abs(A))), shape[1]) == (rows[0], cols[0])
    # L L(I, :)^{-1} is the interpolative basis of the cross: A = L L(I, :)^{-1} A(I, :), and
    # L(I, :) is unit lower triangular in pivot order
    LI = L[rows, :]
    assert np.allclose(np.diag(LI), 1.0) and np.max(np.abs(np.triu(LI, 1))) <= 1e-12
    assert np.max(np.abs(L @ np.linalg.solve(LI, A[rows, :]) - A)) <= 1e-10 * np.max(np.abs(A))


# --- Sec. 4.5.2-4.5.3: symmetry planes and inflow sides --------------------------------
def _mirror_full(U, axis, momentum_sign):
    """The half state U on the high half of a box, continued across its low face along `axis`:
    cell -1-l of the full box holds cell l, the momentum component normal to the face negated."""
    M = np.flip(U, axis=1 + axis).copy()
    if momentum_sign:
        M[1 + axis] = -M[1 + axis]
    return np.concatenate([M, U], axis=1 + axis)


@pytest.mark.parametrize("ndim,axis", [(1, 0), (2, 0), (2, 1), (3, 2)])
def test_symmetry_plane_is_the_mirrored_full_box(ndim, axis):
    """A symmetry plane at x_axis = 0 on [0, 1] equals the upper half of the problem on [-1, 1]
    whose lower half is the mirror image (the momentum normal to the plane odd, everything else
    even): one right-hand side bit for bit (the faces of the upper half see the same cell values),
    and SSP-RK3 steps to rounding (the mirror is a symmetry of the Euler equations)."""
    rng = np.random.default_rng(40 + 3 * ndim + axis)
    n = tuple(14 if d == axis else 9 - d for d in range(ndim))
    U = _random_state(n, rng)
    bc_half = tuple((oracle.BC_SYMMETRY, oracle.BC_TRANSMISSIVE) if d == axis else oracle.BC_PERIODIC
                    for d in range(ndim))
    bc_full = tuple(oracle.BC_TRANSMISSIVE if d == axis else oracle.BC_PERIODIC for d in range(ndim))
    half = oracle.Problem(n, (0.0,) * ndim, (1.0,) * ndim, bc_half)
    nf = tuple(2 * m if d == axis else m for d, m in enumerate(n))
    full = oracle.Problem(nf, tuple(-1.0 if d == axis else 0.0 for d in range(ndim)), (1.0,) * ndim, bc_full)
    V = _mirror_full(U, axis, True)
    upper = (slice(None),) + tuple(slice(n[axis], None) if d == axis else slice(None) for d in range(ndim))
    a = full.alpha(V)
    assert half.alpha(U) == a
    assert np.array_equal(half.rhs(U, a), full.rhs(V, a)[upper])
    assert np.array_equal(half.rhs(U, a, naive=True), full.rhs(V, a, naive=True)[upper])
    for _ in range(3):
        dt = 0.4 * min(half.h) / a
        al = half.ssprk3(U, dt)
        full.ssprk3(V, dt, alphas=al)
        a = half.alpha(U)
    assert np.max(np.abs(U - V[upper])) <= 1e-13 * np.max(np.abs(U))


def test_symmetry_plane_high_side_and_scalar_mirror():
    """The same at the high face of [-1, 0], and for a scalar law (mirrored without a sign)."""
    rng = np.random.default_rng(44)
    U = _random_state((16,), rng)
    half = oracle.Problem((16,), (-1.0,), (0.0,), ((oracle.BC_TRANSMISSIVE, oracle.BC_SYMMETRY),))
    full = oracle.Problem((32,), (-1.0,), (1.0,), (oracle.BC_TRANSMISSIVE,))
    V = np.flip(_mirror_full(np.flip(U, axis=1).copy(), 0, True), axis=1).copy()
    a = full.alpha(V)
    assert np.array_equal(half.rhs(U, a), full.rhs(V, a)[:, :16])
    u = U[:1].copy()
    shalf = oracle.Problem((16,), (0.0,), (1.0,), ((oracle.BC_SYMMETRY, oracle.BC_TRANSMISSIVE),),
                           model=oracle.BURGERS)
    sfull = oracle.Problem((32,), (-1.0,), (1.0,), (oracle.BC_TRANSMISSIVE,), model=oracle.BURGERS)
    v = _mirror_full(u, 0, False)
    assert np.array_equal(shalf.rhs(u, 1.7), sfull.rhs(v, 1.7)[:, 16:])


def test_inflow_state_from_primitives_hand_values():
    P = oracle.Problem((4, 4), (0, 0), (1, 1), ((oracle.BC_INFLOW, oracle.BC_TRANSMISSIVE), oracle.BC_PERIODIC),
                       gamma=1.4, inflow={(0, 0): (1.2, 0.5, -0.3, 2.0)})
    # rho, rho u, rho v, p / (gamma - 1) + rho |u|^2 / 2 = 5 + 0.6 * 0.34
    assert np.allclose(P.inflow_conserved(0, 0), [1.2, 0.6, -0.36, 5.204], rtol=0, atol=1e-15)
    S = oracle.Problem((4,), (0,), (1,), ((oracle.BC_TRANSMISSIVE, oracle.BC_INFLOW),), model=oracle.LINADV,
                       inflow={(0, 1): (0.25,)})
    assert S.inflow_conserved(0, 1).tolist() == [0.25]
    with pytest.raises(ValueError):
        oracle.Problem((4,), (0,), (1,), ((oracle.BC_PERIODIC, oracle.BC_INFLOW),), inflow={(0, 1): (1, 0, 1)})
    with pytest.raises(ValueError):
        oracle.Problem((4,), (0,), (1,), (oracle.BC_TRANSMISSIVE,), inflow={(0, 0): (1, 0, 1)})


@pytest.mark.parametrize("side", [0, 1])
def test_inflow_side_is_three_explicit_cells(side):
    """An inflow side holds the inflow state in its three ghost cells (the zeroed ghost slices
    plus the rank-1 boundary TT of Sec. 4.5.2): the right-hand side of the interior equals, bit for
    bit, the one of a box extended by three cells that hold that state (their own ghosts never
    reach an interior face)."""
    rng = np.random.default_rng(50 + side)
    n = (13, 7)
    prim = (0.8, 1.3, 0.2, 0.6)
    U = _random_state(n, rng)
    bcs = (oracle.BC_INFLOW, oracle.BC_TRANSMISSIVE) if side == 0 else (oracle.BC_TRANSMISSIVE, oracle.BC_INFLOW)
    P = oracle.Problem(n, (0, 0), (1.3, 1.0), (bcs, oracle.BC_PERIODIC), inflow={(0, side): prim})
    h = P.h[0]
    lo, hi = (0.0 - 3 * h, 0.0) if side == 0 else (0.0, 1.3 + 3 * h)
    ext = oracle.Problem((16, 7), (lo, 0), (hi if side else 1.3, 1.0), (oracle.BC_TRANSMISSIVE, oracle.BC_PERIODIC))
    q = P.inflow_conserved(0, side)
    block = np.broadcast_to(q[:, None, None], (4, 3, 7))
    V = np.concatenate([block, U], axis=1) if side == 0 else np.concatenate([U, block], axis=1)
    V = np.ascontiguousarray(V)
    a = P.alpha(U)
    inner = slice(3, None) if side == 0 else slice(0, 13)
    assert np.array_equal(P.rhs(U, a), ext.rhs(V, a)[:, inner])
    assert np.array_equal(P.rhs(U, a, naive=True), ext.rhs(V, a, naive=True)[:, inner])


def test_uniform_flow_through_an_inflow_side_stays_exact():
    prim = (1.1, 0.7, -0.2, 0.9)
    P = oracle.Problem((10, 6), (0, 0), (1, 1), ((oracle.BC_INFLOW, oracle.BC_TRANSMISSIVE), oracle.BC_PERIODIC),
                       inflow={(0, 0): prim})
    q = P.inflow_conserved(0, 0)
    U = np.ascontiguousarray(np.broadcast_to(q[:, None, None], (4, 10, 6)))
    U0 = U.copy()
    for _ in range(3):
        P.ssprk3(U, 0.01)
    assert np.array_equal(U, U0)
