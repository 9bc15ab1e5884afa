"""Initial states of the synthetic flows, as tensor trains of the conserved variables.

Conventions: a state is one TT per conserved variable (rho, rho u, rho v[, rho w], rho E),
each a list of cores of shape (R_{k-1}, N_k, R_k) with R_0 = R_d = 1, on a cell-centred
grid x_i = lo + (i + 1/2) h, i = 0..N-1. Boundary codes: 0 periodic, 1 transmissive.
All randomness comes from numpy.random.default_rng(seed).

The ideal-gas energy rhoE = p/(gamma-1) + rho |u|^2 / 2 is used to turn primitive
initial data into conserved data; nothing else of the scheme appears here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PERIODIC, TRANSMISSIVE = 0, 1


@dataclasses.dataclass
class Flow:
    name: str
    ndim: int
    n: tuple
    lo: tuple
    hi: tuple
    bc: tuple
    gamma: float
    cores: list  # [ncomp][ndim] numpy arrays
    t_end: float = 0.0
    cfl: float = 0.5
    eps_mode: int = 0  # 0 fixed eps, 1 dynamic
    eps0: float = 1e-10
    note: str = ""
    # density of the exact solution on the grid at time t, where one is known in closed form
    exact_rho: object = None
    # conservation law: 0 Euler (ndim + 2 components), 1 linear advection, 2 Burgers (one)
    law: int = 0
    # C_eps of the dynamic eps_TT when it is given rather than fixed by eps(0) = eps0 (0: not given)
    c_eps: float = 0.0
    # fixed time step, when the workload prescribes one rather than a CFL number (0: none)
    fixed_dt: float = 0.0
    # the whole exact solution on the grid at time t, [ncomp][cells], where known (scalar laws)
    exact: object = None
    # primitive state of each inflow side: {(dimension, side): (rho, u_1..u_ndim, p) or (u,)}
    inflow: object = None

    @property
    def ncomp(self):
        return self.ndim + 2 if self.law == 0 else 1

    @property
    def h(self):
        return tuple((b - a) / m for a, b, m in zip(self.lo, self.hi, self.n))

    def centers(self, d):
        return self.lo[d] + (np.arange(self.n[d]) + 0.5) * self.h[d]

    def ranks(self):
        return [[1] + [int(g.shape[2]) for g in comp[:-1]] + [1] for comp in self.cores]


def _concat_terms(terms):
    """Cores of a sum of TTs (each a list of cores): first cores side by side, middle cores
    block-diagonal, last cores stacked. Used to build separable initial data."""
    d = len(terms[0])
    if len(terms) == 1:
        return [np.array(g, dtype=np.float64) for g in terms[0]]
    out = []
    for k in range(d):
        gs = [t[k] for t in terms]
        n = gs[0].shape[1]
        if d == 1:
            out.append(sum(gs))
            continue
        if k == 0:
            out.append(np.concatenate(gs, axis=2))
        elif k == d - 1:
            out.append(np.concatenate(gs, axis=0))
        else:
            r0 = sum(g.shape[0] for g in gs)
            r1 = sum(g.shape[2] for g in gs)
            c = np.zeros((r0, n, r1))
            a = b = 0
            for g in gs:
                c[a:a + g.shape[0], :, b:b + g.shape[2]] = g
                a += g.shape[0]
                b += g.shape[2]
            out.append(c)
    return out


def _const_term(xs, value):
    d = len(xs)
    t = [np.ones((1, len(x), 1)) for x in xs]
    t[0] = t[0] * value
    return t


def _sin_plane_term(xs, ks, phase, amp):
    """TT of amp * sin(sum_d ks[d] * xs[d] + phase); rank 2 on every bond."""
    d = len(xs)
    angles = [ks[dd] * xs[dd] + (phase if dd == 0 else 0.0) for dd in range(d)]
    if d == 1:
        return [(amp * np.sin(angles[0]))[None, :, None]]
    cores = []
    a = angles[0]
    cores.append(amp * np.stack([np.sin(a), np.cos(a)], axis=-1)[None])  # (1, N, 2)
    for dd in range(1, d - 1):
        b = angles[dd]
        m = np.empty((2, len(b), 2))
        m[0, :, 0], m[0, :, 1] = np.cos(b), -np.sin(b)
        m[1, :, 0], m[1, :, 1] = np.sin(b), np.cos(b)
        cores.append(m)
    c = angles[-1]
    cores.append(np.stack([np.cos(c), np.sin(c)], axis=0)[:, :, None])  # (2, N, 1)
    return cores


def _scale(term, s):
    t = [g.copy() for g in term]
    t[0] = t[0] * s
    return t


def config1_smooth_wave_2d(n: int = 64) -> Flow:
    """2D smooth density wave rho = 1 + 0.2 sin(pi (x+y)), u = v = 1, p = 1 on [0,2]^2,
    periodic. Exact TT rank 3 for every conserved variable."""
    lo, hi = (0.0, 0.0), (2.0, 2.0)
    h = 2.0 / n
    xs = [lo[d] + (np.arange(n) + 0.5) * h for d in range(2)]
    g = 1.4
    wave = _sin_plane_term(xs, (math.pi, math.pi), 0.0, 0.2)
    rho = _concat_terms([_const_term(xs, 1.0), wave])
    mom = rho
    ene = _concat_terms([_const_term(xs, 1.0 / (g - 1.0) + 1.0), wave])  # p/(g-1) + rho (u^2+v^2)/2
    return Flow("smooth_wave_2d", 2, (n, n), lo, hi, (PERIODIC, PERIODIC), g,
                [rho, [c.copy() for c in mom], [c.copy() for c in mom], ene], t_end=0.1, cfl=0.5,
                eps_mode=0, eps0=1e-10, note="rho=1+0.2sin(pi(x+y)), u=v=1, p=1")


def _quadrant_states(rng, gamma):
    while True:
        rho = rng.uniform(0.1, 1.5, size=(2, 2))
        p = rng.uniform(0.03, 1.5, size=(2, 2))
        u = rng.uniform(-1.2, 1.2, size=(2, 2))
        v = rng.uniform(-1.2, 1.2, size=(2, 2))
        a = np.sqrt(gamma * p / rho)
        ok = True
        # x-neighbours (ix=0 left, ix=1 right) and y-neighbours (iy=0 bottom, iy=1 top)
        for iy in range(2):
            if u[1, iy] - u[0, iy] >= 0.5 * 2.0 * (a[0, iy] + a[1, iy]) / (gamma - 1.0):
                ok = False
        for ix in range(2):
            if v[ix, 1] - v[ix, 0] >= 0.5 * 2.0 * (a[ix, 0] + a[ix, 1]) / (gamma - 1.0):
                ok = False
        if ok:
            return rho, u, v, p


def config2_quadrants_2d(n: int = 512, seed: int = 0) -> Flow:
    """2D four-quadrant Riemann problem on [0,1]^2 split at (0.5, 0.5), transmissive.
    Each quadrant draws rho ~ U[0.1,1.5], p ~ U[0.03,1.5], u, v ~ U[-1.2,1.2]; a draw whose
    normal-velocity jump between neighbours reaches half the vacuum-formation threshold
    2(a_L+a_R)/(gamma-1) is redrawn. Initial TT rank 2."""
    g = 1.4
    rng = np.random.default_rng(seed)
    rho, u, v, p = _quadrant_states(rng, g)
    cons = [rho, rho * u, rho * v, p / (g - 1.0) + 0.5 * rho * (u * u + v * v)]
    half = n // 2
    ix = (np.arange(n) >= half).astype(int)
    cores = []
    for q in cons:
        g1 = np.zeros((1, n, 2))
        g1[0, :, 0] = (ix == 0)
        g1[0, :, 1] = (ix == 1)
        g2 = np.zeros((2, n, 1))
        for a in range(2):
            g2[a, :, 0] = q[a, ix]
        cores.append([g1, g2])
    return Flow("quadrants_2d", 2, (n, n), (0.0, 0.0), (1.0, 1.0), (TRANSMISSIVE, TRANSMISSIVE), g, cores,
                t_end=0.2, cfl=0.5, eps_mode=1, eps0=1e-8, note=f"seed {seed}")


def config3_wave_3d(n: int = 256, seed: int = 0, modes: int = 8, amp: float = 1e-3) -> Flow:
    """3D smooth wave rho = 1 + 0.2 sin(pi(x+y+z)) + sum_m amp sin(pi k_m.x + phi_m) on [0,2]^3,
    periodic, u = v = w = 1, p = 1; k_m in {-3..3}^3 \\ {0}. TT rank <= 3 + 2 * modes."""
    g = 1.4
    rng = np.random.default_rng(seed)
    h = 2.0 / n
    xs = [(np.arange(n) + 0.5) * h for _ in range(3)]
    terms = [_const_term(xs, 1.0), _sin_plane_term(xs, (math.pi,) * 3, 0.0, 0.2)]
    waves = [((math.pi,) * 3, 0.0, 0.2)]
    for _ in range(modes):
        while True:
            k = rng.integers(-3, 4, size=3)
            if np.any(k != 0):
                break
        phi = rng.uniform(0.0, 2.0 * math.pi)
        kv = tuple(math.pi * float(kk) for kk in k)
        terms.append(_sin_plane_term(xs, kv, phi, amp))
        waves.append((kv, phi, amp))

    def exact_rho(t):
        # u = v = w = 1 and p = 1 everywhere: every conserved variable is carried along (1, 1, 1)
        r = np.ones((n, n, n))
        for kv, phi, a in waves:
            ph = [kv[d] * (xs[d] - t) for d in range(3)]
            r += a * np.sin(ph[0][:, None, None] + ph[1][None, :, None] + ph[2][None, None, :] + phi)
        return r
    rho = _concat_terms(terms)
    e_terms = [_const_term(xs, 1.0 / (g - 1.0) + 1.5)] + [_scale(t, 1.5) for t in terms[1:]]
    ene = _concat_terms(e_terms)
    return Flow("wave_3d", 3, (n, n, n), (0.0,) * 3, (2.0,) * 3, (PERIODIC,) * 3, g,
                [rho, [c.copy() for c in rho], [c.copy() for c in rho], [c.copy() for c in rho], ene],
                t_end=0.1, cfl=0.5, eps_mode=0, eps0=1e-6, note=f"seed {seed}, {modes} modes",
                exact_rho=exact_rho)


def tt_svd_input(x: np.ndarray, eps: float, rank_cap: int | None = None):
    """TT-SVD used to turn a sampled initial field into a TT (input preparation)."""
    d = x.ndim
    nrm = float(np.linalg.norm(x))
    delta = eps * nrm / math.sqrt(max(d - 1, 1))
    cores, r, c = [], 1, x.reshape(1, -1)
    for k in range(d - 1):
        c = c.reshape(r * x.shape[k], -1)
        u, s, vt = np.linalg.svd(c, full_matrices=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]
        rk = max(int(np.sum(tail > delta)), 1)
        if rank_cap is not None:
            rk = min(rk, rank_cap)
        cores.append(u[:, :rk].reshape(r, x.shape[k], rk))
        c = s[:rk, None] * vt[:rk]
        r = rk
    cores.append(c.reshape(r, x.shape[-1], 1))
    return cores


def config4_blast_3d(seed: int = 0, n=None, eps: float = 1e-4, rank_cap: int = 60, width: float = 0.01) -> Flow:
    """Spherical blast on [0,1]^3 with h_d = 1/N_d, transmissive: rho = 1, u = 0, p = 1 outside,
    p_in ~ U[5,20] inside a sphere of centre ~ U[0.3,0.7]^3 and radius ~ U[0.1,0.3], sampled at
    cell centres. The jump is spread over a tanh profile of the given width (1 to 2.5 cells):
    a sharp ball has one distinct disk per cell slice (ranks 67-128 on these grids), and cutting
    those ranks produces Gibbs oscillations with negative pressure. The TT is a TT-SVD of the
    sampled field at eps with a rank cap (initial ranks 15-26)."""
    g = 1.4
    rng = np.random.default_rng(seed)
    sizes = (64, 96, 128, 192, 256)
    if n is None:
        n = tuple(int(sizes[i]) for i in rng.integers(0, len(sizes), size=3))
    p_in = rng.uniform(5.0, 20.0)
    c0 = rng.uniform(0.3, 0.7, size=3)
    rad = rng.uniform(0.1, 0.3)
    xs = [(np.arange(m) + 0.5) / m for m in n]
    r2 = ((xs[0][:, None, None] - c0[0]) ** 2 + (xs[1][None, :, None] - c0[1]) ** 2
          + (xs[2][None, None, :] - c0[2]) ** 2)
    if width > 0.0:
        p = 1.0 + (p_in - 1.0) * 0.5 * (1.0 - np.tanh((np.sqrt(r2) - rad) / width))
    else:
        p = np.where(r2 < rad * rad, p_in, 1.0)
    ones = [np.ones((1, m, 1)) for m in n]
    zeros = [np.zeros((1, m, 1)) for m in n]
    ene = tt_svd_input(p / (g - 1.0), eps, rank_cap)
    cores = [ones, [z.copy() for z in zeros], [z.copy() for z in zeros], [z.copy() for z in zeros], ene]
    return Flow("blast_3d", 3, tuple(n), (0.0,) * 3, (1.0,) * 3, (TRANSMISSIVE,) * 3, g, cores,
                t_end=0.0, cfl=0.5, eps_mode=1, eps0=1e-6,
                note=f"seed {seed}, p_in {p_in:.3f}, centre {c0.round(3).tolist()}, radius {rad:.3f}")


def sod_1d_like(ndim: int, n: int, axis: int = 0) -> Flow:
    """Sod shock tube (1,0,0,0,1) | (0.125,0,0,0,0.1) across x_axis = 0.5 on [0,1]^ndim,
    transmissive (Sec. 5.5). Every conserved variable has TT rank 1."""
    g = 1.4
    xs = [(np.arange(n) + 0.5) / n for _ in range(ndim)]
    left = xs[axis] < 0.5
    rho = np.where(left, 1.0, 0.125)
    ene = np.where(left, 1.0, 0.1) / (g - 1.0)

    def rank1(vals_axis):
        cores = [np.ones((1, n, 1)) for _ in range(ndim)]
        cores[axis] = np.array(vals_axis, dtype=np.float64)[None, :, None]
        return cores

    cores = [rank1(rho)] + [rank1(np.zeros(n)) for _ in range(ndim)] + [rank1(ene)]
    return Flow("sod_%dd" % ndim, ndim, (n,) * ndim, (0.0,) * ndim, (1.0,) * ndim, (TRANSMISSIVE,) * ndim, g,
                cores, t_end=0.2, cfl=0.5, eps_mode=1, eps0=1e-6)


SOD_LEFT = (1.0, 0.0, 1.0)     # (rho, u, p) on the side n.(x - 1/2) < 0
SOD_RIGHT = (0.125, 0.0, 0.1)  # (rho, u, p) on the other side


def sod_exact_rho(s, t, gamma=1.4, left=SOD_LEFT, right=SOD_RIGHT):
    """Density of the exact solution of a 1D Riemann problem at signed distance s from the
    initial discontinuity and time t > 0 (left state at s < 0). Written from the wave curves of
    the gamma-law gas: the star pressure solves phi_L(p) + phi_R(p) + u_R - u_L = 0, where
    phi_K(p) is the velocity jump across a shock (p > p_K, Rankine-Hugoniot) or a rarefaction
    (p <= p_K, isentrope and Riemann invariant) into state K; Newton iteration from the
    arithmetic mean of the two pressures. Used for the L1 error of the tilted Sod workload."""
    g = gamma
    s = np.asarray(s, dtype=np.float64)

    def phi(p, rho_k, p_k):
        c_k = math.sqrt(g * p_k / rho_k)
        if p > p_k:
            a = 2.0 / ((g + 1.0) * rho_k)
            b = p_k * (g - 1.0) / (g + 1.0)
            q = math.sqrt(a / (b + p))
            return (p - p_k) * q, q * (1.0 - (p - p_k) / (2.0 * (b + p)))
        ratio = p / p_k
        z = (g - 1.0) / (2.0 * g)
        return 2.0 * c_k / (g - 1.0) * (ratio ** z - 1.0), ratio ** (-(g + 1.0) / (2.0 * g)) / (rho_k * c_k)

    (rl, ul, pl), (rr, ur, pr) = left, right
    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dl = phi(p, rl, pl)
        fr, dr = phi(p, rr, pr)
        step = (fl + fr + ur - ul) / (dl + dr)
        p_new = max(p - step, 1e-14 * p)
        done = abs(p_new - p) < 1e-15 * p
        p = p_new
        if done:
            break
    fl, _ = phi(p, rl, pl)
    fr, _ = phi(p, rr, pr)
    u_star = 0.5 * (ul + ur + fr - fl)
    xi = s / t
    out = np.empty_like(xi)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    # left of the contact
    lmask = xi <= u_star
    if p > pl:  # left-facing shock
        rho_sl = rl * (p / pl + gm) / (gm * p / pl + 1.0)
        sh = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * p / pl + (g - 1.0) / (2.0 * g))
        out[lmask] = np.where(xi[lmask] < sh, rl, rho_sl)
    else:  # left rarefaction fan between its head and tail speeds
        rho_sl = rl * (p / pl) ** (1.0 / g)
        c_sl = cl * (p / pl) ** ((g - 1.0) / (2.0 * g))
        head, tail = ul - cl, u_star - c_sl
        x = xi[lmask]
        fan = rl * (2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cl) * (ul - x)) ** (2.0 / (g - 1.0))
        out[lmask] = np.where(x < head, rl, np.where(x > tail, rho_sl, fan))
    rmask = ~lmask
    if p > pr:  # right-facing shock
        rho_sr = rr * (p / pr + gm) / (gm * p / pr + 1.0)
        sh = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * p / pr + (g - 1.0) / (2.0 * g))
        out[rmask] = np.where(xi[rmask] > sh, rr, rho_sr)
    else:  # right rarefaction fan
        rho_sr = rr * (p / pr) ** (1.0 / g)
        c_sr = cr * (p / pr) ** ((g - 1.0) / (2.0 * g))
        head, tail = ur + cr, u_star + c_sr
        x = xi[rmask]
        fan = rr * (2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cr) * (ur - x)) ** (2.0 / (g - 1.0))
        out[rmask] = np.where(x > head, rr, np.where(x < tail, rho_sr, fan))
    return out


def _exact_svd_tt2(field2d, rel=1e-13):
    """Exact low-rank factors of a sampled 2D field: U S V^T with the singular values above
    rel * sigma_max kept (the field of a tilted step has exact rank = its number of distinct
    rows, the rest is rounding)."""
    u, s, vt = np.linalg.svd(field2d, full_matrices=False)
    r = max(1, int(np.sum(s > rel * s[0])))
    return u[:, :r], s[:r], vt[:r]


def config5_tilted_sod_3d(n: int = 512, seed: int = 0) -> Flow:
    """Sod states (1, 0, 0, 0, 1) | (0.125, 0, 0, 0, 0.1) across the plane n.(x - 1/2) = 0 on
    [0,1]^3, transmissive. n is e_x turned by theta ~ U[0, 5] degrees about e_z or e_y (seeded,
    either sign), so the data depend on two coordinates and the TT is exact: for a turn about e_z
    the state is f(x, y) (cores U | S V^T | ones), about e_y it is f(x, z) (cores U | identity |
    S V^T), with ranks = the number of distinct step rows, about N tan(theta) + 1.
    exact_rho(t) gives the exact density (the 1D Riemann solution along n)."""
    g = 1.4
    rng = np.random.default_rng(seed)
    theta = math.radians(rng.uniform(0.0, 5.0))
    about_z = bool(rng.integers(0, 2) == 0)
    sign = 1.0 if rng.integers(0, 2) == 0 else -1.0
    nvec = np.array([math.cos(theta), 0.0, 0.0])
    nvec[1 if about_z else 2] = sign * math.sin(theta)
    x = (np.arange(n) + 0.5) / n - 0.5
    other = 1 if about_z else 2
    s2 = nvec[0] * x[:, None] + nvec[other] * x[None, :]  # signed distance on the (x, other) plane
    left = s2 < 0.0
    rho2 = np.where(left, SOD_LEFT[0], SOD_RIGHT[0])
    ene2 = np.where(left, SOD_LEFT[2], SOD_RIGHT[2]) / (g - 1.0)

    def tt_of(field2d):
        u, s, vt = _exact_svd_tt2(field2d)
        r = u.shape[1]
        g0 = u[None, :, :]
        right = (s[:, None] * vt)
        if about_z:
            return [g0, right[:, :, None], np.ones((1, n, 1))]
        mid = np.zeros((r, n, r))
        mid[np.arange(r), :, np.arange(r)] = 1.0
        return [g0, mid, right[:, :, None]]

    zeros = [np.zeros((1, n, 1)) for _ in range(3)]
    cores = [tt_of(rho2)] + [[z.copy() for z in zeros] for _ in range(3)] + [tt_of(ene2)]
    xs = (np.arange(n) + 0.5) / n - 0.5

    def exact_rho(t, box=None):
        """Exact density on the grid (or on the cells whose centres lie in box = (lo, hi))."""
        idx = np.arange(n) if box is None else np.nonzero((xs + 0.5 >= box[0]) & (xs + 0.5 <= box[1]))[0]
        xx = xs[idx]
        s3 = (nvec[0] * xx[:, None, None] + nvec[1] * xx[None, :, None] + nvec[2] * xx[None, None, :])
        return sod_exact_rho(s3, t, g)

    axis = "z" if about_z else "y"
    return Flow("tilted_sod_3d", 3, (n,) * 3, (0.0,) * 3, (1.0,) * 3, (TRANSMISSIVE,) * 3, g, cores,
                t_end=0.1, cfl=0.5, eps_mode=1, eps0=1e-6,
                note=f"seed {seed}, theta {math.degrees(theta):.3f} deg about {'+' if sign > 0 else '-'}e_{axis}",
                exact_rho=exact_rho)


def scalar_linadv_3d(n: int = 40) -> Flow:
    """3D linear advection u_t + u_x + u_y + u_z = 0 of u0 = sin(2 pi (x+y+z)) on the periodic
    unit cube (Sec. 5.1): one component, TT rank 2, dt = h^{5/3}, T = 0.1, dynamic eps_TT with
    C_eps = 500. Exact solution: u0 translated by t (1, 1, 1)."""
    lo, hi = (0.0,) * 3, (1.0,) * 3
    h = 1.0 / n
    xs = [(np.arange(n) + 0.5) * h for _ in range(3)]
    k = 2.0 * math.pi
    u = _sin_plane_term(xs, (k, k, k), 0.0, 1.0)

    def exact(t):
        s = xs[0][:, None, None] + xs[1][None, :, None] + xs[2][None, None, :]
        return np.sin(k * (s - 3.0 * t))[None]

    return Flow("linadv_3d", 3, (n, n, n), lo, hi, (PERIODIC,) * 3, 1.4, [u], t_end=0.1, cfl=0.0,
                eps_mode=1, eps0=0.0, note="u0=sin(2pi(x+y+z)), C_eps=500, dt=h^(5/3)", law=1,
                c_eps=500.0, fixed_dt=h ** (5.0 / 3.0), exact=exact)


def burgers_exact(xi, t):
    """Solution of u_t + sum_d (u^2/2)_{x_d} = 0 with u0 = 0.5 + 0.5 sin(2 pi xi), xi = x+y+z,
    before the characteristics cross (t < 1/(3 pi)): u = u0(xi - 3 u t), solved by Newton."""
    u = 0.5 + 0.5 * np.sin(2.0 * math.pi * xi)
    for _ in range(100):
        a = 2.0 * math.pi * (xi - 3.0 * u * t)
        g = u - (0.5 + 0.5 * np.sin(a))
        u = u - g / (1.0 + 3.0 * math.pi * t * np.cos(a))
    return u


def scalar_burgers_3d(n: int = 40) -> Flow:
    """3D Burgers u_t + u u_x + u u_y + u u_z = 0 of u0 = 0.5 + 0.5 sin(2 pi (x+y+z)) on the
    periodic unit cube (Sec. 5.2): one component, initial TT rank 3, dt = h^{5/3},
    T = 1/(12 pi), dynamic eps_TT with C_eps = 10."""
    lo, hi = (0.0,) * 3, (1.0,) * 3
    h = 1.0 / n
    xs = [(np.arange(n) + 0.5) * h for _ in range(3)]
    k = 2.0 * math.pi
    u = _concat_terms([_const_term(xs, 0.5), _sin_plane_term(xs, (k, k, k), 0.0, 0.5)])

    def exact(t):
        s = xs[0][:, None, None] + xs[1][None, :, None] + xs[2][None, None, :]
        return burgers_exact(s, t)[None]

    return Flow("burgers_3d", 3, (n, n, n), lo, hi, (PERIODIC,) * 3, 1.4, [u], t_end=1.0 / (12.0 * math.pi),
                cfl=0.0, eps_mode=1, eps0=0.0, note="u0=0.5+0.5sin(2pi(x+y+z)), C_eps=10, dt=h^(5/3)", law=2,
                c_eps=10.0, fixed_dt=h ** (5.0 / 3.0), exact=exact)


def random_positive_tt(n, rank: int, seed: int, amp: float = 0.2, bc=None, rough: bool = False) -> Flow:
    """A random positive state with TT rank <= rank per variable:
    rho = 1 + amp T_0, rho u_d = amp T_d, rho E = 3 + amp T_E, where every T is a random TT
    scaled so that |T| <= 1 everywhere. Its profiles are low-frequency periodic ones (three
    frequencies, so the ranks stay <= 5 whatever `rank` asks for), or with rough=True
    independent normal values in every cell, whose TT ranks are `rank` (generically)."""
    n = tuple(int(m) for m in n)
    d = len(n)
    rng = np.random.default_rng(seed)
    xs = [(np.arange(m) + 0.5) / m for m in n]

    def rand_tt():
        ranks = [1] + [rank] * (d - 1) + [1]
        cores = []
        for k in range(d):
            prof = np.zeros((ranks[k], n[k], ranks[k + 1]))
            if rough:
                prof += rng.normal(size=prof.shape)
            else:
                for f in range(3):
                    c = rng.normal(size=(ranks[k], 1, ranks[k + 1])) / (1.0 + f)
                    ph = rng.uniform(0, 2 * math.pi, size=(ranks[k], 1, ranks[k + 1]))
                    prof += c * np.cos(2 * math.pi * f * xs[k][None, :, None] + ph)
            # bound: |T| <= prod_k max_i ||core_k(i)||_inf-row-sum  -> normalise every core
            row = np.abs(prof).sum(axis=2).max()
            cores.append(prof / row)
        return cores

    def shift_scale(cores, base, s):
        t = [g.copy() for g in cores]
        t[0] = t[0] * s
        return _concat_terms([_const_term(xs, base), t]) if base != 0.0 else t

    comps = [shift_scale(rand_tt(), 1.0, amp)]
    for _ in range(d):
        comps.append(shift_scale(rand_tt(), 0.0, amp))
    comps.append(shift_scale(rand_tt(), 3.0, amp))
    if bc is None:
        bc = (PERIODIC,) * d
    return Flow("random_tt_%dd" % d, d, n, (0.0,) * d, (1.0,) * d, tuple(bc), 1.4, comps, t_end=0.0,
                eps_mode=0, eps0=1e-12, note=f"seed {seed}, rank {rank}" + (", rough" if rough else ""))
