"""Exact solution of the 1D Riemann problem for the gamma-law Euler equations.

TEST INFRASTRUCTURE ONLY (part of the oracle). It provides the exact solution that the
Sod shock tube of Sec. 5.5 is compared with. It is written from the standard
Rankine-Hugoniot (shock) and isentrope (rarefaction) relations: the star pressure p*
solves f_L(p*) + f_R(p*) + (u_R - u_L) = 0, with

  f_K(p) = (p - p_K) sqrt(A_K / (p + B_K)),             p > p_K   (shock),
  f_K(p) = 2 a_K/(gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1),  p <= p_K (rarefaction),

A_K = 2 / ((gamma+1) rho_K), B_K = (gamma-1)/(gamma+1) p_K, a_K the sound speed; then the
self-similar solution is sampled at xi = (x - x0)/t.
"""
from __future__ import annotations

import math

import numpy as np


def _f_and_df(p, rho, pk, gamma):
    a = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    e = (gamma - 1.0) / (2.0 * gamma)
    return 2.0 * a / (gamma - 1.0) * ((p / pk) ** e - 1.0), (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma)) / (rho * a)


def star_state(left, right, gamma=1.4, tol=1e-15, maxit=200):
    """Return (p*, u*) for primitive states left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated; no star state")
    # two-rarefaction guess, then Newton on the pressure function
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) / (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-12)
    for _ in range(maxit):
        fl, dfl = _f_and_df(p, rl, pl, gamma)
        fr, dfr = _f_and_df(p, rr, pr, gamma)
        g = fl + fr + (ur - ul)
        pn = max(p - g / (dfl + dfr), 1e-14)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, gamma)
    fr, _ = _f_and_df(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def pressure_function_residual(left, right, p, gamma=1.4):
    """|f_L(p) + f_R(p) + u_R - u_L| at the given pressure."""
    fl, _ = _f_and_df(p, left[0], left[2], gamma)
    fr, _ = _f_and_df(p, right[0], right[2], gamma)
    return abs(fl + fr + right[1] - left[1])


def sample(left, right, xi, gamma=1.4):
    """Primitive (rho, u, p) of the self-similar solution at speeds xi = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    g1, g2 = (gamma - 1.0) / (gamma + 1.0), 2.0 / (gamma + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                sl = ul - al * math.sqrt((gamma + 1) / (2 * gamma) * ps / pl + (gamma - 1) / (2 * gamma))
                if s <= sl:
                    rho[n], u[n], p[n] = rl, ul, pl
                else:
                    rho[n] = rl * (ps / pl + g1) / (g1 * ps / pl + 1.0)
                    u[n], p[n] = us, ps
            else:  # left rarefaction
                head = ul - al
                a_star = al * (ps / pl) ** ((gamma - 1) / (2 * gamma))
                tail = us - a_star
                if s <= head:
                    rho[n], u[n], p[n] = rl, ul, pl
                elif s >= tail:
                    rho[n] = rl * (ps / pl) ** (1.0 / gamma)
                    u[n], p[n] = us, ps
                else:
                    c = g2 + g1 / al * (ul - s)
                    rho[n] = rl * c ** (2.0 / (gamma - 1))
                    u[n] = g2 * (al + 0.5 * (gamma - 1) * ul + s)
                    p[n] = pl * c ** (2 * gamma / (gamma - 1))
        else:  # right of the contact
            if ps > pr:  # right shock
                sr = ur + ar * math.sqrt((gamma + 1) / (2 * gamma) * ps / pr + (gamma - 1) / (2 * gamma))
                if s >= sr:
                    rho[n], u[n], p[n] = rr, ur, pr
                else:
                    rho[n] = rr * (ps / pr + g1) / (g1 * ps / pr + 1.0)
                    u[n], p[n] = us, ps
            else:  # right rarefaction
                head = ur + ar
                a_star = ar * (ps / pr) ** ((gamma - 1) / (2 * gamma))
                tail = us + a_star
                if s >= head:
                    rho[n], u[n], p[n] = rr, ur, pr
                elif s <= tail:
                    rho[n] = rr * (ps / pr) ** (1.0 / gamma)
                    u[n], p[n] = us, ps
                else:
                    c = g2 - g1 / ar * (ur - s)
                    rho[n] = rr * c ** (2.0 / (gamma - 1))
                    u[n] = g2 * (-ar + 0.5 * (gamma - 1) * ur + s)
                    p[n] = pr * c ** (2 * gamma / (gamma - 1))
    return rho, u, p
