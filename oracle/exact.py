"""Exact solutions and error measures for the shock-tube validation (Section 3.1).

TEST INFRASTRUCTURE ONLY (see ``oracle.lbm``).

* Sod: the exact solution of the Euler Riemann problem (standard two-rarefaction
  / two-shock pressure function, solved by Newton iteration, then sampled in
  x/t), the reference the paper scores its inviscid tube against.
* Becker: the closed-form viscous shock for constant mu and Pr = 3/4, the
  exact integral of the shock-frame balances with constant total enthalpy.
  Written here independently of the input generators.
* Norms L1, L2, Linf and the shock thickness, measured on the density profile
  between two levels bracketing the jump (Table "thickness"; the levels are a
  reading, default 10 % and 90 %).
"""
from __future__ import annotations

import numpy as np


# ----------------------------------------------------------------- Sod / Riemann
def _pressure_function(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * np.sqrt(A / (p + B))
        df = np.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:       # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(left, right, g=1.4):
    """(p*, u*) of the Riemann problem; left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = np.sqrt(g * pl / rl)
    cr = np.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        fl, dfl = _pressure_function(p, rl, pl, cl, g)
        fr, dfr = _pressure_function(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p_new = max(1e-10, p - dp)
        if abs(p_new - p) < 1e-15 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _pressure_function(p, rl, pl, cl, g)
    fr, _ = _pressure_function(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(xi, left, right, g=1.4):
    """rho, u, p at similarity coordinates xi = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = np.sqrt(g * pl / rl)
    cr = np.sqrt(g * pr / rr)
    ps, us = riemann_star(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for j, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                rs = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                S = ul - cl * np.sqrt((g + 1.0) / (2 * g) * ps / pl + (g - 1.0) / (2 * g))
                r, v, pp = (rl, ul, pl) if s <= S else (rs, us, ps)
            else:        # left rarefaction
                rs = rl * (ps / pl) ** (1.0 / g)
                cs = cl * (ps / pl) ** ((g - 1.0) / (2 * g))
                head, tail = ul - cl, us - cs
                if s <= head:
                    r, v, pp = rl, ul, pl
                elif s >= tail:
                    r, v, pp = rs, us, ps
                else:
                    v = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + s)
                    c = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - s))
                    r = rl * (c / cl) ** (2.0 / (g - 1.0))
                    pp = pl * (c / cl) ** (2.0 * g / (g - 1.0))
        else:        # right of contact
            if ps > pr:  # right shock
                rs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                S = ur + cr * np.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g))
                r, v, pp = (rr, ur, pr) if s >= S else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1.0 / g)
                cs = cr * (ps / pr) ** ((g - 1.0) / (2 * g))
                head, tail = ur + cr, us + cs
                if s >= head:
                    r, v, pp = rr, ur, pr
                elif s <= tail:
                    r, v, pp = rs, us, ps
                else:
                    v = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + s)
                    c = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - s))
                    r = rr * (c / cr) ** (2.0 / (g - 1.0))
                    pp = pr * (c / cr) ** (2.0 * g / (g - 1.0))
        rho[j], u[j], p[j] = r, v, pp
    return rho, u, p


SOD_LEFT = (1.0, 0.0, 1.0)
SOD_RIGHT = (0.125, 0.0, 0.1)


def sod_exact(x, t, x0=0.5, g=1.4):
    return riemann_sample((np.asarray(x) - x0) / t, SOD_LEFT, SOD_RIGHT, g)


def sod_star_states(g=1.4):
    """p*, u*, rho*_L, rho*_R, right shock speed, and max |u| + c of the exact solution."""
    ps, us = riemann_star(SOD_LEFT, SOD_RIGHT, g)
    rl, _, pl = SOD_LEFT
    rr, _, pr = SOD_RIGHT
    gm = (g - 1.0) / (g + 1.0)
    rsl = rl * (ps / pl) ** (1.0 / g)
    rsr = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
    cr = np.sqrt(g * pr / rr)
    S = cr * np.sqrt((g + 1.0) / (2 * g) * ps / pr + (g - 1.0) / (2 * g))
    amax = max(abs(us) + np.sqrt(g * ps / rsr), abs(us) + np.sqrt(g * ps / rsl), np.sqrt(g * pl / rl))
    return dict(p_star=ps, u_star=us, rho_star_L=rsl, rho_star_R=rsr, shock_speed=S, a_max=amax)


# ----------------------------------------------------------------- Becker
def becker_exact(x, x_mid, *, gamma=1.4, M=2.0, rho1=1.0, c1=1.0, mu=2e-3, Pr=0.75):
    """rho, u, p of the Becker shock (constant mu, Pr = 3/4), centred at x_mid.

    Momentum balance with constant total enthalpy gives
    u' = (u - u1)(u - u2) / (l u) * u1, l = 8 gamma mu / (3 (gamma+1) rho1 u1);
    integrated: x - x0 = l/(1 - v2) [ln(1 - v) - v2 ln(v - v2)], v = u/u1.
    """
    g = gamma
    u1 = M * c1
    p1 = rho1 * c1 ** 2 / g
    v2 = (g - 1) / (g + 1) + 2 / ((g + 1) * M * M)
    ell = 8 * g * mu / (3 * (g + 1) * rho1 * u1)
    pos = lambda v: ell / (1 - v2) * (np.log(1 - v) - v2 * np.log(v - v2))
    vm = 0.5 * (1 + v2)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    from scipy.optimize import brentq
    a, b = v2 + 1e-15, 1.0 - 1e-15

    def solve(xx):
        g_ = lambda vv: pos(vv) - pos(vm) - (xx - x_mid)
        ga, gb = g_(a), g_(b)
        if ga <= 0.0:      # beyond the downstream tail: v = v2 to round-off
            return a
        if gb >= 0.0:      # beyond the upstream tail
            return b
        return brentq(g_, a, b, xtol=1e-17, rtol=1e-15)

    v = np.array([solve(xx) for xx in x])
    u = u1 * v
    rho = rho1 / v
    H = g / (g - 1) * p1 / rho1 + 0.5 * u1 ** 2
    p = rho * (g - 1) / g * (H - 0.5 * u * u)
    return rho, u, p


def becker_width(levels=(0.1, 0.9), **kw):
    """Exact shock thickness between two levels of the density jump."""
    L = 0.2
    x = np.linspace(0, L, 8001)
    rho, _, _ = becker_exact(x, L / 2, **kw)
    return thickness(x, rho, levels)


# ----------------------------------------------------------------- measures
def norms(num, ref, dx):
    e = np.abs(np.asarray(num) - np.asarray(ref))
    return dict(L1=float(np.sum(e) * dx), L2=float(np.sqrt(np.sum(e * e) * dx)), Linf=float(np.max(e)))


def thickness(x, rho, levels=(0.1, 0.9), lo=None, hi=None):
    """Distance between the crossings of two levels of a monotone density jump."""
    x = np.asarray(x)
    rho = np.asarray(rho)
    if lo is None:
        lo = float(np.min(rho))
    if hi is None:
        hi = float(np.max(rho))
    out = []
    for lev in levels:
        r = lo + lev * (hi - lo)
        s = np.sign(rho - r)
        idx = np.nonzero(np.diff(s) != 0)[0]
        if len(idx) == 0:
            return float("nan")
        j = idx[0]
        x0 = x[j] + (r - rho[j]) * (x[j + 1] - x[j]) / (rho[j + 1] - rho[j])
        out.append(x0)
    return float(abs(out[1] - out[0]))
