"""Exact solution of the Riemann problem for the 1D Euler equations of an ideal
gas (the classical two-rarefaction / two-shock pressure-function method, as in
Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4).

Independent of the oracle: used to pin the B = 0 limit of the full scheme on
shock tubes.
"""
import math

import numpy as np


def _f_and_df(p, rho, pk, ck, g):
    if p > pk:   # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        sq = math.sqrt(A / (p + B))
        f = (p - pk) * sq
        df = sq * (1.0 - 0.5 * (p - pk) / (B + p))
    else:        # rarefaction
        pr = p / pk
        f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, g):
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    du = ur - ul
    # two-rarefaction guess, then Newton on f_L + f_R + du = 0
    z = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * du) / (cl / pl ** z + cr / pr ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(200):
        fl, dfl = _f_and_df(p, rl, pl, cl, g)
        fr, dfr = _f_and_df(p, rr, pr, cr, g)
        pn = p - (fl + fr + du) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f_and_df(p, rl, pl, cl, g)
    fr, _ = _f_and_df(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, g, xi):
    """Primitive state (rho, u, p) at similarity coordinate xi = x / t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    if xi <= us:   # left of contact
        if ps > pl:
            sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
            if xi <= sl:
                return rl, ul, pl
            return rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
        csl = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
        if xi <= ul - cl:
            return rl, ul, pl
        if xi >= us - csl:
            return rl * (ps / pl) ** (1.0 / g), us, ps
        u = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + xi)
        c = 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * (ul - xi))
        return rl * (c / cl) ** (2.0 / (g - 1.0)), u, pl * (c / cl) ** (2.0 * g / (g - 1.0))
    if ps > pr:
        sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
        if xi >= sr:
            return rr, ur, pr
        return rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
    csr = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
    if xi >= ur + cr:
        return rr, ur, pr
    if xi <= us + csr:
        return rr * (ps / pr) ** (1.0 / g), us, ps
    u = 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + xi)
    c = 2.0 / (g + 1.0) * (cr - 0.5 * (g - 1.0) * (ur - xi))
    return rr * (c / cr) ** (2.0 / (g - 1.0)), u, pr * (c / cr) ** (2.0 * g / (g - 1.0))


def cell_averages(left, right, g, x0, t, xl, xr, sub=64):
    """Cell averages of (rho, u, p) over cells [xl, xr) at time t (midpoint
    quadrature with ``sub`` points per cell)."""
    out = np.zeros((3, len(xl)))
    for i, (a, b) in enumerate(zip(xl, xr)):
        xs = a + (np.arange(sub) + 0.5) * (b - a) / sub
        vals = np.array([sample(left, right, g, (x - x0) / t) for x in xs])
        out[:, i] = vals.mean(axis=0)
    return out
