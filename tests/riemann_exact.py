"""Exact solution of the 1D Euler Riemann problem (ideal gas), used only as a
physics sanity check of the oracle's shock-tube results.

Standard two-rarefaction / two-shock pressure function with Newton iteration
for the star pressure, then self-similar sampling at x/t.
"""
from __future__ import annotations

import math

import numpy as np


def _f(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    r = p / pk  # rarefaction
    return (2.0 * ck / (g - 1.0)) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0), \
        (1.0 / (rho * ck)) * r ** (-(g + 1.0) / (2.0 * g))


def star_state(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dl = _f(p, rl, pl, cl, g)
        fr, dr = _f(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dl + dr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, cl, g)
    fr, _ = _f(p, rr, pr, cr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, x, t, x0=0.5, g=1.4):
    """Primitive (rho, u, p) arrays of the exact solution at positions x."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us = star_state(left, right, g)
    out = np.zeros((3, len(x)))
    gm = (g - 1.0) / (g + 1.0)
    for i, xi in enumerate(x):
        s = (xi - x0) / t
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    out[:, i] = (rl, ul, pl)
                else:
                    out[:, i] = (rl * (ps / pl + gm) / (gm * ps / pl + 1), us, ps)
            else:  # left rarefaction
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s <= ul - cl:
                    out[:, i] = (rl, ul, pl)
                elif s >= us - cs:
                    out[:, i] = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rho = rl * (c / cl) ** (2 / (g - 1))
                    out[:, i] = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    out[:, i] = (rr, ur, pr)
                else:
                    out[:, i] = (rr * (ps / pr + gm) / (gm * ps / pr + 1), us, ps)
            else:
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s >= ur + cr:
                    out[:, i] = (rr, ur, pr)
                elif s <= us + cs:
                    out[:, i] = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    rho = rr * (c / cr) ** (2 / (g - 1))
                    out[:, i] = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out
