"""Exact solution of the 1D ideal-gas Riemann problem (TEST INFRASTRUCTURE).

Follows the standard construction in Toro, "Riemann Solvers and Numerical
Methods for Fluid Dynamics", ch. 4: the star-region pressure solves
f_L(p) + f_R(p) + (u_R - u_L) = 0 with the shock / rarefaction branches of
f_K, found by Newton iteration; the solution is then sampled on x/t.
"""
import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:  # shock
        a = 2.0 / ((g + 1.0) * rho)
        b = (g - 1.0) / (g + 1.0) * pk
        q = math.sqrt(a / (p + b))
        f = (p - pk) * q
        df = q * (1.0 - 0.5 * (p - pk) / (b + p))
    else:  # rarefaction
        pr = p / pk
        f = 2.0 * ck / (g - 1.0) * (pr ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * pr ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(100):
        fl, dfl = _fk(p, rl, pl, cl, g)
        fr, dfr = _fk(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= 1e-15 * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, cl, g)
    fr, _ = _fk(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, g):
    """(rho, u, p) at similarity coordinate xi = x / t (array)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    r, uu, pp = rl, ul, pl
                else:
                    r, uu, pp = rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps
            else:
                cs = cl * (ps / pl) ** ((g - 1) / (2 * g))
                head, tail = ul - cl, us - cs
                if s <= head:
                    r, uu, pp = rl, ul, pl
                elif s >= tail:
                    r, uu, pp = rl * (ps / pl) ** (1.0 / g), us, ps
                else:
                    fac = 2.0 / (g + 1) + gm / cl * (ul - s)
                    r = rl * fac ** (2.0 / (g - 1))
                    uu = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    pp = pl * fac ** (2 * g / (g - 1))
        else:  # right of contact
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    r, uu, pp = rr, ur, pr
                else:
                    r, uu, pp = rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps
            else:
                cs = cr * (ps / pr) ** ((g - 1) / (2 * g))
                head, tail = ur + cr, us + cs
                if s >= head:
                    r, uu, pp = rr, ur, pr
                elif s <= tail:
                    r, uu, pp = rr * (ps / pr) ** (1.0 / g), us, ps
                else:
                    fac = 2.0 / (g + 1) - gm / cr * (ur - s)
                    r = rr * fac ** (2.0 / (g - 1))
                    uu = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    pp = pr * fac ** (2 * g / (g - 1))
        rho[n], u[n], p[n] = r, uu, pp
    return rho, u, p
