"""Exact solution of the 1-D Riemann problem for an ideal gas.

Textbook method (Toro, Riemann Solvers and Numerical Methods for Fluid
Dynamics, 3rd ed., Ch. 4): Newton iteration on the pressure function for the
star pressure, then self-similar sampling.  Used only as an independent pin.
"""
import math

import numpy as np


def _fK(p, rho, P, c, g):
    if p > P:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * P
        f = (p - P) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - P) / (B + p))
    else:
        f = 2.0 * c / (g - 1.0) * ((p / P) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * c) * (p / P) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g):
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    p = max(1e-12, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(100):
        f1, d1 = _fK(p, rl, pl, cl, g)
        f2, d2 = _fK(p, rr, pr, cr, g)
        pn = p - (f1 + f2 + ur - ul) / (d1 + d2)
        pn = max(pn, 1e-14)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    f1, _ = _fK(p, rl, pl, cl, g)
    f2, _ = _fK(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (f2 - f1)
    return p, u


def sample(xi, rl, ul, pl, rr, ur, pr, g):
    """Density, velocity, pressure at similarity coordinates xi = (x - x0)/t."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    out = np.zeros((3, len(xi)))
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if s <= sl:
                    out[:, n] = (rl, ul, pl)
                else:
                    r = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                    out[:, n] = (r, us, ps)
            else:
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                if s <= ul - cl:
                    out[:, n] = (rl, ul, pl)
                elif s >= us - csl:
                    out[:, n] = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    r = rl * (c / cl) ** (2 / (g - 1))
                    out[:, n] = (r, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:  # right of contact
            if ps > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if s >= sr:
                    out[:, n] = (rr, ur, pr)
                else:
                    r = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                    out[:, n] = (r, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                if s >= ur + cr:
                    out[:, n] = (rr, ur, pr)
                elif s <= us + csr:
                    out[:, n] = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    r = rr * (c / cr) ** (2 / (g - 1))
                    out[:, n] = (r, u, pr * (c / cr) ** (2 * g / (g - 1)))
    return out
