"""Exact Riemann solver for a stiffened gas (test-side reference, independent of the oracle).

Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", ch. 4: the
pressure function with Newton iteration for p*, then sampling of the
self-similar solution.  A stiffened gas p = (gamma-1) rho e - gamma pi_inf is
an ideal gas in the shifted pressure P = p + pi_inf, so the ideal-gas solver
is applied to P.
"""
from __future__ import annotations

import math

import numpy as np


def _fk(P, rho, Pk, ck, g):
    if P > Pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * Pk
        f = (P - Pk) * math.sqrt(A / (P + B))
        df = math.sqrt(A / (B + P)) * (1.0 - (P - Pk) / (2.0 * (B + P)))
    else:       # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((P / Pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (P / Pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(left, right, gamma, pi_inf=0.0):
    """Return (p*, u*) for primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    PL, PR = pl + pi_inf, pr + pi_inf
    cl, cr = math.sqrt(g * PL / rl), math.sqrt(g * PR / rr)
    P = max(1e-12 * (PL + PR), 0.5 * (PL + PR))
    for _ in range(200):
        fl, dl = _fk(P, rl, PL, cl, g)
        fr, dr = _fk(P, rr, PR, cr, g)
        Pn = P - (fl + fr + ur - ul) / (dl + dr)
        if Pn <= 0:
            Pn = 1e-6 * P
        if abs(Pn - P) <= 1e-14 * (Pn + P):
            P = Pn
            break
        P = Pn
    fl, _ = _fk(P, rl, PL, cl, g)
    fr, _ = _fk(P, rr, PR, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return P - pi_inf, u


def sample(left, right, gamma, xi, pi_inf=0.0):
    """Exact (rho, u, p) at similarity coordinates xi = (x - x0) / t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    g = gamma
    PL, PR = pl + pi_inf, pr + pi_inf
    cl, cr = math.sqrt(g * PL / rl), math.sqrt(g * PR / rr)
    ps, us = star_state(left, right, gamma, pi_inf)
    Ps = ps + pi_inf
    gm1, gp1 = g - 1.0, g + 1.0
    out = np.zeros((3, len(xi)))
    for k, s in enumerate(np.asarray(xi, dtype=float)):
        if s <= us:  # left of contact
            if Ps > PL:  # left shock
                rs = rl * ((Ps / PL + gm1 / gp1) / (gm1 / gp1 * Ps / PL + 1.0))
                SL = ul - cl * math.sqrt(gp1 / (2 * g) * Ps / PL + gm1 / (2 * g))
                st = (rl, ul, PL) if s <= SL else (rs, us, Ps)
            else:        # left rarefaction
                rs = rl * (Ps / PL) ** (1.0 / g)
                cs = cl * (Ps / PL) ** (gm1 / (2 * g))
                if s <= ul - cl:
                    st = (rl, ul, PL)
                elif s >= us - cs:
                    st = (rs, us, Ps)
                else:
                    u = 2.0 / gp1 * (cl + gm1 / 2 * ul + s)
                    c = 2.0 / gp1 * (cl + gm1 / 2 * (ul - s))
                    st = (rl * (c / cl) ** (2 / gm1), u, PL * (c / cl) ** (2 * g / gm1))
        else:        # right of contact
            if Ps > PR:
                rs = rr * ((Ps / PR + gm1 / gp1) / (gm1 / gp1 * Ps / PR + 1.0))
                SR = ur + cr * math.sqrt(gp1 / (2 * g) * Ps / PR + gm1 / (2 * g))
                st = (rr, ur, PR) if s >= SR else (rs, us, Ps)
            else:
                rs = rr * (Ps / PR) ** (1.0 / g)
                cs = cr * (Ps / PR) ** (gm1 / (2 * g))
                if s >= ur + cr:
                    st = (rr, ur, PR)
                elif s <= us + cs:
                    st = (rs, us, Ps)
                else:
                    u = 2.0 / gp1 * (-cr + gm1 / 2 * ur + s)
                    c = 2.0 / gp1 * (cr - gm1 / 2 * (ur - s))
                    st = (rr * (c / cr) ** (2 / gm1), u, PR * (c / cr) ** (2 * g / gm1))
        out[:, k] = (st[0], st[1], st[2] - pi_inf)
    return out
