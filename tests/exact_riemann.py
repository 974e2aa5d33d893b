"""Exact Riemann solver for the gamma-law Euler equations (test utility).

Written independently of the oracle: the textbook pressure-function form
(shock branch from the Rankine-Hugoniot relations, rarefaction branch from
the isentropic Riemann invariants), solved by safeguarded Newton iteration,
and the complete self-similar wave fan sampled at any x/t.  It pins the
oracle's two-shock solver (both agree exactly when both waves are shocks) and
the 1-D shock-tube runs of the whole step.
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, cK, g):
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        f = (p - pK) * s
        df = s * (1.0 - 0.5 * (p - pK) / (B + p))
    else:  # rarefaction
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * cK / (g - 1.0) * ((p / pK) ** e - 1.0)
        df = 1.0 / (rho * cK) * (p / pK) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rl, ul, pl, rr, ur, pr, g, tol=1e-15, maxit=200):
    """(p*, u*) of the exact solution."""
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    du = ur - ul
    # two-rarefaction guess, bounded below
    e = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * du) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    p = max(p, 1e-14 * min(pl, pr))
    for _ in range(maxit):
        fl, dfl = _fK(p, rl, pl, cl, g)
        fr, dfr = _fK(p, rr, pr, cr, g)
        pn = p - (fl + fr + du) / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fK(p, rl, pl, cl, g)
    fr, _ = _fK(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(rl, ul, pl, rr, ur, pr, g, xi):
    """Exact (rho, u, p) at similarity coordinate xi = x/t (array)."""
    ps, us = star_state(rl, ul, pl, rr, ur, pr, g)
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros((3,) + xi.shape)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    gm = (g - 1.0) / (g + 1.0)
    for idx, s in np.ndenumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:
                rs = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                sh = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                val = (rl, ul, pl) if s <= sh else (rs, us, ps)
            else:
                rs = rl * (ps / pl) ** (1.0 / g)
                csl = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                shd, stl = ul - cl, us - csl
                if s <= shd:
                    val = (rl, ul, pl)
                elif s >= stl:
                    val = (rs, us, ps)
                else:
                    r = rl * (2.0 / (g + 1.0) + gm / cl * (ul - s)) ** (2.0 / (g - 1.0))
                    u = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + s)
                    p = pl * (2.0 / (g + 1.0) + gm / cl * (ul - s)) ** (2.0 * g / (g - 1.0))
                    val = (r, u, p)
        else:
            if ps > pr:
                rs = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                sh = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                val = (rr, ur, pr) if s >= sh else (rs, us, ps)
            else:
                rs = rr * (ps / pr) ** (1.0 / g)
                csr = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                shd, stl = ur + cr, us + csr
                if s >= shd:
                    val = (rr, ur, pr)
                elif s <= stl:
                    val = (rs, us, ps)
                else:
                    r = rr * (2.0 / (g + 1.0) - gm / cr * (ur - s)) ** (2.0 / (g - 1.0))
                    u = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + s)
                    p = pr * (2.0 / (g + 1.0) - gm / cr * (ur - s)) ** (2.0 * g / (g - 1.0))
                    val = (r, u, p)
        out[(slice(None),) + idx] = val
    return out
