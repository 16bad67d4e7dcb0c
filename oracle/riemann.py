"""Exact solution of the one-dimensional Riemann problem of an ideal gas
(TEST INFRASTRUCTURE).

The Sod shock tube of Sec. 4.2 is compared against this solution.  Two
uniform states (rho, u, p) meet at x0 at t = 0; for t > 0 the solution is
self-similar in S = (x - x0)/t and consists of a left wave (rarefaction or
shock), a contact discontinuity moving with the star-region velocity u*, and
a right wave.  This is the textbook construction (Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", Ch. 4): the star pressure p* is the
root of

    f(p) = f_L(p) + f_R(p) + (u_R - u_L) = 0,

    f_K(p) = (p - p_K) sqrt(A_K / (p + B_K))                       p > p_K (shock)
           = 2 c_K/(gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1)    p <= p_K (rarefaction)

with A_K = 2/((gamma+1) rho_K), B_K = (gamma-1)/(gamma+1) p_K, and
u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.  The root is bracketed and found
by bisection refined to machine precision (f is monotone increasing).
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, ck, g):
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, gamma):
    """(p*, u*, rho*_L, rho*_R) for left = (rho, u, p), right = (rho, u, p)."""
    rl, ul, pl = map(float, left)
    rr, ur, pr = map(float, right)
    g = float(gamma)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("the states produce a vacuum")
    f = lambda p: _fk(p, rl, pl, cl, g) + _fk(p, rr, pr, cr, g) + (ur - ul)
    lo, hi = 0.0, max(pl, pr)
    while f(hi) < 0.0:
        hi *= 2.0
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    ps = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_fk(ps, rr, pr, cr, g) - _fk(ps, rl, pl, cl, g))
    gm = (g - 1.0) / (g + 1.0)

    def rho_star(rk, pk):
        if ps > pk:
            return rk * (ps / pk + gm) / (gm * ps / pk + 1.0)
        return rk * (ps / pk) ** (1.0 / g)

    return ps, us, rho_star(rl, pl), rho_star(rr, pr)


def solution(S, left, right, gamma):
    """rho, u, p at the similarity coordinates S = (x - x0)/t (array)."""
    rl, ul, pl = map(float, left)
    rr, ur, pr = map(float, right)
    g = float(gamma)
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)
    ps, us, rsl, rsr = star_state(left, right, gamma)
    S = np.asarray(S, dtype=np.float64)
    rho, u, p = np.empty_like(S), np.empty_like(S), np.empty_like(S)
    e = (g - 1.0) / (2.0 * g)
    for k, s in enumerate(S.ravel()):
        if s <= us:       # left of the contact
            if ps > pl:   # left shock
                sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + e)
                val = (rl, ul, pl) if s <= sl else (rsl, us, ps)
            else:         # left rarefaction: head at u_L - c_L, tail at u* - c*_L
                csl = cl * (ps / pl) ** e
                if s <= ul - cl:
                    val = (rl, ul, pl)
                elif s >= us - csl:
                    val = (rsl, us, ps)
                else:
                    t = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cl) * (ul - s)
                    val = (rl * t ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (cl + 0.5 * (g - 1.0) * ul + s),
                           pl * t ** (2.0 * g / (g - 1.0)))
        else:             # right of the contact
            if ps > pr:   # right shock
                sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + e)
                val = (rr, ur, pr) if s >= sr else (rsr, us, ps)
            else:         # right rarefaction: head at u_R + c_R, tail at u* + c*_R
                csr = cr * (ps / pr) ** e
                if s >= ur + cr:
                    val = (rr, ur, pr)
                elif s <= us + csr:
                    val = (rsr, us, ps)
                else:
                    t = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cr) * (ur - s)
                    val = (rr * t ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (-cr + 0.5 * (g - 1.0) * ur + s),
                           pr * t ** (2.0 * g / (g - 1.0)))
        rho.flat[k], u.flat[k], p.flat[k] = val
    return rho, u, p


def shock_speed_right(left, right, gamma):
    """Speed of the right-moving shock (requires p* > p_R)."""
    rr, ur, pr = map(float, right)
    g = float(gamma)
    cr = math.sqrt(g * pr / rr)
    ps = star_state(left, right, gamma)[0]
    return ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
