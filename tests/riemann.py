"""Exact solution of the Riemann problem of the 1-D Euler equations (ideal
gas), for validating computed shock-tube solutions.

Textbook construction: the star-region pressure p* solves
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock relation
(p - p_K) sqrt(A_K / (p + B_K)), A_K = 2 / ((gamma+1) rho_K),
B_K = (gamma-1)/(gamma+1) p_K, when p > p_K, and the rarefaction relation
2 c_K/(gamma-1) ((p/p_K)^((gamma-1)/(2 gamma)) - 1) otherwise; it is found by
Newton's method from the two-rarefaction estimate.  The solution is then
sampled on x/t through the left wave, the contact (speed u*) and the right
wave (shock speeds from the Rankine-Hugoniot conditions, rarefaction fans
self-similar).
"""

import numpy as np


def _f(p, rho, pk, g):
    c = np.sqrt(g * pk / rho)
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = np.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (p + B))
    r = p / pk
    e = (g - 1.0) / (2.0 * g)
    return 2.0 * c / (g - 1.0) * (r ** e - 1.0), r ** (-(g + 1.0) / (2.0 * g)) / (rho * c)


def star_state(left, right, g=1.4):
    """(p*, u*) for primitive states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    e = (g - 1.0) / (2.0 * g)
    p = ((cl + cr - 0.5 * (g - 1.0) * (ur - ul)) / (cl / pl ** e + cr / pr ** e)) ** (1.0 / e)
    for _ in range(100):
        fl, dl = _f(p, rl, pl, g)
        fr, dr = _f(p, rr, pr, g)
        step = (fl + fr + ur - ul) / (dl + dr)
        pn = max(p - step, 1e-14)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _f(p, rl, pl, g)
    fr, _ = _f(p, rr, pr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) at similarity coordinates xi = (x - x0)/t."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    out = np.zeros((3,) + xi.shape)
    gm, gp = (g - 1.0) / (g + 1.0), (g + 1.0) / (2.0 * g)
    for idx, s in np.ndenumerate(xi):
        if s <= us:    # left of the contact
            c = np.sqrt(g * pl / rl)
            if ps > pl:
                sh = ul - c * np.sqrt(gp * ps / pl + (g - 1.0) / (2.0 * g))
                st = (rl * (ps / pl + gm) / (gm * ps / pl + 1.0), us, ps)
                w = (rl, ul, pl) if s <= sh else st
            else:
                cs = c * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                head, tail = ul - c, us - cs
                if s <= head:
                    w = (rl, ul, pl)
                elif s >= tail:
                    w = (rl * (ps / pl) ** (1.0 / g), us, ps)
                else:
                    k = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * c) * (ul - s)
                    w = (rl * k ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (c + 0.5 * (g - 1.0) * ul + s),
                         pl * k ** (2.0 * g / (g - 1.0)))
        else:          # right of the contact
            c = np.sqrt(g * pr / rr)
            if ps > pr:
                sh = ur + c * np.sqrt(gp * ps / pr + (g - 1.0) / (2.0 * g))
                st = (rr * (ps / pr + gm) / (gm * ps / pr + 1.0), us, ps)
                w = (rr, ur, pr) if s >= sh else st
            else:
                cs = c * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                head, tail = ur + c, us + cs
                if s >= head:
                    w = (rr, ur, pr)
                elif s <= tail:
                    w = (rr * (ps / pr) ** (1.0 / g), us, ps)
                else:
                    k = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * c) * (ur - s)
                    w = (rr * k ** (2.0 / (g - 1.0)), 2.0 / (g + 1.0) * (-c + 0.5 * (g - 1.0) * ur + s),
                         pr * k ** (2.0 * g / (g - 1.0)))
        out[(slice(None),) + idx] = w
    return out
