"""Exact solution of the Riemann problem of 1D gas dynamics (ideal gas),
written from the standard textbook construction (pressure function of the
two non-linear waves, Newton iteration for the star pressure, self-similar
sampling of shocks and rarefaction fans).  Test helper: the hydrodynamic
limit (B = 0) of the MHD solvers is checked against it.  Shares nothing
with the oracle or the GPU library."""
from __future__ import annotations

import math

import numpy as np


def _wave_fn(p, rho, pk, gamma):
    """Velocity jump across the wave joining state (rho, pk) to pressure p,
    and its derivative in p (shock if p > pk, rarefaction otherwise)."""
    a = math.sqrt(gamma * pk / rho)
    if p > pk:
        A = 2.0 / ((gamma + 1.0) * rho)
        Bc = (gamma - 1.0) / (gamma + 1.0) * pk
        q = math.sqrt(A / (p + Bc))
        return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (Bc + p))
    r = (p / pk) ** ((gamma - 1.0) / (2.0 * gamma))
    return 2.0 * a / (gamma - 1.0) * (r - 1.0), 1.0 / (rho * a) * (p / pk) ** (-(gamma + 1.0) / (2.0 * gamma))


def star_state(left, right, gamma):
    """(p*, u*) between the left and right states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al, ar = math.sqrt(gamma * pl / rl), math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise ValueError("the states generate a vacuum")
    # two-rarefaction estimate as the starting point (positive by construction)
    z = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul)) / (al / pl ** z + ar / pr ** z)) ** (1.0 / z)
    for _ in range(100):
        fl, dl = _wave_fn(p, rl, pl, gamma)
        fr, dr = _wave_fn(p, rr, pr, gamma)
        f = fl + fr + ur - ul
        pn = max(p - f / (dl + dr), 1e-14 * p)
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _wave_fn(p, rl, pl, gamma)
    fr, _ = _wave_fn(p, rr, pr, gamma)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, gamma, s):
    """(rho, u, p) of the exact solution at x / t = s (array)."""
    ps, us = star_state(left, right, gamma)
    s = np.atleast_1d(np.asarray(s, dtype=np.float64))
    out = np.empty((3, s.size))
    g1, g2 = (gamma - 1.0) / (gamma + 1.0), (gamma - 1.0) / (2.0 * gamma)
    for n, x in enumerate(s):
        if x <= us:
            rho, u, p, sign = left[0], left[1], left[2], 1.0
        else:
            rho, u, p, sign = right[0], right[1], right[2], -1.0
        a = math.sqrt(gamma * p / rho)
        # work in the frame where the wave of interest is the left one
        xs, uk, ust = sign * x, sign * u, sign * us
        if ps > p:                                    # shock
            S = uk - a * math.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / p + g2)
            if xs <= S:
                out[:, n] = (rho, u, p)
            else:
                out[:, n] = (rho * (ps / p + g1) / (g1 * ps / p + 1.0), us, ps)
        else:                                         # rarefaction
            head = uk - a
            a_star = a * (ps / p) ** g2
            tail = ust - a_star
            if xs <= head:
                out[:, n] = (rho, u, p)
            elif xs >= tail:
                out[:, n] = (rho * (ps / p) ** (1.0 / gamma), us, ps)
            else:
                uf = 2.0 / (gamma + 1.0) * (a + 0.5 * (gamma - 1.0) * uk + xs)
                af = 2.0 / (gamma + 1.0) * (a + 0.5 * (gamma - 1.0) * (uk - xs))
                out[:, n] = (rho * (af / a) ** (2.0 / (gamma - 1.0)), sign * uf,
                             p * (af / a) ** (2.0 * gamma / (gamma - 1.0)))
    return out
