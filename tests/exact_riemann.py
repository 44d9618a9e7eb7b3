"""Exact Riemann solver for the 1D Euler equations (Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", ch. 4): Newton iteration for the star
pressure, then sampling of the self-similar solution.  Used only as an
independent pin for the oracle's HLLC + FOG shock tubes."""
import math

import numpy as np


def _fk(p, rho, pk, g):
    a = math.sqrt(g * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1.0 - 0.5 * (p - pk) / (B + p))
    # rarefaction
    r = p / pk
    return (2.0 * a / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0),
            1.0 / (rho * a) * r ** (-(g + 1.0) / (2.0 * g)))


def star(left, right, g=1.4):
    rl, ul, pl = left
    rr, ur, pr = right
    p = max(1e-8, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dl = _fk(p, rl, pl, g)
        fr, dr = _fk(p, rr, pr, g)
        f = fl + fr + (ur - ul)
        pn = max(1e-12, p - f / (dl + dr))
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, g)
    fr, _ = _fk(p, rr, pr, g)
    return p, 0.5 * (ul + ur) + 0.5 * (fr - fl)


def sample(left, right, xi, g=1.4):
    """(rho, u, p) at similarity coordinate xi = x/t."""
    ps, us = star(left, right, g)
    rl, ul, pl = left
    rr, ur, pr = right
    if xi <= us:
        rho, u, p = rl, ul, pl
        a = math.sqrt(g * p / rho)
        if ps > p:
            sh = u - a * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
            if xi <= sh:
                return rho, u, p
            r = ps / p
            return rho * (r + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * r + 1), us, ps
        ast = a * (ps / p) ** ((g - 1) / (2 * g))
        if xi <= u - a:
            return rho, u, p
        if xi >= us - ast:
            return rho * (ps / p) ** (1 / g), us, ps
        c = 2 / (g + 1) + (g - 1) / ((g + 1) * a) * (u - xi)
        return rho * c ** (2 / (g - 1)), 2 / (g + 1) * (a + (g - 1) / 2 * u + xi), p * c ** (2 * g / (g - 1))
    rho, u, p = rr, ur, pr
    a = math.sqrt(g * p / rho)
    if ps > p:
        sh = u + a * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
        if xi >= sh:
            return rho, u, p
        r = ps / p
        return rho * (r + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * r + 1), us, ps
    ast = a * (ps / p) ** ((g - 1) / (2 * g))
    if xi >= u + a:
        return rho, u, p
    if xi <= us + ast:
        return rho * (ps / p) ** (1 / g), us, ps
    c = 2 / (g + 1) - (g - 1) / ((g + 1) * a) * (u - xi)
    return rho * c ** (2 / (g - 1)), 2 / (g + 1) * (-a + (g - 1) / 2 * u + xi), p * c ** (2 * g / (g - 1))


def cell_average_density(left, right, nx, t, x0=0.5, g=1.4, sub=64):
    """Cell averages of the exact density on [0, 1] (midpoint sub-sampling)."""
    out = np.zeros(nx)
    for i in range(nx):
        xs = (i + (np.arange(sub) + 0.5) / sub) / nx
        out[i] = np.mean([sample(left, right, (x - x0) / t, g)[0] for x in xs])
    return out
