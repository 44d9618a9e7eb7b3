"""Seeded synthetic initial conditions shared by the HIP path's tests and the oracle.

This module holds input recipes only: it draws seeded states and converts pointwise
initial data into cell averages.  It contains none of the method's arithmetic (no GP
weights, no fluxes, no detection), so both sides can use it without sharing any code
of the scheme itself.

Every array returned is float64, conservative variables, structure-of-arrays with
shape (nvar, ny, nx) in 2D (nvar = 4: rho, rho*u, rho*v, E) and (5, nz, ny, nx) in
3D, row-major with x fastest.

Recipes (paper: Sec. "Grid convergence -- the isentropic vortex test" for the vortex
and its Gauss-Legendre cell averaging; the four-quadrant and blast problems are
synthetic stand-ins shaped like the paper's shock problems):
  * isentropic vortex, strength beta, mean flow (1, 1), cell averages by the
    5-point Gauss-Legendre rule per axis (25 nodes per cell),
  * four-quadrant Riemann problem, states drawn from numpy's PCG64 with the given
    seed: rho in [0.1, 2], |u|, |v| <= 1.5, p in [0.02, 2]; exact cell averages by
    area fractions,
  * smooth density wave advected at constant velocity and pressure (exact solution
    is a translation), used for convergence checks,
  * 3D blast: ambient rho = 1 with seeded +-1% noise, p = 1e-5, and p = 1e4 in the
    cells whose centres lie within r = 3 dx of the cube centre,
  * implosion (Sec. "The implosion problem in 2D", the set-up of Liska and
    Wendroff that it cites): [0, 0.3]^2 at rest, rho = 0.125, p = 0.14 below the
    line x + y = 0.15 and rho = 1, p = 1 above it, exact cell averages by the
    area below the line; the state is symmetric under x <-> y,
  * Mach 100 light jet (Sec. "Numerical results", Mach jets): [0, 1.5]^2 at rest
    with rho = 10 gamma, p = 1; the jet (rho, u, v, p) = (gamma, 0, 100, 1) enters
    through the slit 0.7 <= x <= 0.8 of the bottom boundary (`MACH_JET_SLIT`).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def _gl5():
    x, w = np.polynomial.legendre.leggauss(5)
    # map [-1, 1] -> [-1/2, 1/2]; weights sum to 1
    return 0.5 * x, 0.5 * w


def prim_to_cons(rho, u, v, p, gamma=GAMMA):
    """Pointwise primitive -> conservative (2D ideal gas)."""
    return np.stack([rho, rho * u, rho * v,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


def cell_centres(n, lo, hi):
    d = (hi - lo) / n
    return lo + (np.arange(n) + 0.5) * d, d


# --------------------------------------------------------------------------
# isentropic vortex (paper: isentropic vortex test, pointwise IC formulas)
# --------------------------------------------------------------------------
def vortex_point(x, y, xc, yc, beta=5.0, mean=(1.0, 1.0), gamma=GAMMA):
    """Pointwise conservative state of the isentropic vortex centred at (xc, yc)."""
    dx = x - xc
    dy = y - yc
    r2 = dx * dx + dy * dy
    e = np.exp(1.0 - r2)
    rho = (1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * e) ** (1.0 / (gamma - 1.0))
    s = beta / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    u = mean[0] - s * dy
    v = mean[1] + s * dx
    p = rho ** gamma
    return prim_to_cons(rho, u, v, p, gamma)


def vortex(nx, ny, lo=(0.0, 0.0), hi=(10.0, 10.0), centre=None, beta=5.0,
           mean=(1.0, 1.0), t=0.0, gamma=GAMMA):
    """Cell-averaged vortex at time t (exact solution: translation by mean*t, periodic).

    The vortex centre is moved by mean*t and wrapped into the box; each quadrature
    node uses the nearest periodic image of the centre.
    """
    Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
    if centre is None:
        centre = (lo[0] + 0.5 * Lx, lo[1] + 0.5 * Ly)
    xc = lo[0] + ((centre[0] + mean[0] * t - lo[0]) % Lx)
    yc = lo[1] + ((centre[1] + mean[1] * t - lo[1]) % Ly)
    xcen, dx = cell_centres(nx, lo[0], hi[0])
    ycen, dy = cell_centres(ny, lo[1], hi[1])
    g, w = _gl5()
    out = np.zeros((4, ny, nx))
    for a in range(5):
        yy = (ycen + g[a] * dy)[:, None]
        for b in range(5):
            xx = (xcen + g[b] * dx)[None, :]
            ddx = xx - xc
            ddy = yy - yc
            ddx = ddx - Lx * np.round(ddx / Lx)
            ddy = ddy - Ly * np.round(ddy / Ly)
            out += w[a] * w[b] * vortex_point(ddx, ddy, 0.0, 0.0, beta, mean, gamma)
    return out


def vortex_bump(nx, ny, lo=(0.0, 0.0), hi=(10.0, 10.0), seed=5, amp=0.05, gamma=GAMMA):
    """Centred vortex plus a Gaussian density bump (velocity and pressure unchanged),
    cell-averaged with the 5x5 Gauss-Legendre rule.  The bump's centre is uniform in
    the middle half of the box and its width in [0.05, 0.1] times the box side
    (numpy PCG64, given seed)."""
    rng = np.random.default_rng(seed)
    Lx, Ly = hi[0] - lo[0], hi[1] - lo[1]
    bx = lo[0] + Lx * (0.25 + 0.5 * rng.random())
    by = lo[1] + Ly * (0.25 + 0.5 * rng.random())
    wid = min(Lx, Ly) * (0.05 + 0.05 * rng.random())
    xc, yc = lo[0] + 0.5 * Lx, lo[1] + 0.5 * Ly
    xcen, dx = cell_centres(nx, lo[0], hi[0])
    ycen, dy = cell_centres(ny, lo[1], hi[1])
    g, w = _gl5()
    out = np.zeros((4, ny, nx))
    for a in range(5):
        yy = (ycen + g[a] * dy)[:, None] + 0.0 * xcen[None, :]
        for b in range(5):
            xx = (xcen + g[b] * dx)[None, :] + 0.0 * ycen[:, None]
            U = vortex_point(xx, yy, xc, yc, 5.0, (1.0, 1.0), gamma)
            rho = U[0]
            u, v = U[1] / rho, U[2] / rho
            p = (gamma - 1.0) * (U[3] - 0.5 * rho * (u * u + v * v))
            rho = rho + amp * np.exp(-((xx - bx) ** 2 + (yy - by) ** 2) / (2.0 * wid * wid))
            out += w[a] * w[b] * prim_to_cons(rho, u, v, p, gamma)
    return out


# --------------------------------------------------------------------------
# four-quadrant Riemann problem (seeded)
# --------------------------------------------------------------------------
def quadrant_states(seed):
    """Four primitive states (rho, u, v, p), quadrants ordered NE, NW, SW, SE."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = []
    for _ in range(4):
        rho = rng.uniform(0.1, 2.0)
        u = rng.uniform(-1.5, 1.5)
        v = rng.uniform(-1.5, 1.5)
        p = rng.uniform(0.02, 2.0)
        st.append((rho, u, v, p))
    return st


def quadrants(nx, ny, seed=1, lo=(0.0, 0.0), hi=(1.0, 1.0), split=(0.5, 0.5), gamma=GAMMA):
    """Exact cell averages of the piecewise-constant four-quadrant state."""
    st = quadrant_states(seed)
    cons = [prim_to_cons(*[np.float64(c) for c in s], gamma=gamma) for s in st]
    xe = np.linspace(lo[0], hi[0], nx + 1)
    ye = np.linspace(lo[1], hi[1], ny + 1)
    # fraction of each cell on the east (x > split) / north (y > split) side
    fe = np.clip((xe[1:] - np.maximum(xe[:-1], split[0])) / (xe[1:] - xe[:-1]), 0.0, 1.0)
    fn = np.clip((ye[1:] - np.maximum(ye[:-1], split[1])) / (ye[1:] - ye[:-1]), 0.0, 1.0)
    fw, fs = 1.0 - fe, 1.0 - fn
    out = np.zeros((4, ny, nx))
    for q, (ax, ay) in enumerate([(fe, fn), (fw, fn), (fw, fs), (fe, fs)]):
        area = ay[:, None] * ax[None, :]
        out += cons[q][:, None, None] * area[None]
    return out


# --------------------------------------------------------------------------
# smooth density wave (constant u, v, p; exact solution is a translation)
# --------------------------------------------------------------------------
def density_wave(nx, ny, L=1.0, amp=0.2, u=1.0, v=1.0, p=1.0, t=0.0, gamma=GAMMA):
    """Cell averages of rho = 1 + amp*sin(2 pi (x + y - (u+v) t)/L), exact by integration."""
    dx = L / nx
    dy = L / ny
    k = 2.0 * math.pi / L
    xe = np.arange(nx + 1) * dx
    ye = np.arange(ny + 1) * dy
    sh = (u + v) * t
    # average of sin(k(x + y - sh)) over a cell = -(1/(k^2 dx dy)) * second difference of sin
    X0, X1 = xe[None, :-1], xe[None, 1:]
    Y0, Y1 = ye[:-1, None], ye[1:, None]
    def S(X, Y):
        return np.sin(k * (X + Y - sh))
    avg = -(S(X1, Y1) - S(X0, Y1) - S(X1, Y0) + S(X0, Y0)) / (k * k * dx * dy)
    rho = 1.0 + amp * avg
    out = np.zeros((4, ny, nx))
    out[0] = rho
    out[1] = rho * u
    out[2] = rho * v
    out[3] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return out


# --------------------------------------------------------------------------
# 1D shock tube laid out along x in an nx-by-ny strip
# --------------------------------------------------------------------------
def shock_tube(nx, ny, left, right, x0=0.5, gamma=GAMMA):
    """Primitive (rho, u, p) left/right states split at x0 on [0,1]; v = 0."""
    xe = np.linspace(0.0, 1.0, nx + 1)
    fr = np.clip((xe[1:] - np.maximum(xe[:-1], x0)) / (xe[1:] - xe[:-1]), 0.0, 1.0)
    cl = prim_to_cons(np.float64(left[0]), np.float64(left[1]), 0.0, np.float64(left[2]), gamma)
    cr = prim_to_cons(np.float64(right[0]), np.float64(right[1]), 0.0, np.float64(right[2]), gamma)
    row = cl[:, None] * (1.0 - fr)[None] + cr[:, None] * fr[None]
    return np.repeat(row[:, None, :], ny, axis=1).copy()


# --------------------------------------------------------------------------
# Random cell-wise state (stress input: most cells troubled)
# --------------------------------------------------------------------------
def noise(nx, ny, seed=11, sigma=0.6, gamma=GAMMA):
    """Cell-wise random state: log-normal density and pressure (log-sd sigma),
    standard-normal velocities (PCG64 seed).  Almost every cell is rough, so a
    stage lowers a large share of the grid."""
    rng = np.random.default_rng(seed)
    rho = np.exp(rng.normal(0.0, sigma, (ny, nx)))
    u = rng.normal(0.0, 1.0, (ny, nx))
    v = rng.normal(0.0, 1.0, (ny, nx))
    p = np.exp(rng.normal(0.0, sigma, (ny, nx)))
    return prim_to_cons(rho, u, v, p, gamma)


# --------------------------------------------------------------------------
# Implosion in a box with reflecting walls
# --------------------------------------------------------------------------
def implosion(n, L=0.3, cut=0.15, inner=(0.125, 0.14), outer=(1.0, 1.0), gamma=GAMMA):
    """Cell averages on an n-by-n grid of [0, L]^2: (rho, p) = inner below the line
    x + y = cut, outer above it, at rest.  The fraction of cell (i, j) below the line
    is the area of {a + b < s} in the unit square, s = cut/dx - i - j."""
    dx = L / n
    idx = np.arange(n, dtype=np.float64)
    s = cut / dx - (idx[None, :] + idx[:, None])
    frac = np.where(s <= 0.0, 0.0, np.where(s >= 2.0, 1.0,
                    np.where(s <= 1.0, 0.5 * s * s, 1.0 - 0.5 * (2.0 - s) ** 2)))
    rho = inner[0] * frac + outer[0] * (1.0 - frac)
    E = (inner[1] * frac + outer[1] * (1.0 - frac)) / (gamma - 1.0)
    out = np.zeros((4, n, n))
    out[0] = rho
    out[3] = E
    return out


# --------------------------------------------------------------------------
# Mach 100 light jet
# --------------------------------------------------------------------------
MACH_JET_SLIT = (1, 0.7, 0.8, (GAMMA, 0.0, 100.0, 1.0))  # bottom side, x range, (rho, u, v, p)


DOUBLE_JET_SLIT = (3, 0.7, 0.8, (GAMMA, 0.0, 800.0, 1.0), (GAMMA, 0.0, -800.0, 1.0))  # both sides


def double_jet(n, gamma=GAMMA):
    """The double Mach 800 jet collision: the stratified ambient rho = -9.24 y + 14
    (cell averages of a linear profile: its value at the centre), p = 1, at rest, on
    [0, 1.5]^2; jets (gamma, 0, +-800, 1) enter through DOUBLE_JET_SLIT."""
    y = (np.arange(n) + 0.5) * 1.5 / n
    rho = np.repeat((-9.24 * y + 14.0)[:, None], n, axis=1)
    z = np.zeros((n, n))
    return prim_to_cons(rho, z, z, np.ones((n, n)), gamma)


def mach_jet(n, gamma=GAMMA):
    """The ambient state (rho, u, v, p) = (10 gamma, 0, 0, 1) on an n-by-n grid of
    [0, 1.5]^2; the jet enters through the boundary slit MACH_JET_SLIT."""
    rho = np.full((n, n), 10.0 * gamma)
    z = np.zeros((n, n))
    return prim_to_cons(rho, z, z, np.ones((n, n)), gamma)


# --------------------------------------------------------------------------
# 3D blast (seeded density noise)
# --------------------------------------------------------------------------
def density_wave3d(n, amp=0.2, u=1.0, v=1.0, w=1.0, p=1.0, t=0.0, gamma=GAMMA):
    """Smooth 3D density wave on the periodic unit cube, rho = 1 + amp sin(2 pi (x+y+z -
    (u+v+w) t)), constant velocity and pressure: exact cell averages of the translated
    wave (5, n, n, n)."""
    c, d = cell_centres(n, 0.0, 1.0)
    ph = 2.0 * math.pi * (c[None, None, :] + c[None, :, None] + c[:, None, None] - (u + v + w) * t)
    f = (math.sin(math.pi * d) / (math.pi * d)) ** 3
    rho = 1.0 + amp * f * np.sin(ph)
    out = np.zeros((5, n, n, n))
    out[0] = rho
    out[1] = rho * u
    out[2] = rho * v
    out[3] = rho * w
    out[4] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return out


def blast3d(n, seed=3, r_cells=3.0, p_in=1e4, p_out=1e-5, noise=0.01, gamma=GAMMA):
    rng = np.random.Generator(np.random.PCG64(seed))
    rho = 1.0 + noise * rng.uniform(-1.0, 1.0, size=(n, n, n))
    c = (np.arange(n) + 0.5) - 0.5 * n  # cell-centre offsets in cell units
    d2 = c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2
    p = np.where(d2 <= r_cells * r_cells, p_in, p_out)
    out = np.zeros((5, n, n, n))
    out[0] = rho
    out[4] = p / (gamma - 1.0)
    return out
