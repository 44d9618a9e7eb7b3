"""Oracle GP weights in 3D, in high precision (mpmath).  TEST INFRASTRUCTURE ONLY.

The 3D form of the reconstruction of Sec. "The (2R+1)th-order GP reconstruction":
eq. (SE-pred) and eq. (SE-cov) are products over the space directions, so in 3D
t*_m = prod_d F(x*_d - m_d; a_d) and C_mn = prod_d G(n_d - m_d; a_d) with the
one-direction factors of the 2D generator (weights_mp.t_factor, c_factor).
Readings (3D is future work in the paper):
  * the stencil of radius R is the L1 ball |di| + |dj| + |dk| <= R (7 cells for
    R = 1, 25 for R = 2), the 3D analogue of the blocky diamond;
  * a face carries the tensor product of the (R+1)-point Gauss rule in its two
    tangential directions (q^2 nodes, weights w_a w_b);
  * z = C^{-1} t*, normalised by its signed sum (as in 2D);
  * the u2 curvature weights are App. B's second derivative of t* at the cell
    centre along each direction, times C^{-1}, on the R = 1 stencil, unnormalised.
"""
from __future__ import annotations

import functools

import mpmath as mp

from . import weights_mp as w2

DPS = 80

# faces: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+
FACES3 = ("x-", "x+", "y-", "y+", "z-", "z+")


def stencil3(R):
    """Offsets (di, dj, dk) with |di| + |dj| + |dk| <= R, ordered by ring then lexicographically."""
    out = []
    for k in range(R + 1):
        ring = [(a, b, c) for a in range(-k, k + 1) for b in range(-k, k + 1) for c in range(-k, k + 1)
                if abs(a) + abs(b) + abs(c) == k]
        out.extend(sorted(ring))
    return out


def face_nodes3(face, R):
    """Gauss nodes of a face: list of ((x*, y*, z*) in cell units, weight), tangential
    directions in increasing axis order, first tangential index outer."""
    g, w = w2.gauss_rule(w2.nq(R))
    ax = face // 2
    s = mp.mpf(-1) / 2 if face % 2 == 0 else mp.mpf(1) / 2
    tang = [d for d in range(3) if d != ax]
    out = []
    for i1, g1 in enumerate(g):
        for i2, g2 in enumerate(g):
            p = [mp.mpf(0)] * 3
            p[ax] = s
            p[tang[0]] = g1
            p[tang[1]] = g2
            out.append((tuple(p), w[i1] * w[i2]))
    return out


def cov3(R, a):
    st = stencil3(R)
    n = len(st)
    C = mp.matrix(n, n)
    for m in range(n):
        for k in range(n):
            v = mp.mpf(1)
            for d in range(3):
                v *= w2.c_factor(mp.mpf(st[k][d] - st[m][d]), a[d])
            C[m, k] = v
    return C


def t3(R, xstar, a):
    st = stencil3(R)
    t = mp.matrix(len(st), 1)
    for m, off in enumerate(st):
        v = mp.mpf(1)
        for d in range(3):
            v *= w2.t_factor(xstar[d] - off[d], a[d])
        t[m] = v
    return t


@functools.lru_cache(maxsize=None)
def _weights3(R, ax, ay, az):
    mp.mp.dps = DPS
    a = (mp.mpf(ax), mp.mpf(ay), mp.mpf(az))
    C = cov3(R, a)
    out = []
    for f in range(6):
        rows = []
        for xs, _ in face_nodes3(f, R):
            z = mp.cholesky_solve(C, t3(R, xs, a))
            s = mp.fsum(z)
            rows.append([z[m] / s for m in range(len(z))])
        out.append(rows)
    return out


def weights3(R, ax, ay=None, az=None, as_float=True):
    """z[face][node][m] for radius R in 3D (faces x-, x+, y-, y+, z-, z+; nodes of
    face_nodes3; stencil order of stencil3).  R = 0: the cell value, one node."""
    ay = ax if ay is None else ay
    az = ax if az is None else az
    if R == 0:
        z = [[[mp.mpf(1)]] for _ in range(6)]
    else:
        z = _weights3(R, str(mp.mpf(ax)), str(mp.mpf(ay)), str(mp.mpf(az)))
    if as_float:
        return [[[float(v) for v in row] for row in face] for face in z]
    return z


def node_weights3(R):
    """Gauss weights of a face's nodes (products of the 1D weights), as floats."""
    return [float(w) for _, w in face_nodes3(1, R)] if R > 0 else [1.0]


@functools.lru_cache(maxsize=None)
def _d2_weights3(ax, ay, az, ell):
    mp.mp.dps = DPS
    a = (mp.mpf(ax), mp.mpf(ay), mp.mpf(az))
    ell = mp.mpf(ell)
    C = cov3(1, a)
    st = stencil3(1)
    out = []
    for d in range(3):
        t = mp.matrix(len(st), 1)
        for m, off in enumerate(st):
            v = mp.mpf(1)
            for e in range(3):
                s = -mp.mpf(off[e])
                v *= w2.d2_t_factor(s, a[e], ell) if e == d else w2.t_factor(s, a[e])
            t[m] = v
        z = mp.cholesky_solve(C, t)
        out.append([z[m] for m in range(len(st))])
    return out


def d2_weights3(ax, ay, az, ell, as_float=True):
    """u2 curvature weights w_d[m] on the R = 1 stencil (order stencil3(1)) for d = x, y, z."""
    z = _d2_weights3(str(mp.mpf(ax)), str(mp.mpf(ay)), str(mp.mpf(az)), str(mp.mpf(ell)))
    if as_float:
        return [[float(v) for v in row] for row in z]
    return z
