"""Oracle GP weights in high precision (mpmath).  TEST INFRASTRUCTURE ONLY.

This is the oracle's own generator of GP prediction vectors.  Only tests/, the
smoke check and the benchmark's CPU-baseline leg may use it; the product library
generates its weights independently (quad precision C++) and never imports this.

Everything follows Bourgeois & Lee, "GP-MOOD", Sec. "The (2R+1)th-order GP
reconstruction" and Sec. "Singularity of the covariance kernel matrix":

  * the GP stencil of radius R is the blocky diamond |di| + |dj| <= R
    (Sec. "The GP stencil": 5 / 13 / 25 cells for R = 1 / 2 / 3);
  * the face points are the Gauss rules of Table tab:QR-pt-weight with q = R + 1;
  * t*_m is eq. (SE-pred), C_mn is eq. (SE-cov), with Delta_{mn,d} of eq. (delta_mnd)
    in cell units and a_d = ell / Delta_d;
  * z = C^{-1} t* by Cholesky (as the paper does), then normalised by its signed
    sum so that z^T 1 = 1 (eq. (normalized_z); see the reading below);
  * the u2 curvature weights are App. B's second derivative of t* at the cell
    centre, times C^{-1}, for the R = 1 stencil, not normalised.

Readings of the paper taken here (each is also listed in the design notes):
  * eq. (normalized_z) says "L1 norm" but states the purpose z^T 1 = 1; the GP
    weights have negative entries, so only the signed sum achieves that purpose.
  * eq. (SE-cov) drops the subscript d on one Delta; it is ell/Delta_d.
  * the integrand printed for t* is q(x); it is the kernel K(x*, x) averaged over
    the cell, consistent with eq. (SE-pred).
  * R = 2, 3 stencil orderings are only in figures; any fixed order gives the same
    result.  The order used here is ring by ring (|di| + |dj| = k), each ring
    clockwise starting at (-k, 0); for R = 1 this is App. A's order
    (centre, left, top, right, bottom).

The paper computes in quadruple precision and rounds to double; here mpmath runs
at 80 significant digits and rounds to double at the end.
"""
from __future__ import annotations

import functools

import mpmath as mp

DPS = 80

FACES = ("x-", "x+", "y-", "y+")


def _ctx():
    mp.mp.dps = DPS


def stencil(R, shape="diamond"):
    """Offsets (di, dj) of the radius-R GP stencil in the oracle's order."""
    if R == 0:
        return [(0, 0)]
    out = [(0, 0)]
    for k in range(1, R + 1):
        ring = []
        # clockwise from (-k, 0): up-left edge to (0, k), then to (k, 0), (0, -k), back
        for t in range(k):
            ring.append((-k + t, t))          # (-k,0) -> (0,k) exclusive
        for t in range(k):
            ring.append((t, k - t))           # (0,k) -> (k,0) exclusive
        for t in range(k):
            ring.append((k - t, -t))          # (k,0) -> (0,-k) exclusive
        for t in range(k):
            ring.append((-t, -k + t))         # (0,-k) -> (-k,0) exclusive
        if shape == "cross":
            ring = [o for o in ring if o[0] == 0 or o[1] == 0]
        out.extend(ring)
    return out


def gauss_rule(q):
    """Nodes and weights on [-1/2, 1/2] from Table tab:QR-pt-weight (nodes g_1 > g_2 > ...)."""
    _ctx()
    if q == 1:
        return [mp.mpf(0)], [mp.mpf(1)]
    if q == 2:
        g = 1 / (2 * mp.sqrt(3))
        return [g, -g], [mp.mpf(1) / 2, mp.mpf(1) / 2]
    if q == 3:
        g = mp.sqrt(mp.mpf(3) / 5) / 2
        return [g, mp.mpf(0), -g], [mp.mpf(5) / 18, mp.mpf(8) / 18, mp.mpf(5) / 18]
    if q == 4:
        s = mp.sqrt(mp.mpf(6) / 5)
        g1 = mp.sqrt(mp.mpf(3) / 7 + 2 * s / 7) / 2
        g2 = mp.sqrt(mp.mpf(3) / 7 - 2 * s / 7) / 2
        w1 = (18 - mp.sqrt(30)) / 72
        w2 = (18 + mp.sqrt(30)) / 72
        return [g1, g2, -g2, -g1], [w1, w2, w2, w1]
    raise ValueError("q must be 1..4")


def nq(R):
    """Quadrature points per face for radius R (Step 3 of the stepwise algorithm; FOG: 1)."""
    return 1 if R == 0 else R + 1


def face_point(face, g):
    """x* in cell units relative to the cell centre for face index and node g."""
    return {0: (mp.mpf(-1) / 2, g), 1: (mp.mpf(1) / 2, g),
            2: (g, mp.mpf(-1) / 2), 3: (g, mp.mpf(1) / 2)}[face]


def delta_table(R, xstar):
    """Delta_{mn,d} of eq. (delta_mnd) for the stencil plus the point x* (App. A layout).

    Returns (dx_table, dy_table) as lists of rows indexed [n][m] over the stencil cells
    followed by x*.
    """
    pts = [(mp.mpf(a), mp.mpf(b)) for a, b in stencil(R)] + [xstar]
    tx = [[pts[n][0] - pts[m][0] for m in range(len(pts))] for n in range(len(pts))]
    ty = [[pts[n][1] - pts[m][1] for m in range(len(pts))] for n in range(len(pts))]
    return tx, ty


def t_factor(s, a):
    """One-direction factor of eq. (SE-pred): sqrt(pi/2) a [erf((s+1/2)/(sqrt2 a)) - erf((s-1/2)/(sqrt2 a))]."""
    r2a = mp.sqrt(2) * a
    return mp.sqrt(mp.pi / 2) * a * (mp.erf((s + mp.mpf(1) / 2) / r2a) - mp.erf((s - mp.mpf(1) / 2) / r2a))


def c_factor(D, a):
    """One-direction factor of eq. (SE-cov) at integer separation D (cell units)."""
    r2a = mp.sqrt(2) * a
    up, um, u0 = (D + 1) / r2a, (D - 1) / r2a, D / r2a
    return mp.sqrt(mp.pi) * a * a * (
        (up * mp.erf(up) + um * mp.erf(um))
        + (mp.exp(-up * up) + mp.exp(-um * um)) / mp.sqrt(mp.pi)
        - 2 * (u0 * mp.erf(u0) + mp.exp(-u0 * u0) / mp.sqrt(mp.pi)))


def d2_t_factor(s, a, ell):
    """App. B: second derivative of the eq. (SE-pred) factor w.r.t. the physical x*_d."""
    e = lambda x: mp.exp(-(x * x) / (2 * a * a))
    h = mp.mpf(1) / 2
    return ((s - h) * e(s - h) - (s + h) * e(s + h)) / (ell * ell)


def cov_matrix(R, ax, ay, shape="diamond"):
    _ctx()
    st = stencil(R, shape)
    n = len(st)
    C = mp.matrix(n, n)
    for m in range(n):
        for k in range(n):
            Dx = mp.mpf(st[k][0] - st[m][0])
            Dy = mp.mpf(st[k][1] - st[m][1])
            C[m, k] = c_factor(Dx, ax) * c_factor(Dy, ay)
    return C


def t_vector(R, xstar, ax, ay, shape="diamond"):
    _ctx()
    st = stencil(R, shape)
    t = mp.matrix(len(st), 1)
    for m, (di, dj) in enumerate(st):
        t[m] = t_factor(xstar[0] - di, ax) * t_factor(xstar[1] - dj, ay)
    return t


@functools.lru_cache(maxsize=None)
def _weights_mp(R, ax, ay, shape):
    _ctx()
    ax = mp.mpf(ax)
    ay = mp.mpf(ay)
    C = cov_matrix(R, ax, ay, shape)
    g, _ = gauss_rule(nq(R))
    out = []
    for f in range(4):
        rows = []
        for gk in g:
            t = t_vector(R, face_point(f, gk), ax, ay, shape)
            z = mp.cholesky_solve(C, t)            # z = C^{-1} t (C symmetric)
            s = mp.fsum(z)
            rows.append([z[m] / s for m in range(len(z))])
        out.append(rows)
    return out


def weights(R, ax, ay=None, shape="diamond", as_float=True):
    """Normalised prediction vectors z[face][point][m] for radius R.

    ax, ay: ell / dx and ell / dy (given as strings or numbers; converted exactly).
    Faces are ordered x-, x+, y-, y+; points follow Table tab:QR-pt-weight; the
    stencil order is stencil(R).
    """
    if ay is None:
        ay = ax
    if R == 0:
        z = [[[mp.mpf(1)]] for _ in range(4)]
    else:
        z = _weights_mp(R, str(mp.mpf(ax)) if not isinstance(ax, str) else ax,
                        str(mp.mpf(ay)) if not isinstance(ay, str) else ay, shape)
    if as_float:
        return [[[float(v) for v in row] for row in face] for face in z]
    return z


def poly3_weights(as_float=True):
    """POL-MOOD3 (Sec. "POL-MOOD3", eqs. (poly3), (p3_coeffs)): point values of the
    quadratic p3(x, y) = a0 + a1 x + a2 x^2 + a3 y + a4 y^2 whose cell averages
    match the five cells of the radius-1 stencil, in the layout of weights(1, ...)
    (faces x-, x+, y-, y+; 2-point rule; stencil order stencil(1)).  Along the
    face's normal the 1D quadratic gives -1/6, 5/6, 1/3; along the face only the
    linear term survives at the Gauss nodes (x*^2 = 1/12 cancels the average of
    the quadratic), so the two tangential neighbours weigh +-x*/2."""
    _ctx()
    g, _ = gauss_rule(2)
    st = stencil(1)
    out = []
    for f in range(4):
        rows = []
        for gk in g:
            xs, ys = face_point(f, gk)
            w = {}
            if f < 2:  # x faces: normal along x, tangential along y
                s = 1 if xs > 0 else -1
                w[(0, 0)] = mp.mpf(5) / 6
                w[(s, 0)] = mp.mpf(1) / 3
                w[(-s, 0)] = -mp.mpf(1) / 6
                w[(0, 1)] = ys / 2
                w[(0, -1)] = -ys / 2
            else:
                s = 1 if ys > 0 else -1
                w[(0, 0)] = mp.mpf(5) / 6
                w[(0, s)] = mp.mpf(1) / 3
                w[(0, -s)] = -mp.mpf(1) / 6
                w[(1, 0)] = xs / 2
                w[(-1, 0)] = -xs / 2
            rows.append([w[o] for o in st])
        out.append(rows)
    if as_float:
        return [[[float(v) for v in row] for row in face] for face in out]
    return out


def raw_weight_sum(R, ax, ay=None, face=1, point=0):
    """Sum of the un-normalised z = C^{-1} t (for the normalisation pin)."""
    _ctx()
    if ay is None:
        ay = ax
    ax, ay = mp.mpf(ax), mp.mpf(ay)
    C = cov_matrix(R, ax, ay)
    g, _ = gauss_rule(nq(R))
    t = t_vector(R, face_point(face, g[point]), ax, ay)
    return mp.fsum(mp.cholesky_solve(C, t))


@functools.lru_cache(maxsize=None)
def _d2_weights_mp(ax, ay, ellx_str):
    _ctx()
    ax, ay = mp.mpf(ax), mp.mpf(ay)
    ell = mp.mpf(ellx_str)
    # physical ell is the same in both directions; Delta_d = ell / a_d
    C = cov_matrix(1, ax, ay)
    st = stencil(1)
    out = []
    for d in range(2):
        t2 = mp.matrix(len(st), 1)
        for m, (di, dj) in enumerate(st):
            sx = mp.mpf(0) - di
            sy = mp.mpf(0) - dj
            if d == 0:
                t2[m] = d2_t_factor(sx, ax, ell) * t_factor(sy, ay)
            else:
                t2[m] = t_factor(sx, ax) * d2_t_factor(sy, ay, ell)
        w = mp.cholesky_solve(C, t2)
        out.append([w[m] for m in range(len(st))])
    return out


def d2_weights(ax, ay, ell, as_float=True):
    """GP-R1 second-derivative weights w[d][m] at the cell centre (App. B), unnormalised.

    ax = ell/dx, ay = ell/dy; ell is the physical length scale (1/ell^2 units).
    """
    w = _d2_weights_mp(str(mp.mpf(ax)), str(mp.mpf(ay)), str(mp.mpf(ell)))
    if as_float:
        return [[float(v) for v in row] for row in w]
    return w


def gauss_rule_float(q):
    g, w = gauss_rule(q)
    return [float(x) for x in g], [float(x) for x in w]
