"""Pins of the oracle's relaxed discrete maximum principle (2D and 3D) on each side of
every threshold the paper fixes:

- eq. (DMP_RK): the bounds are taken over the face neighbours AND the cell itself;
- eq. (plateau): the variation of the neighbourhood against min_d Delta_d^3 (not the
  square, not the largest spacing);
- eq. (u2_a): Cmin Cmax > -delta and max(|Cmax|, |Cmin|) < delta, delta = min_d Delta_d;
- eq. (u2_b): Cmin Cmax > -delta and |Cmin| / |Cmax| >= 1/2 (the ratio of the smallest
  to the largest curvature, not its inverse), required for every direction d.

The neighbourhoods are built by hand: the density is solved for so that the curvature
values kappa_d(m) = w_d . rho(stencil of m) at the cell and its face neighbours take
chosen values (w_d: the App. B second-derivative weights, pinned on their own in
test_oracle_weights.py).  The curvature map has a left null space (in the flat limit the
mixed fourth difference kappa_x(c) - (kappa_x(S) + kappa_x(N))/2 equals
kappa_y(c) - (kappa_y(W) + kappa_y(E))/2), so only the tested direction's values are
chosen freely; every other direction takes a large baseline s, moved by the least
offsets that meet the constraint and kept within a ratio 0.8 of s, which (b) accepts,
so the tested direction decides the verdict.  Each expected verdict is fixed by the chosen values and the
inequality, far from any rounding tie, so a dropped or altered term in the oracle
(delta^2 for delta, 1/4 for 1/2, the inverted ratio, a dropped product condition, a
single direction, the squared plateau threshold, the cell left out of its own bounds)
fails one of these cases.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import weights3d_mp, weights_mp

G = 1.4


def _cons2(rho):
    """Fluid at rest with p = 1 and the given density field (ny, nx)."""
    return np.stack([rho, 0 * rho, 0 * rho, np.full_like(rho, 1.0 / (G - 1))])


def _solve_targets(A, values, groups):
    """Right-hand side for A rho = kappa: kappa starts from `values` (one per row);
    each group of rows in `groups` takes one shared additive offset, the offsets of
    least norm that put kappa in the range of A.  Returns kappa."""
    u, sv, _ = np.linalg.svd(A)
    null = u[:, sv < 1e-9 * sv[0]]
    base = np.asarray(values, dtype=float)
    if not groups:
        return base
    E = np.zeros((A.shape[0], len(groups)))
    for g, rows in enumerate(groups):
        E[rows, g] = 1.0
    t = np.linalg.lstsq(null.T @ E, -null.T @ base, rcond=None)[0]
    return base + E @ t


# ---------------------------------------------------------------- 2D builders
N2 = 9
C2 = N2 // 2
NB2 = [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]


def _solve_kappa_2d(o, kx, ky):
    """Density on an N2 x N2 grid (1 away from the centre's radius-2 diamond) whose
    curvatures at the centre cell and its four face neighbours are kx (d = x) or ky
    (d = y), in the order self, W, E, S, N; the direction given as None takes a
    uniform value."""
    w2 = np.array(weights_mp.d2_weights(o.ell / o.dx, o.ell / o.dy, o.ell))  # [2][5]
    off1 = weights_mp.stencil(1)
    cells = [(di, dj) for dj in range(-2, 3) for di in range(-2, 3) if abs(di) + abs(dj) <= 2]
    col = {c: k for k, c in enumerate(cells)}
    A = np.zeros((10, len(cells)))
    for d in range(2):
        for m, (mi, mj) in enumerate(NB2):
            for e, (oi, oj) in enumerate(off1):
                A[5 * d + m, col[(mi + oi, mj + oj)]] += w2[d, e]
    base = 2.0 + 10.0 * max(abs(v) for k in (kx, ky) if k is not None for v in k)
    values, groups = [], []
    for d, k in enumerate((kx, ky)):
        values += [base] * 5 if k is None else list(k)
        if k is None:
            groups.append([5 * d])  # the cell itself
    rhs = _solve_targets(A, values, groups)
    for d, k in enumerate((kx, ky)):
        if k is None:  # the free direction's own verdict is (b) with ratio >= 0.8
            assert np.all((0.8 * base <= rhs[5 * d:5 * d + 5]) & (rhs[5 * d:5 * d + 5] <= 1.25 * base))
    # rho = 1 + x: the constant field contributes sum(w) to every curvature
    x = np.linalg.lstsq(A, rhs - A.sum(axis=1), rcond=None)[0]
    rho = np.ones((N2, N2))
    for (di, dj), v in zip(cells, x):
        rho[C2 + dj, C2 + di] += v
    # the construction hits its targets (checked on the built field)
    got = A @ (x + 1.0)
    assert np.allclose(got, rhs, rtol=0, atol=1e-12 * (1 + np.abs(rhs).max()))
    assert rho.min() > 0.5
    return rho


def _u2_2d(kx, ky=None, dx=0.1, dy=0.1):
    o = oracle.Oracle(N2, N2, hi=(N2 * dx, N2 * dy), bc=(1, 1), cascade=(1, 0))
    rho = _solve_kappa_2d(o, kx, ky)
    rel = o.relax(_cons2(rho))
    return int(rel[C2, C2, 4])


# delta = min(dx, dy) = 0.1 unless stated; values of kappa in the order self, W, E, S, N
U2_CASES_2D = [
    # only (a) accepts: |C| < delta, ratio 0.11 < 1/2  (delta^2 = 0.01 would reject)
    ((0.09, 0.01, 0.05, 0.05, 0.05), None, 0.1, 0.1, 1),
    # just above delta, ratio < 1/2: neither (a) nor (b)
    ((0.12, 0.01, 0.05, 0.05, 0.05), None, 0.1, 0.1, 0),
    # |C| > delta, ratio 0.45: (b) rejects (a threshold 1/4 would accept)
    ((1.0, 0.45, 0.7, 0.7, 0.7), None, 0.1, 0.1, 0),
    # ratio 0.55: (b) accepts (a threshold 3/4 would reject)
    ((1.0, 0.55, 0.7, 0.7, 0.7), None, 0.1, 0.1, 1),
    # all negative: Cmin = -1, Cmax = -0.45, |Cmin|/|Cmax| = 2.2 accepts; the inverted
    # ratio |Cmax|/|Cmin| = 0.45 would reject (and would accept the 0.45 case above)
    ((-1.0, -0.45, -0.7, -0.7, -0.7), None, 0.1, 0.1, 1),
    # mixed signs: Cmin Cmax = -0.06 > -delta and ratio 0.67: (b) accepts
    # (a product condition "> 0" or "> -delta^2" would reject)
    ((0.3, -0.2, 0.1, 0.1, 0.1), None, 0.1, 0.1, 1),
    # ratio 0.6 but Cmin Cmax = -0.6 < -delta: the product condition rejects
    ((1.0, -0.6, 0.7, 0.7, 0.7), None, 0.1, 0.1, 0),
    # small mixed signs: Cmin Cmax = -0.0045 > -delta, |C| < delta: (a) accepts
    ((0.09, -0.05, 0.0, 0.0, 0.0), None, 0.1, 0.1, 1),
    # x accepts, y has ratio 0.45: the criterion must hold for every direction
    (None, (1.0, 0.45, 0.7, 0.7, 0.7), 0.1, 0.1, 0),
    (None, (1.0, 0.55, 0.7, 0.7, 0.7), 0.1, 0.1, 1),
    # anisotropic: delta = min(0.1, 0.2) = 0.1, so |C| = 0.15 fails (a); max would accept
    ((0.15, 0.01, 0.05, 0.05, 0.05), None, 0.1, 0.2, 0),
    ((0.09, 0.01, 0.05, 0.05, 0.05), None, 0.1, 0.2, 1),
]


@pytest.mark.parametrize("kx,ky,dx,dy,expect", U2_CASES_2D)
def test_u2_thresholds_2d(kx, ky, dx, dy, expect):
    assert _u2_2d(kx, ky, dx, dy) == expect


@pytest.mark.parametrize("dx,dy,var,expect", [
    (0.1, 0.1, 5e-3, 0),   # between dx^3 = 1e-3 and dx^2 = 1e-2: no plateau
    (0.1, 0.1, 5e-4, 1),   # below dx^3
    (0.1, 0.2, 4e-3, 0),   # min(dx^3, dy^3) = 1e-3 < 4e-3 < max = 8e-3
    (0.1, 0.2, 9e-4, 1),
])
def test_plateau_threshold_2d(dx, dy, var, expect):
    o = oracle.Oracle(N2, N2, hi=(N2 * dx, N2 * dy), bc=(1, 1), cascade=(1, 0))
    rho = np.ones((N2, N2))
    rho[C2, C2 + 1] += var  # the neighbourhood's range is exactly var
    rel = o.relax(_cons2(rho))
    assert rel[C2, C2, 1] - rel[C2, C2, 0] == pytest.approx(var, rel=1e-12)
    assert int(rel[C2, C2, 2]) == expect


def test_dmp_bounds_include_the_cell_2d():
    """eq. (DMP_RK): min and max over N(ij) and the cell ij itself."""
    o = oracle.Oracle(N2, N2, hi=(0.9, 0.9), bc=(1, 1), cascade=(1, 0))
    rho = np.ones((N2, N2))
    rho[C2, C2 + 1] = 2.0
    rho[C2, C2] = 3.0              # the cell is the neighbourhood's maximum
    rel = o.relax(_cons2(rho))
    assert rel[C2, C2, 0] == 1.0 and rel[C2, C2, 1] == 3.0
    rho[C2, C2] = 0.5              # and here its minimum
    rel = o.relax(_cons2(rho))
    assert rel[C2, C2, 0] == 0.5 and rel[C2, C2, 1] == 2.0


def test_dmp_decided_by_the_cell_itself_2d():
    """A candidate inside [min, max] only because the cell's own value is included is
    accepted, with CSD, plateau and u2 unable to accept it."""
    n, c = N2, C2
    x = (np.arange(n) - c) * 1.0
    u = np.broadcast_to(-20.0 * x[None, :], (n, n))   # strong compression: CSD rejects
    rho = np.ones((n, n))
    rho[c, c + 1] = 2.0
    rho[c, c] = 3.0
    Us = np.stack([rho, rho * u, 0 * rho, 1.0 / (G - 1) + 0.5 * rho * u * u])
    Ustar = Us.copy()
    Ustar[0, c, c] = 2.5           # in [1, 3] but above every neighbour
    o = oracle.Oracle(n, n, hi=(0.1 * n, 0.1 * n), bc=(1, 1),
                      flags=oracle.ORC_ALL & ~oracle.ORC_U2 & ~oracle.ORC_PLATEAU)
    bits, tr = o.criteria(Us, Ustar, np.full((n, n), 3, np.int32))
    assert not bits[c, c] & 8      # CSD rejects
    assert bits[c, c] & 32 and tr[c, c] == 0
    Ustar[0, c, c] = 3.5           # above the cell too
    bits, tr = o.criteria(Us, Ustar, np.full((n, n), 3, np.int32))
    assert not bits[c, c] & 32 and tr[c, c] == 1


# ---------------------------------------------------------------- 3D builders
N3 = 7
C3 = N3 // 2
NB3 = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def _cons3(rho):
    z = 0 * rho
    return np.stack([rho, z, z, z, np.full_like(rho, 1.0 / (G - 1))])


def _solve_kappa_3d(o, kap):
    """Density on an N3^3 grid whose curvatures kap[d][m] (d = x, y, z; m over the
    cell and its six face neighbours in the order self, -x, +x, -y, +y, -z, +z); a
    direction given as None takes a uniform value."""
    ell = o.ell
    w2 = np.array(weights3d_mp.d2_weights3(ell / o.d[0], ell / o.d[1], ell / o.d[2], ell))  # [3][7]
    off1 = weights3d_mp.stencil3(1)
    cells = [c for c in itertools.product(range(-2, 3), repeat=3) if sum(map(abs, c)) <= 2]
    col = {c: k for k, c in enumerate(cells)}
    A = np.zeros((21, len(cells)))
    for d in range(3):
        for m, nb in enumerate(NB3):
            for e, oo in enumerate(off1):
                A[7 * d + m, col[tuple(nb[t] + oo[t] for t in range(3))]] += w2[d, e]
    base = 2.0 + 10.0 * max(abs(v) for k in kap if k is not None for v in k)
    values, groups = [], []
    for d in range(3):
        values += [base] * 7 if kap[d] is None else list(kap[d])
        if kap[d] is None:
            groups.append([7 * d])  # the cell itself, and each pair across another axis
            for e in range(3):
                if e != d:
                    groups.append([7 * d + 1 + 2 * e, 7 * d + 2 + 2 * e])
    rhs = _solve_targets(A, values, groups)
    for d in range(3):
        if kap[d] is None:
            assert np.all((0.8 * base <= rhs[7 * d:7 * d + 7]) & (rhs[7 * d:7 * d + 7] <= 1.25 * base))
    x = np.linalg.lstsq(A, rhs - A.sum(axis=1), rcond=None)[0]
    rho = np.ones((N3, N3, N3))
    for (di, dj, dk), v in zip(cells, x):
        rho[C3 + dk, C3 + dj, C3 + di] += v
    got = A @ (x + 1.0)
    assert np.allclose(got, rhs, rtol=0, atol=1e-12 * (1 + np.abs(rhs).max()))
    assert rho.min() > 0.5
    return rho


def _u2_3d(kap, d=(0.1, 0.1, 0.1)):
    o = oracle.Oracle3D((N3, N3, N3), hi=tuple(N3 * x for x in d), bc=(1, 1, 1), cascade=(1, 0))
    rho = _solve_kappa_3d(o, kap)
    return int(o.relax(_cons3(rho))[C3, C3, C3, 4])


Z7 = None
U2_CASES_3D = [
    (((0.09, 0.01, 0.05, 0.05, 0.05, 0.05, 0.05), Z7, Z7), (0.1, 0.1, 0.1), 1),
    (((0.12, 0.01, 0.05, 0.05, 0.05, 0.05, 0.05), Z7, Z7), (0.1, 0.1, 0.1), 0),
    (((1.0, 0.45, 0.7, 0.7, 0.7, 0.7, 0.7), Z7, Z7), (0.1, 0.1, 0.1), 0),
    (((1.0, 0.55, 0.7, 0.7, 0.7, 0.7, 0.7), Z7, Z7), (0.1, 0.1, 0.1), 1),
    (((-1.0, -0.45, -0.7, -0.7, -0.7, -0.7, -0.7), Z7, Z7), (0.1, 0.1, 0.1), 1),
    (((0.3, -0.2, 0.1, 0.1, 0.1, 0.1, 0.1), Z7, Z7), (0.1, 0.1, 0.1), 1),
    (((1.0, -0.6, 0.7, 0.7, 0.7, 0.7, 0.7), Z7, Z7), (0.1, 0.1, 0.1), 0),
    ((Z7, Z7, (1.0, 0.45, 0.7, 0.7, 0.7, 0.7, 0.7)), (0.1, 0.1, 0.1), 0),   # the z direction decides
    ((Z7, (1.0, 0.55, 0.7, 0.7, 0.7, 0.7, 0.7), Z7), (0.1, 0.1, 0.1), 1),
    # delta = min spacing: 0.15 fails with spacings (0.2, 0.1, 0.2)
    (((0.15, 0.01, 0.05, 0.05, 0.05, 0.05, 0.05), Z7, Z7), (0.2, 0.1, 0.2), 0),
]


@pytest.mark.parametrize("kap,d,expect", U2_CASES_3D)
def test_u2_thresholds_3d(kap, d, expect):
    assert _u2_3d(kap, d) == expect


@pytest.mark.parametrize("d,var,expect", [
    ((0.1, 0.1, 0.1), 5e-3, 0),
    ((0.1, 0.1, 0.1), 5e-4, 1),
    ((0.2, 0.1, 0.2), 4e-3, 0),    # min of the cubes 1e-3 < 4e-3 < max 8e-3
    ((0.2, 0.1, 0.2), 9e-4, 1),
])
def test_plateau_threshold_3d(d, var, expect):
    o = oracle.Oracle3D((N3, N3, N3), hi=tuple(N3 * x for x in d), bc=(1, 1, 1), cascade=(1, 0))
    rho = np.ones((N3, N3, N3))
    rho[C3 + 1, C3, C3] += var     # the +z neighbour
    rel = o.relax(_cons3(rho))
    assert rel[C3, C3, C3, 1] - rel[C3, C3, C3, 0] == pytest.approx(var, rel=1e-12)
    assert int(rel[C3, C3, C3, 2]) == expect


def test_dmp_bounds_include_the_cell_3d():
    o = oracle.Oracle3D((N3, N3, N3), bc=(1, 1, 1), cascade=(1, 0))
    rho = np.ones((N3, N3, N3))
    rho[C3 - 1, C3, C3] = 2.0
    rho[C3, C3, C3] = 3.0
    rel = o.relax(_cons3(rho))
    assert rel[C3, C3, C3, 0] == 1.0 and rel[C3, C3, C3, 1] == 3.0
    rho[C3, C3, C3] = 0.5
    rel = o.relax(_cons3(rho))
    assert rel[C3, C3, C3, 0] == 0.5 and rel[C3, C3, C3, 1] == 2.0
