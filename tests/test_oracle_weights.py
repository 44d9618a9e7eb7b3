"""Pins of the oracle's GP weights (oracle/weights_mp.py) against what the paper and
the mathematics fix: App. A geometry tables, the closed forms of eqs. (SE-pred) and
(SE-cov) against brute-force integration of the SE kernel, the POL-MOOD3 flat limit,
polynomial reproduction, mirror symmetries, and App. B's second derivative."""
import math
import os

import mpmath as mp
import numpy as np
import pytest

from oracle import weights_mp as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_sections(path):
    sec, out = None, {}
    for line in open(path):
        line = line.split("#")[0].strip()
        if not line:
            continue
        if line.startswith("["):
            sec = line.strip("[]")
            out[sec] = []
        else:
            out[sec].append(line.split())
    return out


def _val(tok, s):
    return float(eval(tok.replace("s", repr(s))))


def test_stencil_sizes_and_shape():
    # Sec. "The GP stencil": 5 / 13 / 25 cells; cross stencils 5 / 9 / 13
    for R, n, nc in ((1, 5, 5), (2, 13, 9), (3, 25, 13)):
        st = W.stencil(R)
        assert len(st) == n and len(set(st)) == n
        assert all(abs(a) + abs(b) <= R for a, b in st)
        assert len(W.stencil(R, "cross")) == nc
    # App. A order for R = 1: centre, left, top, right, bottom
    assert W.stencil(1) == [(0, 0), (-1, 0), (0, 1), (1, 0), (0, -1)]


def test_appendix_a_delta_tables():
    sec = _read_sections(os.path.join(GOLD, "appA_delta_tables.txt"))
    s = 1.0 / (2.0 * math.sqrt(3.0))
    g, _ = W.gauss_rule(2)
    tx, ty = W.delta_table(1, W.face_point(1, g[0]))
    for name, tab in (("x", tx), ("y", ty)):
        gold = np.array([[_val(t, s) for t in row] for row in sec[name]])
        mine = np.array([[float(v) for v in row] for row in tab])
        np.testing.assert_allclose(mine, gold, atol=1e-15)


def test_quadrature_table_exact_on_polynomials():
    # tab:QR-pt-weight: q-point rules of order 2q on [-1/2, 1/2]
    for q in (1, 2, 3, 4):
        g, w = W.gauss_rule(q)
        assert abs(mp.fsum(w) - 1) < mp.mpf(10) ** -70
        for k in range(2 * q):
            exact = mp.mpf(0) if k % 2 else (mp.mpf(1) / 2) ** k / (k + 1)
            assert abs(mp.fsum(wi * gi ** k for gi, wi in zip(g, w)) - exact) < mp.mpf(10) ** -60


@pytest.mark.parametrize("a", [1.5, 2.0, 6.0])
def test_closed_forms_match_kernel_integrals(a):
    """eq. (SE-pred) and eq. (SE-cov) against direct integration of exp(-r^2/(2 ell^2))."""
    mp.mp.dps = 30
    a = mp.mpf(a)
    K = lambda x, y: mp.exp(-(x - y) ** 2 / (2 * a * a))
    for s in (mp.mpf("0.5"), mp.mpf("-1.2886751345948129"), mp.mpf(2)):
        num = mp.quad(lambda x: K(s, x), [-0.5, 0.5])
        assert abs(W.t_factor(s, a) - num) < mp.mpf(10) ** -20
    for D in (0, 1, 3):
        num = mp.quad(lambda x, y: K(x, y + D), [-0.5, 0.5], [-0.5, 0.5])
        assert abs(W.c_factor(mp.mpf(D), a) - num) < mp.mpf(10) ** -20
    W._ctx()


def test_poly3_flat_limit():
    """GP-R1 weights at g1, g2 tend to the POL-MOOD3 values as ell/dx grows, like (dx/ell)^2."""
    r = 1.0 / (4.0 * math.sqrt(3.0))
    gold = {}
    for line in open(os.path.join(GOLD, "poly3_weights.txt")):
        line = line.split("#")[0].strip()
        if line.startswith("g"):
            k, vals = line.split(":")
            gold[k] = np.array([float(eval(v.replace("r", repr(r)))) for v in vals.split()])
    devs = []
    for a in (100.0, 1000.0):
        z = np.array(W.weights(1, a))
        d1 = np.abs(z[1][0] - gold["g1"]).max()
        d2 = np.abs(z[1][1] - gold["g2"]).max()
        devs.append(max(d1, d2))
    assert devs[1] < 1e-6
    assert 80 < devs[0] / devs[1] < 120


def test_poly3_from_appendix_c_coefficients():
    """The printed point values follow from App. C's coefficients at (1/2, +-1/(2 sqrt 3))."""
    r = 1.0 / (4.0 * math.sqrt(3.0))
    rows = {}
    for line in open(os.path.join(GOLD, "poly3_weights.txt")):
        line = line.split("#")[0].strip()
        if line:
            k, vals = line.split(":")
            rows[k] = np.array([float(eval(v.replace("r", repr(r)))) for v in vals.split()])
    for key, y in (("g1", 1 / (2 * math.sqrt(3))), ("g2", -1 / (2 * math.sqrt(3)))):
        x = 0.5
        val = rows["a0"] + rows["a1"] * x + rows["a2"] * x * x + rows["a3"] * y + rows["a4"] * y * y
        np.testing.assert_allclose(val, rows[key], atol=1e-15)


@pytest.mark.parametrize("R", [1, 2, 3])
def test_signed_sum_normalisation(R):
    """eq. (normalized_z): z^T 1 = 1 after normalisation; the raw sum is already close to 1,
    while the L1 norm is far from 1 (negative weights), so the signed sum is the reading
    that meets the stated purpose."""
    raw = float(W.raw_weight_sum(R, 12.0))
    assert abs(raw - 1.0) < 1e-5
    z = W.weights(R, 12.0, as_float=False)
    for f in range(4):
        for row in z[f]:
            assert abs(mp.fsum(row) - 1) < mp.mpf(10) ** -60
            assert mp.fsum(abs(v) for v in row) > 1.1


@pytest.mark.parametrize("R", [1, 2, 3])
def test_polynomial_reproduction(R):
    """Applied to exact cell averages of x^p y^k, the weights followed by the face's
    Gauss rule reproduce the face average of every monomial of degree <= 2R, with an
    error that falls like (dx/ell)^2, and miss degree 2R+1 by O(1): the face flux
    input is (2R+1)th order (Sec. "The (2R+1)th-order GP reconstruction")."""
    g, w = W.gauss_rule(W.nq(R))
    st = W.stencil(R)
    h = mp.mpf(1) / 2

    def cellavg(di, dj, p, k):
        ix = ((di + h) ** (p + 1) - (di - h) ** (p + 1)) / (p + 1)
        iy = ((dj + h) ** (k + 1) - (dj - h) ** (k + 1)) / (k + 1)
        return ix * iy

    def faceavg(f, p, k):
        tang = lambda e: (h ** (e + 1) - (-h) ** (e + 1)) / (e + 1)
        if f < 2:
            return (-h if f == 0 else h) ** p * tang(k)
        return (-h if f == 2 else h) ** k * tang(p)

    def worst(z, deg):
        out = mp.mpf(0)
        for p in range(deg + 1):
            k = deg - p
            for f in range(4):
                val = mp.fsum(w[kk] * mp.fsum(z[f][kk][m] * cellavg(di, dj, p, k)
                                              for m, (di, dj) in enumerate(st)) for kk in range(len(g)))
                out = max(out, abs(val - faceavg(f, p, k)))
        return float(out)

    errs = []
    for a in (200, 400):
        z = W.weights(R, a, as_float=False)
        errs.append(max(worst(z, d) for d in range(2 * R + 1)))
        assert worst(z, 2 * R + 1) > 0.1
    assert errs[1] < 1e-4
    assert 3.0 < errs[0] / errs[1] < 5.0


@pytest.mark.parametrize("R", [1, 2, 3])
def test_mirror_symmetries(R):
    """Faces and nodes are mirror images: z_{x-}(di,dj) = z_{x+}(-di,dj), node -g is the
    mirror of +g, and y faces are x faces with the axes exchanged (dx = dy)."""
    z = W.weights(R, 12.0)
    st = W.stencil(R)
    pos = {o: m for m, o in enumerate(st)}
    g, _ = W.gauss_rule(W.nq(R))
    q = len(g)
    for k in range(q):
        kk = q - 1 - k  # node -g_k
        for m, (di, dj) in enumerate(st):
            v = z[1][k][m]
            assert abs(z[0][k][pos[(-di, dj)]] - v) < 1e-14
            assert abs(z[1][kk][pos[(di, -dj)]] - v) < 1e-14
            assert abs(z[3][k][pos[(dj, di)]] - v) < 1e-14
            assert abs(z[2][k][pos[(dj, -di)]] - v) < 1e-14


def test_second_derivative_weights():
    """App. B: the formula equals a numerical second derivative of eq. (SE-pred) in the
    physical coordinate, and in the flat limit the weights map averages of x^2 to 2."""
    mp.mp.dps = 40
    a, ell = mp.mpf(3), mp.mpf("0.7")
    dx = ell / a
    for s0 in (mp.mpf(0), mp.mpf(1), mp.mpf(-1)):
        f = lambda x: W.t_factor((x - 0) / dx - s0, a)
        num = mp.diff(f, 0, 2)
        assert abs(num - W.d2_t_factor(-s0, a, ell)) < mp.mpf(10) ** -20
    W._ctx()
    # flat limit: weights (with ell = a * dx, dx = 1) applied to cell averages of x^2 and y^2
    st = W.stencil(1)
    for A in (200.0,):
        w = W.d2_weights(A, A, A)  # dx = 1
        avg_x2 = [di * di + 1.0 / 12.0 for di, dj in st]
        avg_y2 = [dj * dj + 1.0 / 12.0 for di, dj in st]
        assert abs(sum(wm * v for wm, v in zip(w[0], avg_x2)) - 2.0) < 1e-3
        assert abs(sum(wm * v for wm, v in zip(w[0], avg_y2))) < 1e-3
        assert abs(sum(wm * v for wm, v in zip(w[1], avg_y2)) - 2.0) < 1e-3
        assert abs(sum(w[0])) < 1e-3 and abs(sum(w[1])) < 1e-3


def test_poly3_closed_form_weights():
    """The oracle's POL-MOOD3 weights (eqs. (poly3), (p3_coeffs)) equal the printed
    x+ face values, are the mirror images on the other faces, sum to 1, and are the
    flat-kernel limit of the GP-R1 weights on every face."""
    r = 1.0 / (4.0 * math.sqrt(3.0))
    gold = {}
    for line in open(os.path.join(GOLD, "poly3_weights.txt")):
        line = line.split("#")[0].strip()
        if line.startswith("g"):
            k, vals = line.split(":")
            gold[k] = np.array([float(eval(v.replace("r", repr(r)))) for v in vals.split()])
    P = np.array(W.poly3_weights())
    g, _ = W.gauss_rule(2)
    first_is_plus = float(g[0]) > 0
    np.testing.assert_allclose(P[1][0], gold["g1"] if first_is_plus else gold["g2"], atol=1e-15)
    np.testing.assert_allclose(P[1][1], gold["g2"] if first_is_plus else gold["g1"], atol=1e-15)
    np.testing.assert_allclose(P.sum(axis=2), 1.0, atol=1e-15)
    flat = np.array(W.weights(1, 3000.0))
    assert np.abs(flat - P).max() < 1e-6


def test_cross_stencils():
    """Cross-shaped stencils (Sec. "Isentropic vortex"): 5 / 9 / 13 cells on the
    axes; radius 1 equals the diamond; weights normalised; in the flat limit the
    radius-2 cross reproduces the face average of x^k on its axis (k <= 4) but not
    of the mixed monomial x y, which the diamond reproduces."""
    for R, n in ((1, 5), (2, 9), (3, 13)):
        st = W.stencil(R, "cross")
        assert len(st) == n and all(a == 0 or b == 0 for a, b in st)
    np.testing.assert_allclose(np.array(W.weights(1, 12.0, shape="cross")), np.array(W.weights(1, 12.0)),
                               rtol=0, atol=0)
    zc = np.array(W.weights(2, 12.0, shape="cross"))
    np.testing.assert_allclose(zc.sum(axis=2), 1.0, atol=1e-13)
    # flat limit: cell averages of x^k on the x+ face at its Gauss nodes
    a = 400.0
    for shape, mixed_ok in (("cross", False), ("diamond", True)):
        st = W.stencil(2, shape)
        z = np.array(W.weights(2, a, shape=shape))
        g, _ = W.gauss_rule(3)

        def avg(c, k):
            return ((c + 0.5) ** (k + 1) - (c - 0.5) ** (k + 1)) / (k + 1)
        for k in range(5):
            cav = np.array([avg(di, k) * avg(dj, 0) for di, dj in st])
            for q in range(3):
                assert abs(z[1][q] @ cav - 0.5 ** k) < 1e-3
        cav = np.array([avg(di, 1) * avg(dj, 1) for di, dj in st])
        errs = [abs(z[1][q] @ cav - 0.5 * float(g[q])) for q in range(3)]
        assert (max(errs) < 1e-3) == mixed_ok
