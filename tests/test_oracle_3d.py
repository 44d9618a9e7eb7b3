"""Pins of the 3D oracle (weights3d_mp.py, gpmood_oracle3d.c) against what the
mathematics fixes: normalisation, exactness on low-degree polynomials in the flat
limit, the symmetries of the L1-ball stencil, HLLC consistency with the 2D form,
free stream, conservation, rotation invariance, measured order 2R+1 and
positivity on the blast."""
import math

import mpmath as mp
import numpy as np
import pytest

import gpmood_inputs as gi
import oracle
from oracle import weights3d_mp as W3
from oracle import weights_mp as W2


def cons3(rho, u, v, w, p, g=1.4):
    return np.array([rho, rho * u, rho * v, rho * w, p / (g - 1) + 0.5 * rho * (u * u + v * v + w * w)])


def test_stencil_is_l1_ball():
    for R, n in ((1, 7), (2, 25)):
        st = W3.stencil3(R)
        assert len(st) == n == len(set(st))
        assert all(abs(a) + abs(b) + abs(c) <= R for a, b, c in st)
        assert st[0] == (0, 0, 0)


@pytest.mark.parametrize("R", [1, 2])
def test_signed_sum_normalisation_3d(R):
    z = W3.weights3(R, 12.0, as_float=False)
    for f in range(6):
        assert len(z[f]) == W2.nq(R) ** 2
        for row in z[f]:
            assert abs(mp.fsum(row) - 1) < mp.mpf(10) ** -60


@pytest.mark.parametrize("R", [1, 2])
def test_polynomial_reproduction_3d(R):
    """Weights, then the face's tensor Gauss rule, applied to exact cell averages of
    x^p y^k z^m reproduce the face average for every degree <= 2R with an error that
    falls like (dx/ell)^2, and miss degree 2R+1 by O(1)."""
    h = mp.mpf(1) / 2
    st = W3.stencil3(R)

    def avg1(c, e):
        return ((c + h) ** (e + 1) - (c - h) ** (e + 1)) / (e + 1)

    def worst(z, deg):
        out = mp.mpf(0)
        nodes = {f: W3.face_nodes3(f, R) for f in range(6)}
        for p in range(deg + 1):
            for k in range(deg + 1 - p):
                m3 = deg - p - k
                ex = (p, k, m3)
                cav = [avg1(a, p) * avg1(b, k) * avg1(c, m3) for a, b, c in st]
                for f in range(6):
                    ax = f // 2
                    s = -h if f % 2 == 0 else h
                    exact = mp.mpf(1)
                    for d in range(3):
                        exact *= s ** ex[d] if d == ax else avg1(mp.mpf(0), ex[d])
                    val = mp.fsum(wq * mp.fsum(z[f][q][mm] * cav[mm] for mm in range(len(st)))
                                  for q, (_, wq) in enumerate(nodes[f]))
                    out = max(out, abs(val - exact))
        return float(out)

    errs = []
    for a in (200, 400):
        z = W3.weights3(R, a, as_float=False)
        errs.append(max(worst(z, d) for d in range(2 * R + 1)))
        assert worst(z, 2 * R + 1) > 0.05
    assert errs[1] < 1e-4
    assert 3.0 < errs[0] / errs[1] < 5.0


@pytest.mark.parametrize("R", [1, 2])
def test_symmetries_3d(R):
    """x- is the mirror of x+, node order mirrors with the tangential coordinates, and the
    faces of the other axes are the x faces with the axes permuted (equal spacing)."""
    z = W3.weights3(R, 12.0)
    st = W3.stencil3(R)
    pos = {o: m for m, o in enumerate(st)}
    nodes = {f: [xs for xs, _ in W3.face_nodes3(f, R)] for f in range(6)}
    node_pos = {f: {tuple(float(c) for c in xs): q for q, xs in enumerate(nodes[f])} for f in range(6)}
    for q, xs in enumerate(nodes[1]):
        x = tuple(float(c) for c in xs)
        for m, (a, b, c) in enumerate(st):
            v = z[1][q][m]
            assert abs(z[0][node_pos[0][(-x[0], x[1], x[2])]][pos[(-a, b, c)]] - v) < 1e-14
            assert abs(z[1][node_pos[1][(x[0], -x[1], x[2])]][pos[(a, -b, c)]] - v) < 1e-14
            # y+ face: axes x <-> y exchanged
            assert abs(z[3][node_pos[3][(x[1], x[0], x[2])]][pos[(b, a, c)]] - v) < 1e-14
            # z+ face: axes x <-> z exchanged
            assert abs(z[5][node_pos[5][(x[2], x[1], x[0])]][pos[(c, b, a)]] - v) < 1e-14


def test_hllc3_consistency_and_2d_agreement():
    g = 1.4
    rng = np.random.default_rng(4)
    for _ in range(20):
        r, u, v, w, p = rng.uniform(0.3, 2.0), *rng.uniform(-1, 1, 3), rng.uniform(0.2, 2.0)
        U = cons3(r, u, v, w, p)
        for d in range(3):
            F = oracle.hllc3(g, U, U, d)
            vel = (u, v, w)
            exact = np.array([r * vel[d], r * vel[d] * u, r * vel[d] * v, r * vel[d] * w, vel[d] * (U[4] + p)])
            exact[1 + d] += p
            np.testing.assert_allclose(F, exact, rtol=1e-13, atol=1e-14)
        # w = 0: the 3D solver on x and y faces is the 2D one
        UL = cons3(r, u, v, 0.0, p)
        UR = cons3(*rng.uniform(0.3, 2.0, 1), *rng.uniform(-1, 1, 2), 0.0, *rng.uniform(0.2, 2.0, 1))
        for d in range(2):
            F3 = oracle.hllc3(g, UL, UR, d)
            F2 = oracle.hllc(UL[[0, 1, 2, 4]], UR[[0, 1, 2, 4]], direction=d, gamma=g)
            np.testing.assert_allclose(F3[[0, 1, 2, 4]], F2, rtol=1e-14, atol=1e-15)
            assert abs(F3[3]) < 1e-15


def test_free_stream_and_conservation_3d():
    n = 8
    U0 = np.broadcast_to(cons3(1.3, 0.7, -0.4, 0.2, 0.9)[:, None, None, None], (5, n, n, n)).copy()
    o = oracle.Oracle3D((n, n, n), bc=(0, 0, 0), cascade=(2, 1, 0))
    U, _, iters, counts = o.run(U0, cfl=0.3, nsteps=2)
    assert np.abs(U - U0).max() < 1e-13
    assert counts[1:].sum() == 0
    # a blast on a periodic box: totals conserved to roundoff with the cascade active
    Ub = gi.blast3d(n, r_cells=2.0, p_in=10.0, p_out=0.1)
    t0 = Ub.reshape(5, -1).sum(axis=1)
    U, _, iters, _ = o.run(Ub, cfl=0.3, nsteps=2)
    assert iters.max() > 1  # the cascade was exercised
    np.testing.assert_allclose(U.reshape(5, -1).sum(axis=1), t0, rtol=1e-13, atol=1e-12)


def test_rotation_invariance_3d():
    """A shock tube along x, along y and along z gives the same solution, permuted."""
    n = 10
    L = cons3(1.0, 0.0, 0.0, 0.0, 1.0)
    R = cons3(0.125, 0.0, 0.0, 0.0, 0.1)
    x = (np.arange(n) + 0.5) / n
    Ux = np.where((x < 0.5)[None, None, None, :], L[:, None, None, None], R[:, None, None, None])
    Ux = np.broadcast_to(Ux, (5, n, n, n)).copy()
    o = oracle.Oracle3D((n, n, n), bc=(1, 1, 1), cascade=(2, 1, 0))
    dt = 0.2 / n
    res = []
    for ax in range(3):
        U = np.moveaxis(Ux, 3, 3 - ax).copy()  # the jump along axis ax (array axis 3 - ax)
        if ax:
            U[[1, 1 + ax]] = U[[1 + ax, 1]]  # momentum follows the axis
        out = o.stage(0, U, U, dt)[0]
        if ax:
            out[[1, 1 + ax]] = out[[1 + ax, 1]]
        res.append(np.moveaxis(out, 3 - ax, 3))
    np.testing.assert_allclose(res[1], res[0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(res[2], res[0], rtol=0, atol=1e-13)


@pytest.mark.slow
@pytest.mark.parametrize("R,eoc", [(1, 2.5), (2, 4.5)])
def test_convergence_order_3d(R, eoc):
    """Diagonal 3D density wave, fixed physical ell = 0.25, dt ~ dx^((2R+1)/3): the L1
    error falls at about order 2R+1."""
    casc = {1: (1, 0), 2: (2, 1, 0)}[R]
    T = 0.03
    errs = []
    ns = (16, 24)
    for n in ns:
        U0 = gi.density_wave3d(n)
        o = oracle.Oracle3D((n, n, n), bc=(0, 0, 0), cascade=casc, ell=0.25)
        dt = 0.2 * (1.0 / n) ** ((2 * R + 1) / 3.0) / 3.0
        nst = int(math.ceil(T / dt))
        U = U0.copy()
        Un = U
        for _ in range(nst):
            Un = U
            U1, _, c1, _ = o.stage(0, Un, Un, T / nst)
            U2, _, c2, _ = o.stage(1, Un, U1, T / nst)
            U, _, c3, _ = o.stage(2, Un, U2, T / nst)
            assert c1[1:].sum() == c2[1:].sum() == c3[1:].sum() == 0
        errs.append(np.abs(U[0] - gi.density_wave3d(n, t=T)[0]).mean())
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    assert rate > eoc, (errs, rate)


def test_blast_positivity_3d():
    n = 12
    U0 = gi.blast3d(n, r_cells=3.0)
    o = oracle.Oracle3D((n, n, n), bc=(1, 1, 1), cascade=(2, 1, 0))
    U, dts, iters, counts = o.run(U0, cfl=0.3, nsteps=2)
    p = 0.4 * (U[4] - 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / U[0])
    assert (U[0] > 0).all() and (p > 0).all()
    assert iters.max() > 1
