"""Pins of the oracle's inflow slit (the injection boundary of the paper's Mach-jet
problems, Sec. "Numerical results"): the ghost cells under the slit hold the jet
state, every other boundary cell is an outflow copy.  On the ambient state at rest
one first-order stage changes only the cells above the slit, by exactly the jet's
HLL flux through the slit faces; the slit sits on the cells whose centres lie in
it; the step size takes the injected state's speed."""
import numpy as np
import pytest

import gpmood_inputs as gi
import oracle

G = 1.4


def jet(n, **kw):
    return oracle.Oracle(n, n, hi=(1.5, 1.5), bc=(1, 1), solver="hll", slit=gi.MACH_JET_SLIT, **kw)


def test_slit_cells_and_the_injected_flux():
    n = 150  # dx = 0.01: slit cells 70..79 (centres 0.705 .. 0.795)
    o = jet(n, cascade=(0,))
    assert (o.cfg.slit, o.cfg.slit_i0, o.cfg.slit_i1) == (1, 70, 80)
    U0 = gi.mach_jet(n)
    dt = 1e-5
    U1, _, _, _ = o.stage(0, U0, U0, dt)
    d = U1 - U0
    # only the bottom row above the slit changes
    changed = np.argwhere(np.abs(d).max(axis=0) > 0)
    assert set(map(tuple, changed)) == {(0, i) for i in range(70, 80)}
    # by dt / dy times the HLL flux of (jet | ambient) through the slit face less the
    # ambient's own flux (0, 0, p, 0) through the cell's top face
    r, u, v, p = gi.MACH_JET_SLIT[3]
    UL = np.array([r, r * u, r * v, p / (G - 1) + 0.5 * r * (u * u + v * v)])
    UR = U0[:, 0, 75]
    F = oracle.hll(UL, UR, 1)
    np.testing.assert_allclose(d[:, 0, 75], dt / o.dy * (F - np.array([0.0, 0.0, 1.0, 0.0])), rtol=1e-12, atol=1e-14)
    assert F[0] > 0 and F[2] > 0  # mass and y momentum flow in


def test_jet_run_stays_positive_with_the_cascade_at_work():
    n = 60
    o = jet(n)
    U, _, counts, _ = o.run(gi.mach_jet(n), cfl=0.8, nsteps=20)
    p = (G - 1) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / U[0])
    assert np.all(np.isfinite(U)) and np.all(U[0] > 0) and np.all(p > 0)
    assert counts[:, :, 1:].sum() > 0
    assert U[2].max() > 1.0  # the jet has entered


def test_jet_stays_mirror_symmetric():
    # the problem is symmetric about x = 0.75; the oracle keeps it to its own
    # summation-order rounding (an inadmissible Riemann state troubles both cells of
    # its face, so no decision depends on which side it is on)
    n = 60
    U, _, counts, _ = jet(n).run(gi.mach_jet(n), cfl=0.8, nsteps=10)
    assert counts[:, :, 1:].sum() > 0
    scale = np.abs(U).max(axis=(1, 2))
    for v, sgn in ((0, 1), (1, -1), (2, 1), (3, 1)):
        assert np.abs(U[v] - sgn * U[v][:, ::-1]).max() <= 1e-12 * scale[v]


def test_step_size_includes_the_jet():
    # at t = 0 the jet is only in the ghost cells; the CFL step still takes its
    # speed |v| + c = 101 (c = 1), not the ambient's
    n = 60
    o = jet(n)
    dt = o.dt(gi.mach_jet(n), 0.8)
    assert abs(dt - 0.8 * (1.5 / n) / 101.0) <= 1e-15


def test_slit_needs_outflow_y_boundaries():
    with pytest.raises(ValueError):
        oracle.Oracle(16, 16, bc=(1, 0), slit=(1, 0.4, 0.6, (1.0, 0.0, 1.0, 1.0)))


def test_top_slit_is_the_bottom_slit_upside_down():
    # a top-only slit injecting downward into the uniform ambient is the bottom
    # jet flipped about y = 0.75 with v reversed
    n = 40
    r, u, v, p = gi.MACH_JET_SLIT[3]
    top = oracle.Oracle(n, n, hi=(1.5, 1.5), bc=(1, 1), solver="hll",
                        slit=(2, 0.7, 0.8, (r, u, v, p), (r, u, -v, p)))
    U0 = gi.mach_jet(n)
    Ub, _, cb, _ = jet(n).run(U0, cfl=0.8, nsteps=6)
    Ut, _, ct, _ = top.run(U0, cfl=0.8, nsteps=6)
    flip = np.array([1.0, 1.0, -1.0, 1.0])[:, None, None] * Ut[:, ::-1, :]
    scale = np.abs(Ub).max(axis=(1, 2))
    assert np.abs(flip - Ub).max(axis=(1, 2)).max() <= 1e-12 * scale.max()
    assert np.array_equal(cb, ct)


def test_double_jet_two_states():
    n = 60
    o = oracle.Oracle(n, n, hi=(1.5, 1.5), bc=(1, 1), solver="hll", slit=gi.DOUBLE_JET_SLIT)
    U0 = gi.double_jet(n)
    assert abs(o.dt(U0, 0.8) - 0.8 * (1.5 / n) / 801.0) <= 1e-15
    U, _, counts, _ = o.run(U0, cfl=0.8, nsteps=10)
    assert U[2, :3].max() > 1.0 and U[2, -3:].min() < -1.0  # both jets entered, opposite ways
    assert np.all(np.isfinite(U)) and np.all(U[0] > 0)
