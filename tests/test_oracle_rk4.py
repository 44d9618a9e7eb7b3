"""Pins of the oracle's five-stage SSP-RK4 (eqs. (rk4), (rk4_substeps)) with the
MOOD loop in every stage: the general stage reproduces the SSP-RK3 stages, the
time integration converges at 4th order in dt on a fixed grid (which also fixes
the reading of the sign of the U(3) term of the last combination: the printed
sign would not be 4th order), the step conserves totals on a periodic grid, and
the stages sum to a consistent method (a constant state stays constant)."""
import math

import numpy as np

import gpmood_inputs as gi
import oracle


def test_general_stage_reproduces_rk3_stages():
    n = 24
    U0 = gi.quadrants(n, n, seed=3)
    o = oracle.Oracle(n, n, bc=(1, 1), cascade=(3, 2, 1, 0))
    U = o.run(U0, cfl=0.8, nsteps=2)[0]
    dt = o.dt(U, 0.8)
    U1, m1, c1, i1 = o.stage(0, U, U, dt)
    G1, g1, d1, j1 = o.stage_coef(U, U, dt, 0.0, 1.0, 1.0)
    np.testing.assert_array_equal(G1, U1)
    np.testing.assert_array_equal(g1, m1)
    U2, m2, c2, i2 = o.stage(1, U, U1, dt)
    G2, g2, d2, j2 = o.stage_coef(U, U1, dt, 0.75, 0.25, 1.0)
    np.testing.assert_allclose(G2, U2, rtol=1e-15, atol=1e-15)
    np.testing.assert_array_equal(g2, m2)
    assert j1 == i1 and j2 == i2 and i1 + i2 > 2  # the cascade was exercised


def test_rk4_stage_table_is_consistent():
    """Each sub-step's combination weights sum to 1; the last combination's state
    weights (with the dt F(U(3)) term expressed through sub-step 4) sum to 1 - b5."""
    st = oracle.rk4_stages()
    for a, b, cf in st["sub"]:
        assert abs(a + b - 1.0) < 1e-14 and cf > 0
    a5, b5, cf5 = st["last"]
    assert abs(sum(st["w"]) + b5 - 1.0) < 1e-14


def test_rk4_free_stream_and_conservation():
    n = 16
    o = oracle.Oracle(n, n, bc=(0, 0), cascade=(2, 1, 0))
    U0 = gi.quadrants(n, n, seed=2)
    t0 = o.totals(U0)
    U = U0
    for _ in range(2):
        U, iters = o.rk4_step(U, o.dt(U, 0.5))
    np.testing.assert_allclose(o.totals(U), t0, rtol=1e-13, atol=1e-13)
    const = np.broadcast_to(U0[:, :1, :1], U0.shape).copy()
    Uc, _ = o.rk4_step(const, 0.01)
    assert np.abs(Uc - const).max() < 1e-13


def _evolve(o, U0, T, nsteps, rk4=True):
    U = U0
    dt = T / nsteps
    for _ in range(nsteps):
        if rk4:
            U, iters = o.rk4_step(U, dt)
            assert max(iters) == 1  # smooth flow: no cell lowered
        else:
            U1 = o.stage(0, U, U, dt)[0]
            U2 = o.stage(1, U, U1, dt)[0]
            U = o.stage(2, U, U2, dt)[0]
    return U


def test_rk4_temporal_order():
    """Fixed 16^2 grid, GP-MOOD5, smooth density wave, T = 0.2: the difference to
    a dt/8 reference falls by about 2^4 per halving of dt (2^3 for SSP-RK3)."""
    n = 16
    o = oracle.Oracle(n, n, bc=(0, 0), cascade=(2, 1, 0))
    U0 = gi.density_wave(n, n)
    T = 0.2
    ref = _evolve(o, U0, T, 64)
    errs = [np.abs(_evolve(o, U0, T, m)[0] - ref[0]).mean() for m in (8, 16)]
    rate = math.log(errs[0] / errs[1], 2)
    assert 3.6 < rate < 4.6, (errs, rate)
    ref3 = _evolve(o, U0, T, 64, rk4=False)
    errs3 = [np.abs(_evolve(o, U0, T, m, rk4=False)[0] - ref3[0]).mean() for m in (8, 16)]
    rate3 = math.log(errs3[0] / errs3[1], 2)
    assert 2.6 < rate3 < 3.5, (errs3, rate3)
