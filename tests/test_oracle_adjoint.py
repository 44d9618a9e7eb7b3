"""Pins of the oracle's derivatives of a stage with the per-cell orders and dt held
fixed (the forced-order stage, stage_forced):

- the forward-mode derivative (stage_jvp) against central finite differences of the
  stage itself, on shock states where the cascade has lowered cells, with periodic,
  outflow and reflecting boundaries and both Riemann solvers;
- the reverse sweep (stage_vjp) against the forward-mode derivative through the
  dot-product identity <lam, J v> = <J^T lam, v>, to rounding.

Together they fix the adjoint the GPU path is compared with: a transposition error
(a dropped boundary face, a sign, a wrong stencil cell or weight side) breaks the
identity, and a wrong derivative breaks the finite differences."""
import numpy as np
import pytest

import gpmood_inputs as gi
import oracle


def _setup(n, bc, cascade, seed, solver="hllc", steps=2):
    o = oracle.Oracle(n, n, bc=bc, cascade=cascade, solver=solver)
    U = gi.quadrants(n, n, seed=seed)
    if bc == (2, 2):
        U = gi.implosion(n)
    U = o.run(U, cfl=0.8, nsteps=steps)[0]
    dt = o.dt(U, 0.8)
    U1, order0, _, _ = o.stage(0, U, U, dt)
    U2, order1, _, _ = o.stage(1, U, U1, dt)
    return o, U, U1, dt, order0, order1


CASES = [(24, (1, 1), (3, 2, 1, 0), 1, "hllc"), (20, (0, 0), (3, 1, 0), 2, "hllc"),
         (20, (1, 0), (2, 1, 0), 3, "hll"), (16, (2, 2), (3, 1, 0), 0, "hllc")]


@pytest.mark.parametrize("n,bc,cascade,seed,solver", CASES)
def test_jvp_matches_central_differences(n, bc, cascade, seed, solver):
    o, U, U1, dt, order0, order1 = _setup(n, bc, cascade, seed, solver)
    assert (order1 < cascade[0]).any() or bc == (2, 2)  # mixed orders somewhere
    rng = np.random.default_rng(seed)
    for s, Us, order in ((0, U, order0), (1, U1, order1), (2, U1, order1)):
        v = rng.standard_normal(U.shape) * np.abs(U).mean(axis=(1, 2), keepdims=True)
        w = rng.standard_normal(U.shape) * np.abs(U).mean(axis=(1, 2), keepdims=True)
        Jv = o.stage_jvp(s, Us, v, w, dt, order)
        h = 1e-7  # truncation ~h^2, rounding ~1e-16/h: both near 1e-9 here
        plus = o.stage_forced(s, U + h * w, Us + h * v, dt, order) if s else o.stage_forced(0, Us + h * v, Us + h * v, dt, order)
        minus = o.stage_forced(s, U - h * w, Us - h * v, dt, order) if s else o.stage_forced(0, Us - h * v, Us - h * v, dt, order)
        fd = (plus - minus) / (2 * h)
        err = np.abs(fd - Jv).max(axis=(1, 2)) / np.abs(fd).max(axis=(1, 2))
        assert np.all(err < 1e-6), (s, err)


@pytest.mark.parametrize("n,bc,cascade,seed,solver", CASES)
def test_vjp_is_the_transpose_of_jvp(n, bc, cascade, seed, solver):
    o, U, U1, dt, order0, order1 = _setup(n, bc, cascade, seed, solver)
    rng = np.random.default_rng(100 + seed)
    for s, Us, order in ((0, U, order0), (1, U1, order1), (2, U1, order1)):
        v = rng.standard_normal(U.shape)
        w = rng.standard_normal(U.shape)
        lam = rng.standard_normal(U.shape)
        Jv = o.stage_jvp(s, Us, v, w, dt, order)
        lus, lun = o.stage_vjp(s, Us, dt, order, lam)
        lhs = float((lam * Jv).sum())
        rhs = float((lus * v).sum()) + (float((lun * w).sum()) if s else 0.0)
        scale = float(np.abs(lam * Jv).sum())
        assert abs(lhs - rhs) <= 1e-13 * scale, (s, lhs, rhs)
