"""GPU parity with reflecting walls (bc = 2, the four walls of Sec. "The implosion
problem in 2D"): the HIP path through the C ABI against the FP64 oracle.

Each RK stage is replayed on the oracle's own inputs (relative L1 <= 1e-12 per field,
identical masks, per-level counts and evaluations) on grids that span several strips
with ragged tails, walls on one or both axes, and axes of the minimum 4 cells.  The
implosion runs with the paper's contrast against the oracle and keeps its diagonal
symmetry; a closed box conserves mass and energy at a size past the oracle's reach.
"""
import sys

import numpy as np
import pytest

import gpmood_inputs as gi
import oracle
from tests.parity_util import assert_fields_close

pytestmark = pytest.mark.gpu


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gp(*a, **k):
    from paper_2110_08683_amd import GPMood
    return GPMood(*a, **k)


def _rel_l1(a, b):
    return np.array([np.abs(a[v] - b[v]).sum() / max(np.abs(b[v]).sum(), 1e-300) for v in range(4)])


def _input(kind, nx, ny, hi):
    if kind == "implosion":
        return gi.implosion(nx)
    return gi.quadrants(nx, ny, seed=int(kind[1:]), hi=hi)


@pytest.mark.parametrize("nx,ny,kind,bc,cascade,hi,pre", [
    (96, 64, "q1", (2, 2), (3, 2, 1, 0), (1.0, 1.0), 2),
    (70, 50, "q5", (2, 1), (2, 1, 0), (1.0, 1.0), 2),
    (64, 64, "implosion", (2, 2), (3, 2, 1, 0), (0.3, 0.3), 1),
    (64, 64, "implosion", (2, 2), (3, 2, 1, 0), (0.3, 0.3), 0),
    (5, 66, "q8", (2, 2), (3, 2, 1, 0), (1.0, 1.0), 2),
    (66, 4, "q3", (0, 2), (3, 2, 1, 0), (1.0, 1.0), 2),
    (130, 127, "q2", (2, 0), (3, 2, 1, 0), (1.0, 1.0), 2),
])
def test_reflect_stage_replay_fp64(torch_cuda, nx, ny, kind, bc, cascade, hi, pre):
    torch = torch_cuda
    _note(f"reflect replay {nx}x{ny} {kind} bc={bc} cascade={cascade} after {pre} steps")
    U0 = _input(kind, nx, ny, hi)
    o = oracle.Oracle(nx, ny, hi=hi, bc=bc, cascade=cascade)
    g = _gp(nx, ny, hi=hi, bc=bc, prec="f64", cascade=cascade)
    U = o.run(U0, cfl=0.8, nsteps=pre)[0] if pre else U0
    dt = o.dt(U, 0.8)
    U1 = o.stage(0, U, U, dt)[0]
    U2 = o.stage(1, U, U1, dt)[0]
    dev = torch.device("cuda")
    exercised = 0
    for s, Us in ((0, U), (1, U1), (2, U2)):
        tn, ts = torch.from_numpy(U).to(dev), torch.from_numpy(Us).to(dev)
        tout = torch.empty_like(ts)
        g.gpm_set_dt(dt)
        g.gpm_stage_dev(s, tn, ts, tout)
        torch.cuda.synchronize()
        Ug = tout.cpu().numpy()
        mask = g.gpm_get_order_mask().astype(np.int32)
        counts, iters = g.gpm_troubled_counts()
        Uo, order, ocounts, oiters = o.stage(s, U, Us, dt)
        assert np.array_equal(mask, order), (s, int((mask != order).sum()))
        np.testing.assert_array_equal(counts[:len(cascade)], ocounts)
        assert iters == oiters
        err = _rel_l1(Ug, Uo)
        assert np.all(err <= 1e-12), (s, err)
        assert_fields_close(Ug, Uo, what=f"stage {s}")
        exercised += int(ocounts[1:].sum())
    assert exercised > 0


def test_implosion_steps_fp64(torch_cuda):
    """The paper's implosion contrast at 128^2, 20 GPU steps at CFL 0.8: close to the
    oracle's run and symmetric under x <-> y (momenta exchanged)."""
    n = 128
    _note("implosion 128 f64 20 steps")
    U0 = gi.implosion(n)
    g = _gp(n, n, hi=(0.3, 0.3), bc=(2, 2), prec="f64")
    g.gpm_init_state(U0)
    g.gpm_step(0.8, 20)
    U = g.gpm_get_state()
    Uo = oracle.Oracle(n, n, hi=(0.3, 0.3), bc=(2, 2)).run(U0, cfl=0.8, nsteps=20)[0]
    err = _rel_l1(U, Uo)
    assert np.all(err < 1e-9), err
    scale = np.abs(U).max(axis=(1, 2))
    assert np.abs(U[0] - U[0].T).max() <= 1e-12 * scale[0]
    assert np.abs(U[3] - U[3].T).max() <= 1e-12 * scale[3]
    assert np.abs(U[1] - U[2].T).max() <= 1e-12 * scale[1]
    c, it = g.gpm_troubled_counts()
    assert c[1:].sum() > 0


@pytest.mark.parametrize("prec,tol", [("f64", 1e-13), ("f32", 2e-6)])
def test_closed_box_conservation(torch_cuda, prec, tol):
    """The implosion box (reflecting walls on all four sides) at 1024^2, 10 steps: mass
    and energy stay at their initial totals.  A wall face's two Riemann states are
    mirror images, and CAD on the Riemann states keeps every final one at a positive
    pressure, so the walls carry no mass or energy."""
    n = 1024
    _note(f"closed box {n} {prec} 10 steps")
    U0 = gi.implosion(n)
    g = _gp(n, n, hi=(0.3, 0.3), bc=(2, 2), prec=prec)
    g.gpm_init_state(U0)
    t0 = g.gpm_totals()
    g.gpm_step(0.8, 10)
    t1 = g.gpm_totals()
    assert abs(t1[0] - t0[0]) <= tol * abs(t0[0]), (t0, t1)
    assert abs(t1[3] - t0[3]) <= tol * abs(t0[3]), (t0, t1)
    U = g.gpm_get_state()
    assert np.all(U[0] > 0)
    c, it = g.gpm_troubled_counts()
    assert c[1:].sum() > 0


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_implosion_diagonal_symmetry_is_exact(torch_cuda, prec):
    """Sec. "The implosion problem in 2D" asks that the diagonal symmetry hold at all
    times.  On an isotropic grid a y face computes exactly what an x face computes on
    the transposed grid (diagonally paired parity sums, x weights in the x order,
    transposed gathers in the cascade, unfused axis sums), so the state stays
    bit-for-bit symmetric under x <-> y with the momenta exchanged, through shocks,
    wall reflections and the cascade: 300 steps at 128^2 in both precisions (at
    400^2 to t = 2.5 as well, 8300 steps)."""
    n = 128
    _note(f"implosion exact symmetry {n} {prec} 300 steps")
    g = _gp(n, n, hi=(0.3, 0.3), bc=(2, 2), prec=prec, cascade=(3, 1, 0))
    g.gpm_init_state(gi.implosion(n))
    lowered = 0
    for _ in range(30):
        g.gpm_step(0.8, 10)
        c, _ = g.gpm_troubled_counts()
        lowered += int(c[1:].sum())
    U = g.gpm_get_state()
    assert np.array_equal(U[0], U[0].T)
    assert np.array_equal(U[3], U[3].T)
    assert np.array_equal(U[1], U[2].T)
    assert lowered > 0


def test_stage_adjoint_rejects_walls(torch_cuda):
    """The stage adjoint has periodic and outflow boundaries only: with a reflecting
    axis it returns GPM_EUNSUPPORTED before any device work."""
    from paper_2110_08683_amd.binding import GpmError
    torch = torch_cuda
    n = 16
    g = _gp(n, n, bc=(2, 1), prec="f64")
    dev = torch.device("cuda")
    U = torch.from_numpy(gi.quadrants(n, n, seed=1)).to(dev)
    lam = torch.zeros_like(U)
    out = torch.empty_like(U)
    order = torch.full((n, n), 3, dtype=torch.uint8, device=dev)
    with pytest.raises(GpmError, match="periodic and outflow"):
        g.gpm_stage_vjp(0, None, U, order, 1e-3, lam, out)
