"""GPU parity of the HLL Riemann solver (gpm_scheme.solver = GPM_SOLVER_HLL, the
solver of the paper's Mach-jet problems) against the FP64 oracle run with
solver="hll": RK stages replayed on the oracle's inputs (relative L1 <= 1e-12,
identical masks, counts and evaluations), a batch of problems, and an FP32 run that
stays positive.  The stage adjoint rejects the HLL scheme."""
import ctypes
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


def _rel_l1(a, b):
    return np.array([np.abs(a[v] - b[v]).sum() / max(np.abs(b[v]).sum(), 1e-300) for v in range(4)])


@pytest.mark.parametrize("nx,ny,seed,bc,cascade", [
    (70, 66, 2, (1, 1), (3, 2, 1, 0)),
    (64, 48, 5, (2, 0), (2, 1, 0)),
    (96, 96, 7, (0, 0), (3, 1, 0)),
])
def test_hll_stage_replay_fp64(torch_cuda, nx, ny, seed, bc, cascade):
    from paper_2110_08683_amd import GPMood
    torch = torch_cuda
    _note(f"hll replay {nx}x{ny} seed={seed} bc={bc} cascade={cascade}")
    U0 = gi.quadrants(nx, ny, seed=seed)
    o = oracle.Oracle(nx, ny, bc=bc, cascade=cascade, solver="hll")
    g = GPMood(nx, ny, bc=bc, prec="f64", cascade=cascade, solver="hll")
    U = o.run(U0, cfl=0.8, nsteps=2)[0]
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
    # and the HLLC scheme gives another answer on the same stage
    gc = GPMood(nx, ny, bc=bc, prec="f64", cascade=cascade)
    tn, ts = torch.from_numpy(U).to(dev), torch.from_numpy(U).to(dev)
    tout = torch.empty_like(ts)
    gc.gpm_set_dt(dt)
    gc.gpm_stage_dev(0, tn, ts, tout)
    torch.cuda.synchronize()
    assert np.abs(tout.cpu().numpy() - o.stage(0, U, U, dt)[0]).max() > 1e-8


def test_hll_batch_matches_oracle_fp64(torch_cuda):
    from paper_2110_08683_amd import GPMoodBatch
    sizes = [(48, 48), (64, 40), (33, 57)]
    _note(f"hll batch f64 sizes={sizes} 2 steps")
    b = GPMoodBatch(sizes, bc=(1, 1), prec="f64", cascade=(3, 2, 1, 0), device="cuda:0", solver="hll")
    U0s = [gi.quadrants(nx, ny, seed=40 + k) for k, (nx, ny) in enumerate(sizes)]
    for k, U0 in enumerate(U0s):
        b.gpm_batch_init_state(k, U0)
    b.gpm_batch_step(0.8, 2, use_graph=True)
    for k, (nx, ny) in enumerate(sizes):
        Uo = oracle.Oracle(nx, ny, bc=(1, 1), solver="hll").run(U0s[k], cfl=0.8, nsteps=2)[0]
        err = _rel_l1(b.gpm_batch_get_state(k), Uo).max()
        assert_fields_close(b.gpm_batch_get_state(k), Uo, what=f"problem {k}")
        _note(f"  problem {k} {nx}x{ny}: rel L1 {err:.2e}")
        assert err <= 1e-12
    b.close()


def test_hll_fp32_positivity(torch_cuda):
    from paper_2110_08683_amd import GPMood
    n = 128
    _note("hll f32 positivity 20 steps")
    g = GPMood(n, n, bc=(1, 1), prec="f32", solver="hll")
    g.gpm_init_state(gi.quadrants(n, n, seed=1))
    g.gpm_step(0.8, 20)
    U = g.gpm_get_state()
    p = 0.4 * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / U[0])
    assert np.all(U[0] > 0) and np.all(p > 0)


def test_stage_adjoint_rejects_hll(torch_cuda):
    from paper_2110_08683_amd import GPMood
    from paper_2110_08683_amd.binding import GpmError
    torch = torch_cuda
    n = 16
    g = GPMood(n, n, bc=(1, 1), prec="f64", solver="hll")
    dev = torch.device("cuda")
    U = torch.from_numpy(gi.quadrants(n, n, seed=1)).to(dev)
    lam = torch.zeros_like(U)
    out = torch.empty_like(U)
    order = torch.full((n, n), 3, dtype=torch.uint8, device=dev)
    with pytest.raises(GpmError, match="HLLC scheme only"):
        g.gpm_stage_vjp(0, None, U, order, 1e-3, lam, out)


def test_unknown_solver_is_rejected(torch_cuda):
    from paper_2110_08683_amd import GPMood
    from paper_2110_08683_amd import binding as B
    with pytest.raises(KeyError):
        GPMood(8, 8, solver="roe")
    g = GPMood(8, 8, bc=(1, 1), prec="f64", cascade=(1, 0))
    s = B.gpm_scheme()
    s.nlev, s.radius[0], s.radius[1] = 2, 1, 0
    s.sigma_v = s.sigma_p = 5.0
    s.flags = B.GPM_FLAGS_ALL
    s.solver = 7
    L = B.lib()
    assert L.gpm_set_scheme(g.ctx, ctypes.byref(s)) == B.GPM_EINVAL
    assert b"solver" in L.gpm_last_error(g.ctx)
