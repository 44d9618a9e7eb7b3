"""GPU parity where the small replays do not reach, element by element against the
plain FP64 oracle (Sec. "Stepwise implementation", Steps 3-10, the MOOD loop run to
completion):

- the headline grid itself: the four-quadrant problem at 2048^2 (seed 1), a full
  SSP-RK3 step replayed stage by stage on the GPU's own stage inputs;
- late-run states where a stage needs 100 to 350 MOOD evaluations (long chains of
  lowered cells along the shock fronts), at 512^2 and 1024^2;
- every cascade path of the engine on such a stage: multi-block passes only, the
  single-workgroup tail only, and the tail handing back to multi-block passes, plus
  first-pass march lengths and check batches: bit for bit the default's result;
- the 3D blast's own input (p 1e4 inside, 1e-5 outside, 1% density noise).

Bar (FP64): per field, relative L1 <= 1e-12 and max |dU| <= 1e-12 max |U|; order
masks, per-level counts and evaluation counts identical."""
import sys

import numpy as np
import pytest

import gpmood_inputs as gi
import oracle
from tests.parity_util import assert_fields_close

pytestmark = pytest.mark.gpu

CASCADE = (3, 2, 1, 0)


def _note(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _gp(nx, ny, prec="f64", bc=(1, 1)):
    from paper_2110_08683_amd import GPMood
    return GPMood(nx, ny, bc=bc, prec=prec, cascade=CASCADE, device="cuda:0")


def _gpu_stage(torch, g, s, Un, Us):
    out = torch.empty_like(Us)
    g.gpm_stage_dev(s, Un, Us, out)
    torch.cuda.synchronize()
    counts, iters = g.gpm_troubled_counts()
    return out, g.gpm_get_order_mask().astype(np.int32), counts, iters, g.gpm_cascade_stats()


def _replay_step(torch, g, o, U, stages=(0, 1, 2), what=""):
    """One SSP-RK3 step on the GPU from the device state U (FP64): each stage's output
    against the oracle's stage run on the GPU's own stage input.  Returns the GPU's
    evaluations per stage."""
    dt = g.gpm_compute_dt_dev(U, 0.8)
    Un_h = U.cpu().numpy()
    assert abs(dt - o.dt(Un_h, 0.8)) <= 1e-12 * dt
    g.gpm_set_dt(dt)
    Us = U
    iters_out = []
    for s in (0, 1, 2):
        out, mask, counts, iters, stats = _gpu_stage(torch, g, s, U, Us)
        iters_out.append(iters)
        if s in stages:
            Us_h = Us.cpu().numpy()
            Uo, order, ocounts, oiters = o.stage(s, Un_h, Us_h, dt)
            _note(f"  {what} stage {s}: evaluations {iters} / {oiters}, passes (multi-block, tail, hand-backs) {stats}")
            assert np.array_equal(mask, order), f"{what} stage {s}: mask differs at {int((mask != order).sum())} cells"
            np.testing.assert_array_equal(counts[:len(CASCADE)], ocounts)
            assert iters == oiters
            assert stats[0] + stats[1] + 1 == iters
            assert_fields_close(out.cpu().numpy(), Uo, what=f"{what} stage {s}")
        Us = out
    return iters_out


@pytest.mark.timeout(900)
def test_headline_grid_2048_step_replay(torch_cuda):
    """The benchmark's own problem: 2048^2, seed 1, outflow, GP-MOOD7 7-5-3-1, FP64.
    Four GPU steps let the waves develop; the fifth is replayed stage by stage."""
    torch = torch_cuda
    n = 2048
    _note("headline 2048^2 seed 1 f64: 4 steps, then step 5 replayed")
    g = _gp(n, n)
    o = oracle.Oracle(n, n, bc=(1, 1), cascade=CASCADE)
    g.gpm_init_state(gi.quadrants(n, n, seed=1))
    g.gpm_step(0.8, 4)
    U = g.slot(g.current_slot())
    iters = _replay_step(torch, g, o, U.clone(), what="2048^2")
    assert max(iters) >= 5
    g.close()


@pytest.fixture(scope="module")
def late512(torch_cuda):
    """The 512^2 four-quadrant problem (seed 1) after 224 GPU steps: the last stage of
    step 225 needs more than 100 MOOD evaluations."""
    torch = torch_cuda
    n = 512
    g = _gp(n, n)
    g.gpm_init_state(gi.quadrants(n, n, seed=1))
    g.gpm_step(0.8, 224)
    torch.cuda.synchronize()
    U = g.slot(g.current_slot()).clone()
    g.close()
    return U


@pytest.mark.timeout(600)
def test_late_run_512_step_replay(torch_cuda, late512):
    torch = torch_cuda
    n = 512
    _note("late run 512^2 seed 1 f64: step 225 replayed")
    g = _gp(n, n)
    o = oracle.Oracle(n, n, bc=(1, 1), cascade=CASCADE)
    iters = _replay_step(torch, g, o, late512, what="512^2 late")
    assert max(iters) >= 100
    g.close()


# (passes_per_check, rows_per_wave, tail_threshold) and what each must exercise
TUNINGS = [
    ((4, 12, 0), "multi-block passes only"),
    ((4, 12, 4096), "the tail from the first cascade pass"),
    ((4, 12, 1), "the tail handing back to multi-block passes"),
    ((1, 4, 32), "4-row marches, one pass per check"),
    ((128, 32, 32), "32-row marches, 128 passes per check"),
    ((4, 256, 8), "256-row marches"),
]


@pytest.mark.timeout(600)
def test_cascade_paths_are_bitwise_equal(torch_cuda, late512):
    """The last stage of step 225 at 512^2 (100+ evaluations) under every cascade path
    and first-pass march length: outputs, masks, counts and evaluations equal the
    default configuration's bit for bit, and the default's equal the oracle's."""
    torch = torch_cuda
    n = 512
    g = _gp(n, n)
    U = late512
    dt = g.gpm_compute_dt_dev(U, 0.8)
    g.gpm_set_dt(dt)
    U1, *_ = _gpu_stage(torch, g, 0, U, U)
    U2, *_ = _gpu_stage(torch, g, 1, U, U1)
    ref = _gpu_stage(torch, g, 2, U, U2)
    _note(f"late 512^2 stage 2 default: evaluations {ref[3]}, passes {ref[4]}")
    assert ref[3] >= 100
    o = oracle.Oracle(n, n, bc=(1, 1), cascade=CASCADE)
    Uo, order, ocounts, oiters = o.stage(2, U.cpu().numpy(), U2.cpu().numpy(), dt)
    assert np.array_equal(ref[1], order) and ref[3] == oiters
    assert_fields_close(ref[0].cpu().numpy(), Uo, what="512^2 late stage 2")
    ref_h = ref[0].cpu().numpy()
    for tun, what in TUNINGS:
        g.gpm_set_tuning(*tun)
        out, mask, counts, iters, stats = _gpu_stage(torch, g, 2, U, U2)
        _note(f"  tuning {tun} ({what}): evaluations {iters}, passes (multi-block, tail, hand-backs) {stats}")
        assert np.array_equal(out.cpu().numpy(), ref_h), what
        assert np.array_equal(mask, ref[1]) and np.array_equal(counts, ref[2]) and iters == ref[3], what
        assert stats[0] + stats[1] + 1 == iters
        if tun[2] == 0:
            assert stats[1] == 0 and stats[0] == iters - 1
        if tun[2] == 4096:
            assert stats[1] == iters - 1 and stats[0] == 0
        if tun[2] == 1:
            assert stats[2] >= 1 and stats[0] > 0 and stats[1] > 0
    g.close()


@pytest.mark.timeout(900)
def test_very_long_cascade_1024(torch_cuda):
    """1024^2, seed 2, after 724 GPU steps: the last stage of step 725 runs about 350
    MOOD evaluations, with tail hand-backs; replayed against the oracle."""
    torch = torch_cuda
    n = 1024
    _note("1024^2 seed 2 f64: 724 steps, stage 2 of step 725 replayed")
    g = _gp(n, n)
    g.gpm_init_state(gi.quadrants(n, n, seed=2))
    g.gpm_step(0.8, 724)
    U = g.slot(g.current_slot()).clone()
    o = oracle.Oracle(n, n, bc=(1, 1), cascade=CASCADE)
    iters = _replay_step(torch, g, o, U, stages=(2,), what="1024^2 late")
    assert iters[2] >= 300
    g.close()


@pytest.mark.parametrize("n,nsteps", [(16, 2), (18, 1)])
def test_3d_blast_input_fp64(torch_cuda, n, nsteps):
    """The 3D blast's own input at 16^3 and 18^3: rho = 1 +- 1% (seed 3), p = 1e-5, and
    p = 1e4 within 3 cells of the centre (a pressure ratio of 1e9), outflow,
    GP-MOOD5, CFL 0.3: whole steps against the 3D oracle."""
    from paper_2110_08683_amd import GPMood3D
    _note(f"3d blast input {n}^3 f64 {nsteps} steps")
    U0 = gi.blast3d(n)
    g = GPMood3D((n, n, n), bc=(1, 1, 1), prec="f64", cascade=(2, 1, 0), device="cuda:0")
    g.gpm3_init_state(U0)
    o = oracle.Oracle3D((n, n, n), bc=(1, 1, 1), cascade=(2, 1, 0))
    Uo, dts, iters, counts = o.run(U0, cfl=0.3, nsteps=nsteps)
    g.gpm3_step(0.3, nsteps)
    U = g.gpm3_get_state()
    c, it = g.gpm3_troubled_counts()
    _note(f"  counts {c} / {counts} evaluations {it} / {iters[-1, 2]}")
    assert list(c[:3]) == list(counts) and it == iters[-1, 2]
    assert counts[1:].sum() > 0  # the cascade ran
    assert_fields_close(U, Uo, what=f"3d blast {n}^3")
    g.close()
