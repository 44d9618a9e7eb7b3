"""GPU parity of the batched ensemble through the C ABI.

Problems of uneven (and non-square) sizes advance together; each must match the
FP64 oracle run of that problem alone (relative L1 <= 1e-12, identical dt, final
per-level counts and evaluations of the last stage), and the HIP-graph replay must
reproduce the eager batch exactly, step by step.
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


def _rel_l1(a, b):
    return max(np.abs(a[v] - b[v]).sum() / np.abs(b[v]).sum() for v in range(4))


SIZES = [(48, 48), (64, 40), (40, 72), (96, 96), (33, 57)]


def _batch(torch_cuda, sizes, bc, cascade, prec, seed0):
    from paper_2110_08683_amd import GPMoodBatch
    b = GPMoodBatch(sizes, bc=bc, prec=prec, cascade=cascade, device="cuda:0")
    U0s = [gi.quadrants(nx, ny, seed=seed0 + k) for k, (nx, ny) in enumerate(sizes)]
    for k, U0 in enumerate(U0s):
        b.gpm_batch_init_state(k, U0)
    return b, U0s


@pytest.mark.parametrize("bc,cascade,use_graph", [((1, 1), (3, 2, 1, 0), False), ((0, 0), (3, 1, 0), True),
                                                  ((1, 0), (2, 1, 0), True), ((2, 2), (3, 2, 1, 0), True)])
def test_batch_matches_oracle_fp64(torch_cuda, bc, cascade, use_graph):
    nsteps = 2
    _note(f"batch f64 sizes={SIZES} bc={bc} cascade={cascade} graph={use_graph} steps={nsteps}")
    b, U0s = _batch(torch_cuda, SIZES, bc, cascade, "f64", 20)
    b.gpm_batch_step(0.8, nsteps, use_graph=use_graph)
    iters, dts = b.gpm_batch_status()
    for k, (nx, ny) in enumerate(SIZES):
        o = oracle.Oracle(nx, ny, bc=bc, cascade=cascade)
        Uo, dto, co, io = o.run(U0s[k], cfl=0.8, nsteps=nsteps)
        U = b.gpm_batch_get_state(k)
        err = _rel_l1(U, Uo)
        assert_fields_close(U, Uo, what=f"problem {k}")
        counts, it = b.gpm_batch_troubled_counts(k)
        _note(f"  problem {k} {nx}x{ny}: rel L1 {err:.2e} dt {dts[k]:.6e}/{dto[-1]:.6e} "
              f"counts {counts[:len(cascade)]}/{co[-1, 2]} iters {it}/{io[-1, 2]}")
        assert err <= 1e-12
        assert abs(dts[k] - dto[-1]) <= 1e-12 * dto[-1]
        assert list(counts[:len(cascade)]) == list(co[-1, 2])
        assert it == io[-1, 2] == iters[k]
    b.close()


def test_batch_graph_replays_match_eager_fp32(torch_cuda):
    """Each graph replay (one SSP-RK3 step) equals the eager batch after the same step,
    bitwise, with host synchronisation and state reads between the replays."""
    sizes = SIZES[:4]
    _note(f"batch f32 graph vs eager sizes={sizes} 4 steps")
    bg, _ = _batch(torch_cuda, sizes, (1, 1), (3, 2, 1, 0), "f32", 40)
    be, _ = _batch(torch_cuda, sizes, (1, 1), (3, 2, 1, 0), "f32", 40)
    for step in range(4):
        bg.gpm_batch_step(0.8, 1, use_graph=True)
        be.gpm_batch_step(0.8, 1, use_graph=False)
        torch_cuda.cuda.synchronize()
        for k in range(len(sizes)):
            a, e = bg.gpm_batch_get_state(k), be.gpm_batch_get_state(k)
            assert np.array_equal(a, e), (step, k)
            assert np.array_equal(bg.gpm_batch_get_order_mask(k), be.gpm_batch_get_order_mask(k))
    bg.close()
    be.close()


def test_batch_equals_single_problem_contexts_fp32(torch_cuda):
    """A batch gives, bitwise, what one single-problem context per problem gives."""
    from paper_2110_08683_amd import GPMood
    sizes = [(64, 64), (80, 48)]
    _note(f"batch f32 vs single contexts sizes={sizes} 3 steps")
    b, U0s = _batch(torch_cuda, sizes, (1, 1), (3, 2, 1, 0), "f32", 60)
    b.gpm_batch_step(0.8, 3, use_graph=True)
    for k, (nx, ny) in enumerate(sizes):
        g = GPMood(nx, ny, bc=(1, 1), prec="f32", cascade=(3, 2, 1, 0), device="cuda:0")
        g.gpm_init_state(U0s[k])
        g.gpm_step(0.8, 3)
        assert np.array_equal(g.gpm_get_state(), b.gpm_batch_get_state(k)), k
        assert np.array_equal(g.gpm_get_order_mask(), b.gpm_batch_get_order_mask(k)), k
        g.close()
    b.close()


def test_batch_u2_weights_are_per_problem(torch_cuda):
    """Problems whose length scale is the same in cells share their reconstruction
    weights, but not the u2 curvature weights, which are second derivatives in
    physical units (1 / dx^2).  An 8^2 problem ahead of a 96^2 one: the 96^2 problem
    (y walls, where u2 decides cells near the wall in the second step) must match the
    oracle run of it alone."""
    from paper_2110_08683_amd import GPMoodBatch
    sizes = [(8, 8), (96, 96)]
    _note("batch u2 weights per problem: 8^2 + 96^2, bc (1, 2), cascade (1, 0), 2 steps")
    b = GPMoodBatch(sizes, bc=(1, 2), prec="f64", cascade=(1, 0), device="cuda:0")
    U0s = [gi.density_wave(8, 8), gi.quadrants(96, 96, seed=23)]
    for k, U0 in enumerate(U0s):
        b.gpm_batch_init_state(k, U0)
    b.gpm_batch_step(0.8, 2, use_graph=False)
    for k, (nx, ny) in enumerate(sizes):
        Uo = oracle.Oracle(nx, ny, bc=(1, 2), cascade=(1, 0)).run(U0s[k], cfl=0.8, nsteps=2)[0]
        err = _rel_l1(b.gpm_batch_get_state(k), Uo)
        assert_fields_close(b.gpm_batch_get_state(k), Uo, what=f"problem {k}")
        _note(f"  problem {k} {nx}x{ny}: rel L1 {err:.2e}")
        assert err <= 1e-12
    b.close()


def test_autotuned_batch_is_bitwise_equal(torch_cuda, tmp_path):
    """The library's autotuner picks a first-pass march length per size class; the
    tuned batch gives the same bits as the default one (FP32, uneven sizes, graph
    replay), its timing launches leave the states unchanged, and a cached choice is
    applied without timing."""
    from paper_2110_08683_amd import GPMoodBatch
    sizes = [(64, 64), (96, 96), (128, 128), (200, 200), (256, 256), (300, 300)]
    _note(f"batch autotune f32 sizes={sizes}")
    U0s = [gi.quadrants(nx, ny, seed=60 + k) for k, (nx, ny) in enumerate(sizes)]
    states = []
    for tuned in (False, True):
        b = GPMoodBatch(sizes, bc=(1, 1), prec="f32", cascade=(3, 2, 1, 0), device="cuda:0")
        for k, U0 in enumerate(U0s):
            b.gpm_batch_init_state(k, U0)
        if tuned:
            rows, gain = b.autotune(0.8, reps=2, cache=str(tmp_path / "tune.json"))
            _note(f"  chosen rows per problem {rows}, first-pass gain over the default {gain:.3f}")
            assert all(4 <= r <= 64 for r in rows) and gain > 0
            # the timing launches did not touch the states
            for k, U0 in enumerate(U0s):
                assert np.array_equal(b.gpm_batch_get_state(k), U0.astype(np.float32).astype(np.float64))
        b.gpm_batch_step(0.8, 3, use_graph=True)
        states.append([b.gpm_batch_get_state(k) for k in range(len(sizes))])
        b.close()
    for k in range(len(sizes)):
        assert np.array_equal(states[0][k], states[1][k]), k
    # a second batch takes the cached choice
    b = GPMoodBatch(sizes, bc=(1, 1), prec="f32", cascade=(3, 2, 1, 0), device="cuda:0")
    rows2, gain2 = b.autotune(0.8, reps=2, cache=str(tmp_path / "tune.json"))
    assert gain2 is None and rows2 == rows
    b.close()


def test_cascade_autotuned_batch_is_bitwise_equal(torch_cuda):
    """The cascade threshold the autotuner picks changes the schedule only: the
    tuned batch gives the same bits as the default one (FP64, uneven sizes, graph
    replay), and its timing stages leave the states unchanged."""
    from paper_2110_08683_amd import GPMoodBatch
    sizes = [(64, 64), (96, 80), (128, 128), (200, 160)]
    _note(f"batch cascade autotune f64 sizes={sizes}")
    U0s = [gi.quadrants(nx, ny, seed=80 + k) for k, (nx, ny) in enumerate(sizes)]
    states = []
    for tuned in (False, True):
        b = GPMoodBatch(sizes, bc=(1, 1), prec="f64", cascade=(3, 2, 1, 0), device="cuda:0")
        for k, U0 in enumerate(U0s):
            b.gpm_batch_init_state(k, U0)
        b.gpm_batch_step(0.8, 2, use_graph=True)
        if tuned:
            before = [b.gpm_batch_get_state(k) for k in range(len(sizes))]
            tail, gain = b.gpm_batch_autotune_cascade(0.8, reps=2)
            _note(f"  chosen cascade threshold {tail}, gain over the default {gain:.3f}")
            assert tail in (8, 16, 32, 64, 128, 256) and gain > 0
            for k in range(len(sizes)):
                assert np.array_equal(b.gpm_batch_get_state(k), before[k])
        b.gpm_batch_step(0.8, 3, use_graph=True)
        states.append([b.gpm_batch_get_state(k) for k in range(len(sizes))])
        b.close()
    for k in range(len(sizes)):
        assert np.array_equal(states[0][k], states[1][k]), k
