"""gpm_totals_static, the totals entry point that allocates nothing, against
gpm_totals_dev (the same kernels with the bound workspace) through the C ABI: two
calls in a row, the second on a smaller grid (the static scratch keeps the first
call's partials), each equal bit for bit to gpm_totals_dev; and a call on a
context that was never bound."""
import ctypes
import sys

import numpy as np
import pytest

import gpmood_inputs as gi

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


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_totals_static_matches_totals_dev(torch_cuda, prec):
    from paper_2110_08683_amd import GPMood
    dtype = torch_cuda.float64 if prec == "f64" else torch_cuda.float32
    for n in (640, 96):  # 1600 blocks (capped at 1024, grid-stride) then 36 blocks
        _note(f"totals_static {prec} {n}^2")
        g = GPMood(n, n, bc=(1, 1), prec=prec, cascade=(3, 2, 1, 0), device="cuda:0")
        U = torch_cuda.tensor(gi.quadrants(n, n, seed=7 + n), dtype=dtype, device="cuda:0")
        t_dev = g.gpm_totals_dev(U)
        t_st = g.gpm_totals_static(U)
        np.testing.assert_array_equal(t_st, t_dev)
        ref = U.double().sum(dim=(1, 2)).cpu().numpy() / n ** 2  # cell area on the unit square
        np.testing.assert_allclose(t_st, ref, rtol=1e-12)
        g.close()


def test_totals_static_on_an_unbound_context(torch_cuda):
    from paper_2110_08683_amd import binding as B
    L = B.lib()
    n = 200
    _note(f"totals_static unbound context {n}^2")
    grid = B.gpm_grid()
    grid.dim = 2
    grid.n[0] = grid.n[1] = n
    grid.lo[0] = grid.lo[1] = 0.0
    grid.hi[0] = grid.hi[1] = 1.0
    grid.bc[0] = grid.bc[1] = 1
    grid.gamma = 1.4
    ctx = ctypes.c_void_p()
    stream = torch_cuda.cuda.current_stream().cuda_stream
    assert L.gpm_create(ctypes.byref(grid), 1, ctypes.c_void_p(stream), ctypes.byref(ctx)) == 0
    try:
        U = torch_cuda.tensor(gi.quadrants(n, n, seed=3), dtype=torch_cuda.float64, device="cuda:0")
        t = np.zeros(4)
        st = L.gpm_totals_static(ctx, ctypes.c_void_p(U.data_ptr()), t.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        assert st == 0, L.gpm_last_error(ctx)
        ref = U.double().sum(dim=(1, 2)).cpu().numpy() / n ** 2
        np.testing.assert_allclose(t, ref, rtol=1e-12)
        # a NULL state is rejected before any device work
        assert L.gpm_totals_static(ctx, None, t.ctypes.data_as(ctypes.POINTER(ctypes.c_double))) == 1
    finally:
        L.gpm_destroy(ctx)
