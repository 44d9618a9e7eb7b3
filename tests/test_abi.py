"""The C-ABI library loads and exports every symbol include/gpmood.h declares (no GPU
needed: nothing is called that touches a device), and the header and the binding
agree on the exported names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gpmood.h")).read()
    return set(re.findall(r"^\S.*?\b(gpm3?_[a-z_0-9]+)\s*\(", src, flags=re.M))


def test_header_names_match_binding():
    from paper_2110_08683_amd.binding import EXPORTS
    assert _declared() == set(EXPORTS)


def test_library_exports_all_symbols():
    from paper_2110_08683_amd.binding import LIB_PATH
    if not os.path.exists(LIB_PATH):
        pytest.fail("libgpmood.so not built: run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name


def test_strerror_and_argument_errors_without_gpu():
    from paper_2110_08683_amd import binding as B
    L = B.lib()
    assert L.gpm_strerror(0) == b"ok"
    assert L.gpm_strerror(5).startswith(b"MOOD")
    # invalid grids are rejected before any device call
    g = B.gpm_grid()
    g.dim = 3
    ctx = ctypes.c_void_p()
    assert L.gpm_create(ctypes.byref(g), 0, None, ctypes.byref(ctx)) == B.GPM_EUNSUPPORTED
    g.dim = 2
    g.n[0], g.n[1] = 0, 4
    assert L.gpm_create(ctypes.byref(g), 0, None, ctypes.byref(ctx)) == B.GPM_EINVAL
    assert L.gpm_create(None, 0, None, ctypes.byref(ctx)) == B.GPM_EINVAL
    # a periodic axis must hold the 4-cell reach of the widest stencil
    g.n[0], g.n[1] = 3, 8
    g.lo[0], g.lo[1], g.hi[0], g.hi[1] = 0.0, 0.0, 1.0, 1.0
    g.bc[0], g.bc[1] = 0, 1
    g.gamma = 1.4
    assert L.gpm_create(ctypes.byref(g), 0, None, ctypes.byref(ctx)) == B.GPM_EUNSUPPORTED
    # so must a reflecting one (the mirror image of 4 ghost cells); unknown bc values fail
    g.bc[0] = B.GPM_BC_REFLECT
    assert L.gpm_create(ctypes.byref(g), 0, None, ctypes.byref(ctx)) == B.GPM_EUNSUPPORTED
    g.bc[0] = 3
    assert L.gpm_create(ctypes.byref(g), 0, None, ctypes.byref(ctx)) == B.GPM_EINVAL
    # reflecting walls are 2D only
    g3 = B.gpm_grid()
    g3.dim = 3
    for a in range(3):
        g3.n[a], g3.lo[a], g3.hi[a], g3.bc[a] = 8, 0.0, 1.0, 1
    g3.bc[2] = B.GPM_BC_REFLECT
    g3.gamma = 1.4
    assert L.gpm3_create(ctypes.byref(g3), 0, None, ctypes.byref(ctx)) == B.GPM_EUNSUPPORTED
    # and so is an inflow slit
    g3.bc[2] = 1
    g3.slit = 1
    assert L.gpm3_create(ctypes.byref(g3), 0, None, ctypes.byref(ctx)) == B.GPM_EUNSUPPORTED
