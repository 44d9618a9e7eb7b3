"""MI355X (gfx950) GP-MOOD stage engine: HIP kernels behind a C ABI (include/gpmood.h).

    from paper_2110_08683_amd import GPMood
    g = GPMood(2048, 2048, bc=(1, 1), prec="f32", cascade=(3, 2, 1, 0))
    g.gpm_init_state(U0)          # float64 host array (4, ny, nx)
    g.gpm_step(cfl=0.8, nsteps=10)
    counts, iters = g.gpm_troubled_counts()

The binding only marshals arguments; all arithmetic runs in libgpmood.so.
"""
from .binding import (EXPORTS, GPM_BC_OUTFLOW, GPM_BC_PERIODIC, GPM_BC_REFLECT, GPM_CSD, GPM_F32, GPM_F64,
                      GPM_FLAGS_ALL, GPM_PLATEAU, GPM_RSCAD, GPM_U2, GPMood, GPMood3D, GPMoodBatch, GpmError, LIB_PATH, lib)

__all__ = ["GPMood", "GPMood3D", "GPMoodBatch", "GpmError", "lib", "LIB_PATH", "EXPORTS", "GPM_F32", "GPM_F64",
           "GPM_BC_PERIODIC", "GPM_BC_OUTFLOW", "GPM_CSD", "GPM_PLATEAU", "GPM_U2", "GPM_RSCAD",
           "GPM_FLAGS_ALL"]
