// Host-callable launchers of the stage kernels (internal).
#ifndef GPMOOD_LAUNCH_H
#define GPMOOD_LAUNCH_H

#include <hip/hip_runtime.h>

#include "gpmood_device.h"

namespace gpm {

struct LowerArgsHost {
    const int *list_in;
    const int *count_in;
    int *aff;
    int *count_aff;
    uint8_t *order;
    unsigned *stamp;
    unsigned long long *levcnt;
    int nx, ny, bcx, bcy;
    unsigned pass;
    int next[4];
    int levidx[4];
    int nblocks;
};

template <typename real>
hipError_t launch_first_pass(const StageArgs<real> &A, hipStream_t st);
hipError_t launch_cascade_lower(const LowerArgsHost &h, hipStream_t st);
template <typename real>
hipError_t launch_cascade_recompute(const StageArgs<real> &A, const int *aff, const int *count_aff, int nblocks,
                                    hipStream_t st);
hipError_t launch_reset(Ctl *ctl, int top_level, unsigned long long ncell, hipStream_t st);
template <typename real>
hipError_t launch_dt(const real *U, size_t ncell, double gamma, double dx, double dy, double cfl, Ctl *ctl,
                     hipStream_t st);
hipError_t launch_set_dt(Ctl *ctl, double dt, hipStream_t st);
template <typename real>
hipError_t launch_totals(const real *U, size_t ncell, double area, double *partial, int nblk, Ctl *ctl,
                         hipStream_t st);

}  // namespace gpm

#endif
