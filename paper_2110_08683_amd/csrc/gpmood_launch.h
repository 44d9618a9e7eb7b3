// Host-callable launchers of the stage kernels (internal).
#ifndef GPMOOD_LAUNCH_H
#define GPMOOD_LAUNCH_H

#include <hip/hip_runtime.h>

#include "gpmood_device.h"

namespace gpm {

template <typename real>
hipError_t launch_first_pass(const StageArgs<real> &A, const PassOut &P, hipStream_t st);
template <typename real>
hipError_t launch_cascade_pass(const StageArgs<real> &A, const Cascade &C, int k, int nblocks, hipStream_t st);
template <typename real>
hipError_t launch_cascade_tail(const StageArgs<real> &A, const Cascade &C, int kbeg, int kdef, int kend,
                               hipStream_t st);
hipError_t launch_reset(Ctl *ctl, int nzero, hipStream_t st);
hipError_t launch_level_hist(const uint8_t *order, size_t ncell, const LevIdx &levidx, Ctl *ctl, hipStream_t st);
template <typename real>
hipError_t launch_dt(const real *U, size_t ncell, double gamma, double dx, double dy, double cfl, Ctl *ctl,
                     hipStream_t st);
hipError_t launch_set_dt(Ctl *ctl, double dt, hipStream_t st);
hipError_t launch_stats(Ctl *ctl, int npass, int reset, hipStream_t st);
template <typename real>
hipError_t launch_totals(const real *U, size_t ncell, double area, double *partial, int nblk, Ctl *ctl,
                         hipStream_t st);

}  // namespace gpm

#endif
