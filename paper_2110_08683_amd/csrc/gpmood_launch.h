// Host-callable launchers of the stage kernels (internal).
#ifndef GPMOOD_LAUNCH_H
#define GPMOOD_LAUNCH_H

#include <hip/hip_runtime.h>

#include "gpmood_device.h"

namespace gpm {

template <typename real>
hipError_t launch_first_pass(const StageArgs<real> &A, const PassOut &P, const Cascade &C, hipEvent_t mid, hipStream_t st);
template <typename real>
hipError_t launch_cascade_pass(const StageArgs<real> &A, const Cascade &C, int k, int nblocks, hipStream_t st);
template <typename real>
hipError_t launch_cascade_tail(const StageArgs<real> &A, const Cascade &C, int kbeg, int kdef, int kend,
                               hipStream_t st);
hipError_t launch_reset(Ctl *ctl, int nzero, unsigned stamp0, hipStream_t st);
hipError_t launch_level_hist(const uint8_t *order, size_t ncell, const LevIdx &levidx, Ctl *ctl, hipStream_t st);
template <typename real>
hipError_t launch_lincomb4(real *out, const real *x0, const real *x1, const real *x2, const real *x3, double w0,
                           double w1, double w2, double w3, size_t n, hipStream_t st);
template <typename real>
hipError_t launch_dt(const real *U, size_t ncell, double gamma, double dx, double dy, double cfl, double lam0, Ctl *ctl,
                     hipStream_t st);
hipError_t launch_set_dt(Ctl *ctl, double dt, hipStream_t st);
hipError_t launch_stats(Ctl *ctl, int npass, int reset, hipStream_t st);
template <typename real>
hipError_t launch_totals(const real *U, size_t ncell, double area, double *partial, int nblk, double *out,
                         hipStream_t st);

template <typename real>
hipError_t launch_batch_stage(const BatchTabs<real> &B, int top, int nfp_blocks, const Cascade *casc, hipStream_t st);
template <typename real>
hipError_t launch_batch_first_pass(const BatchTabs<real> &B, int top, int nfp_blocks, const Cascade *casc,
                                   hipStream_t st);
template <typename real>
hipError_t launch_batch_dt(const BatchTabs<real> &B, int ndt_blocks, const Cascade *casc, double cfl, hipStream_t st);
hipError_t launch_batch_status(const Cascade *casc, int nprob, int *iters, double *dts, hipStream_t st);
hipError_t launch_batch_stamp_restart(const Cascade *casc, int nprob, hipStream_t st);
template <typename real>
hipError_t launch_stage_vjp(const AdjArgs<real> &J, int nblk_faces, double *dl_out, bool accumulate, hipStream_t st);

}  // namespace gpm

#endif
