// Adjoint (vector-Jacobian product) of one SSP-RK3 stage with the cell orders of
// the forward stage and its dt held fixed.
//
// With the orders frozen the stage is U_out = combine(s, U^n, U*), U* = U_s - dt
// (F_{i+1/2} - F_{i-1/2}) / dx - dt (G_{j+1/2} - G_{j-1/2}) / dy (eq. (fvm_discrete)),
// every face flux a Gauss sum of HLLC fluxes of GP-reconstructed states at the
// face's EDP_1 radius (eq. (fvm_F), eq. (gp_reconstructor)).  Given lambda_out =
// dL/dU_out this returns dL/dU_s, adds dL/dU^n, and sums dL/d(ell) through the
// ell-dependence of the GP weights.  Per face:
//   1. lambda_F = (alpha lambda_out(R) - alpha lambda_out(L)) dt / Delta, from the
//      cells whose update uses this copy of the face (alpha = 1, 1/4, 2/3);
//   2. the node states are rebuilt in the quarter basis (as in the cascade);
//   3. per Gauss node, J^T (w_g lambda_F) for both states, with J from eight
//      forward-mode (dual-number) evaluations of the same HLLC code;
//   4. the transposed reconstruction: node adjoints -> accumulator adjoints ->
//      parity-sum adjoints -> the four mirror cells, added with FP64 atomics into
//      an accumulator (stencil cells remapped exactly as the forward gathers them);
//   5. dL/d(ell) += sum of accumulator adjoints times d(accumulator)/d(ell).
// A second kernel forms dL/dU_s = alpha lambda_out + accumulator and adds
// beta lambda_out to dL/dU^n (beta = 3/4, 1/3); in stage 0, where U^n is also U_s,
// a given dL/dU^n from the later stages is added to dL/dU_s instead.
#include "gpmood_device.h"
#include "gpmood_launch.h"

namespace gpm {

// ------------------------------------------------------------ dual numbers
template <typename real>
struct Dual {
    real v, d;
    __device__ Dual() {}
    __device__ Dual(real x) : v(x), d(real(0)) {}
    __device__ Dual(real x, real y) : v(x), d(y) {}
};
template <typename real>
__device__ __forceinline__ Dual<real> operator+(Dual<real> a, Dual<real> b) { return Dual<real>(a.v + b.v, a.d + b.d); }
template <typename real>
__device__ __forceinline__ Dual<real> operator-(Dual<real> a, Dual<real> b) { return Dual<real>(a.v - b.v, a.d - b.d); }
template <typename real>
__device__ __forceinline__ Dual<real> operator-(Dual<real> a) { return Dual<real>(-a.v, -a.d); }
template <typename real>
__device__ __forceinline__ Dual<real> operator*(Dual<real> a, Dual<real> b)
{
    return Dual<real>(a.v * b.v, a.d * b.v + a.v * b.d);
}
// Division and square root go through dv / sq: IEEE in FP64, the hardware
// reciprocal and square root in FP32 (as in the forward stage).
template <typename real>
__device__ __forceinline__ Dual<real> operator/(Dual<real> a, Dual<real> b)
{
    const real q = dv(a.v, b.v);
    return Dual<real>(q, dv(a.d - q * b.d, b.v));
}
template <typename real>
__device__ __forceinline__ bool operator<(Dual<real> a, Dual<real> b) { return a.v < b.v; }
template <typename real>
__device__ __forceinline__ bool operator>(Dual<real> a, Dual<real> b) { return a.v > b.v; }
template <typename real>
__device__ __forceinline__ bool operator>=(Dual<real> a, Dual<real> b) { return a.v >= b.v; }
template <typename real>
__device__ __forceinline__ Dual<real> sqrt(Dual<real> a)
{
    const real r = sq(a.v);
    return Dual<real>(r, dv(a.d, real(2) * r));
}
template <typename real>
__device__ __forceinline__ bool finite(Dual<real> a) { return __builtin_isfinite(a.v); }
template <typename real>
__device__ __forceinline__ bool pos_finite(Dual<real> a) { return pos_finite(a.v); }

// ------------------------------------------------------------ per-face adjoint
template <typename real>
__global__ __launch_bounds__(128) void k_adj_faces(const AdjArgs<real> J)
{
    __shared__ double red[128];
    const StageArgs<real> &A = J.A;
    const int nx = A.nx, ny = A.ny;
    const size_t plane = (size_t)nx * ny;
    const int nfx = (nx + 1) * ny, nft = nfx + nx * (ny + 1);
    const real alpha = A.s == 0 ? real(1) : (A.s == 1 ? real(0.25) : real(2) / real(3));
    const real dt = (real)(*A.dt);
    double dl = 0.0;
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nft; f += gridDim.x * blockDim.x) {
        int dir, iL, jL, i, j;
        bool hasL, hasR;
        if (f < nfx) {
            dir = 0;
            j = f / (nx + 1);
            i = f - j * (nx + 1);  // between cells i-1 and i
            iL = i - 1;
            jL = j;
            hasL = i >= 1;
            hasR = i < nx;
        } else {
            dir = 1;
            const int g = f - nfx;
            j = g / nx;
            i = g - j * nx;  // between cells (i, j-1) and (i, j)
            iL = i;
            jL = j - 1;
            hasL = j >= 1;
            hasR = j < ny;
        }
        const int iR = iL + (dir == 0), jR = jL + (dir == 1);
        const real inv = dt / (dir == 0 ? A.dx : A.dy);
        real lF[4];
        bool any = false;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const real lr = hasR ? J.lam_out[v * plane + (size_t)jR * nx + iR] : real(0);
            const real ll = hasL ? J.lam_out[v * plane + (size_t)jL * nx + iL] : real(0);
            lF[v] = (alpha * lr - alpha * ll) * inv;
            any = any || lF[v] != real(0);
        }
        if (!any) continue;
        const int cL = wrap(jL, ny, A.bcy) * nx + wrap(iL, nx, A.bcx);
        const int cR = wrap(jR, ny, A.bcy) * nx + wrap(iR, nx, A.bcx);
        const int R = min((int)A.order[cL], (int)A.order[cR]);
        const int np = R <= 0 ? 1 : (R == 1 ? 3 : (R == 2 ? 6 : 10));
        const int q = R <= 0 ? 1 : R + 1;
        const real *wt = A.gtab + (R * 2 + dir) * kGtabPerDir;
        const real *dwt = A.gtab_dl + (R * 2 + dir) * kGtabPerDir;
        // 1. accumulators of both cells (quarter basis, as the forward)
        real PL[4][2][4], PR[4][2][4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int c = 0; c < 4; ++c) PL[v][p][c] = PR[v][p][c] = real(0);
        for (int e = 0; e < np; ++e) {
            const int a = (int)((kPosA >> (4 * e)) & 15u), b = (int)((kPosB >> (4 * e)) & 15u);
            const int xLp = wrap(iL + a, nx, A.bcx), xLm = wrap(iL - a, nx, A.bcx);
            const int xRp = wrap(iR + a, nx, A.bcx), xRm = wrap(iR - a, nx, A.bcx);
            const size_t yLp = (size_t)wrap(jL + b, ny, A.bcy) * nx, yLm = (size_t)wrap(jL - b, ny, A.bcy) * nx;
            const size_t yRp = (size_t)wrap(jR + b, ny, A.bcy) * nx, yRm = (size_t)wrap(jR - b, ny, A.bcy) * nx;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const real *U = A.Us + v * plane;
                real ql[4], qr[4];
                parity4(U[yLp + xLp], U[yLp + xLm], U[yLm + xLp], U[yLm + xLm], ql);
                parity4(U[yRp + xRp], U[yRp + xRm], U[yRm + xRp], U[yRm + xRm], qr);
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const real w = wt[p * (kNPos * 4) + e * 4 + c];
                        PL[v][p][c] = fma(w, ql[c], PL[v][p][c]);
                        PR[v][p][c] = fma(w, qr[c], PR[v][p][c]);
                    }
            }
        }
        // 2-3. per node: states, J^T (w_g lambda_F), adjoints of the accumulators
        real gL[4][2][4], gR[4][2][4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int c = 0; c < 4; ++c) gL[v][p][c] = gR[v][p][c] = real(0);
        for (int k = 0; k < q; ++k) {
            const int slot = (R >= 2 && k >= 1 && k <= q - 2) ? 1 : 0;
            const bool single = R <= 0 || (R == 2 && k == 1);
            const bool plus = k < (q >> 1);
            const real sg = single ? real(0) : (plus ? real(1) : real(-1));
            real UL[4], UR[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const real lee = slot ? PL[v][1][C_EE] : PL[v][0][C_EE], loe = slot ? PL[v][1][C_OE] : PL[v][0][C_OE];
                const real leo = slot ? PL[v][1][C_EO] : PL[v][0][C_EO], loo = slot ? PL[v][1][C_OO] : PL[v][0][C_OO];
                const real ree = slot ? PR[v][1][C_EE] : PR[v][0][C_EE], roe = slot ? PR[v][1][C_OE] : PR[v][0][C_OE];
                const real reo = slot ? PR[v][1][C_EO] : PR[v][0][C_EO], roo = slot ? PR[v][1][C_OO] : PR[v][0][C_OO];
                const real lF = dir ? leo : loe, lN = dir ? loe : leo;  // odd across / along the face
                const real rF = dir ? reo : roe, rN = dir ? roe : reo;
                const real Ap = lee + lF, Cp = lN + loo;
                const real Bm = ree - rF, Dm = rN - roo;
                UL[v] = single ? Ap : (plus ? Ap + Cp : Ap - Cp);
                UR[v] = single ? Bm : (plus ? Bm + Dm : Bm - Dm);
            }
            const real wq_ = A.gtab[kGtabNodeOff + R * 2 + slot];
            real gs[8];  // d(w_g lambda_F . F) / d(UL, UR)
#pragma unroll
            for (int jv = 0; jv < 8; ++jv) {
                Dual<real> dl_[4], dr_[4], fd[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    dl_[v] = Dual<real>(UL[v], jv == v ? real(1) : real(0));
                    dr_[v] = Dual<real>(UR[v], jv == 4 + v ? real(1) : real(0));
                }
                // rotate the momenta into the x-face form, as hllc_rt does
                const Dual<real> L4[4] = {dl_[0], dir ? dl_[2] : dl_[1], dir ? dl_[1] : dl_[2], dl_[3]};
                const Dual<real> R4[4] = {dr_[0], dir ? dr_[2] : dr_[1], dir ? dr_[1] : dr_[2], dr_[3]};
                bool bl, br;
                hllc<0>(Dual<real>(A.gamma), L4, R4, fd, bl, br);
                const real f1 = dir ? fd[2].d : fd[1].d, f2 = dir ? fd[1].d : fd[2].d;
                gs[jv] = wq_ * (lF[0] * fd[0].d + lF[1] * f1 + lF[2] * f2 + lF[3] * fd[3].d);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // left state A + sg C with A = EE + F, C = N + OO; right state
                // Bm + sg D with Bm = EE - F, D = N - OO (F, N: OE / EO by direction)
                const real la = gs[v], lc = sg * gs[v], rb = gs[4 + v], rd = sg * gs[4 + v];
                const real cl[4] = {la, dir ? lc : la, dir ? la : lc, lc};
                const real cr[4] = {rb, dir ? rd : -rb, dir ? -rb : rd, -rd};
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    gL[v][0][c] += slot == 0 ? cl[c] : real(0);
                    gL[v][1][c] += slot == 1 ? cl[c] : real(0);
                    gR[v][0][c] += slot == 0 ? cr[c] : real(0);
                    gR[v][1][c] += slot == 1 ? cr[c] : real(0);
                }
            }
        }
        // 4-5. transposed reconstruction into the mirror cells, and the ell term
        for (int e = 0; e < np; ++e) {
            const int a = (int)((kPosA >> (4 * e)) & 15u), b = (int)((kPosB >> (4 * e)) & 15u);
            const int xLp = wrap(iL + a, nx, A.bcx), xLm = wrap(iL - a, nx, A.bcx);
            const int xRp = wrap(iR + a, nx, A.bcx), xRm = wrap(iR - a, nx, A.bcx);
            const size_t yLp = (size_t)wrap(jL + b, ny, A.bcy) * nx, yLm = (size_t)wrap(jL - b, ny, A.bcy) * nx;
            const size_t yRp = (size_t)wrap(jR + b, ny, A.bcy) * nx, yRm = (size_t)wrap(jR - b, ny, A.bcy) * nx;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const real *U = A.Us + v * plane;
                real ql[4], qr[4];
                parity4(U[yLp + xLp], U[yLp + xLm], U[yLm + xLp], U[yLm + xLm], ql);
                parity4(U[yRp + xRp], U[yRp + xRm], U[yRm + xRp], U[yRm + xRm], qr);
                real hl[4], hr[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    hl[c] = real(0);
                    hr[c] = real(0);
#pragma unroll
                    for (int p = 0; p < 2; ++p) {
                        const real w = wt[p * (kNPos * 4) + e * 4 + c];
                        const real dw = dwt[p * (kNPos * 4) + e * 4 + c];
                        hl[c] += w * gL[v][p][c];
                        hr[c] += w * gR[v][p][c];
                        dl += (double)(dw * (gL[v][p][c] * ql[c] + gR[v][p][c] * qr[c]));
                    }
                }
                // transpose of the parity sums (pp, mp, pm, mm) -> (EE, OE, EO, OO)
                double *acc = J.acc + v * plane;
                atomicAdd(&acc[yLp + xLp], (double)(hl[C_EE] + hl[C_OE] + hl[C_EO] + hl[C_OO]));
                atomicAdd(&acc[yLp + xLm], (double)(hl[C_EE] - hl[C_OE] + hl[C_EO] - hl[C_OO]));
                atomicAdd(&acc[yLm + xLp], (double)(hl[C_EE] + hl[C_OE] - hl[C_EO] - hl[C_OO]));
                atomicAdd(&acc[yLm + xLm], (double)(hl[C_EE] - hl[C_OE] - hl[C_EO] + hl[C_OO]));
                atomicAdd(&acc[yRp + xRp], (double)(hr[C_EE] + hr[C_OE] + hr[C_EO] + hr[C_OO]));
                atomicAdd(&acc[yRp + xRm], (double)(hr[C_EE] - hr[C_OE] + hr[C_EO] - hr[C_OO]));
                atomicAdd(&acc[yRm + xRp], (double)(hr[C_EE] + hr[C_OE] - hr[C_EO] - hr[C_OO]));
                atomicAdd(&acc[yRm + xRm], (double)(hr[C_EE] - hr[C_OE] - hr[C_EO] + hr[C_OO]));
            }
        }
    }
    // dL/d(ell) partial of this block, summed in a fixed order
    red[threadIdx.x] = dl;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) J.dl_partial[blockIdx.x] = red[0];
}

template <typename real>
__global__ __launch_bounds__(256) void k_adj_cells(const AdjArgs<real> J)
{
    const StageArgs<real> &A = J.A;
    const size_t n = (size_t)A.nx * A.ny;
    const real alpha = A.s == 0 ? real(1) : (A.s == 1 ? real(0.25) : real(2) / real(3));
    const real beta = A.s == 0 ? real(0) : (A.s == 1 ? real(0.75) : real(1) / real(3));
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < 4 * n; k += (size_t)gridDim.x * blockDim.x) {
        const real lo = J.lam_out[k];
        const real ls = alpha * lo + (real)J.acc[k];
        if (A.s > 0) {
            J.lam_Us[k] = ls;
            J.lam_Un[k] += beta * lo;
        } else {
            // U^n feeds both arguments of stage 0: fold in its other adjoint if given
            J.lam_Us[k] = J.lam_Un ? ls + J.lam_Un[k] : ls;
        }
    }
}

__global__ void k_adj_zero(double *acc, size_t n)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        acc[k] = 0.0;
}

// Fixed-order sum of the per-block partials into *out (one block of 256 threads):
// thread t sums the contiguous chunk t in order, then a pairwise tree in LDS.  The
// order does not depend on timing, so the result is the same on every run.
__global__ __launch_bounds__(256) void k_adj_dl_final(const double *partial, int n, double *out)
{
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int chunk = (n + 255) / 256;
    const int k0 = t * chunk, k1 = min(n, k0 + chunk);
    double s = 0.0;
    for (int k = k0; k < k1; ++k) s += partial[k];
    red[t] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) *out = red[0];
}

template <typename real>
hipError_t launch_stage_vjp(const AdjArgs<real> &J, int nblk_faces, double *dl_out, hipStream_t st)
{
    const size_t n = (size_t)J.A.nx * J.A.ny;
    hipLaunchKernelGGL(k_adj_zero, dim3(1024), dim3(256), 0, st, J.acc, 4 * n);
    hipLaunchKernelGGL(k_adj_faces<real>, dim3(nblk_faces), dim3(128), 0, st, J);
    size_t nb = (4 * n + 255) / 256;
    if (nb > 4096) nb = 4096;
    hipLaunchKernelGGL(k_adj_cells<real>, dim3((unsigned)nb), dim3(256), 0, st, J);
    hipLaunchKernelGGL(k_adj_dl_final, dim3(1), dim3(256), 0, st, J.dl_partial, nblk_faces, dl_out);
    return hipGetLastError();
}

template hipError_t launch_stage_vjp<float>(const AdjArgs<float> &, int, double *, hipStream_t);
template hipError_t launch_stage_vjp<double>(const AdjArgs<double> &, int, double *, hipStream_t);

}  // namespace gpm
