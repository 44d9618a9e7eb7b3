// HIP kernels of the 2D GP-MOOD stage for gfx950 (CDNA4).
//
// First pass (k_first_pass): every cell at the top order.  One 64-lane wavefront
// owns a strip of 62 columns (lanes 1..62; lanes 0 and 63 are the halo that
// supplies the neighbouring face states) and marches upward through `rows` rows.
// The stage input of rows j-3..j+4 sits in a per-wavefront ring of 8 LDS rows
// (70 columns x 4 variables), loaded once with coalesced row loads and the
// boundary conditions applied as index remaps.  At row j each lane reconstructs
// all 4q face states of its cell (eq. (gp_reconstructor) in the quarter basis),
// exchanges x-face states with its right neighbour by a lane shuffle, evaluates
// HLLC on its own x face, and evaluates the y face below it against the y+ states
// it kept from row j-1.  Cell (i, j-1) is then complete: candidate, detection,
// RK combine and the wavefront-ballot append of troubled cells.  No block
// barrier is needed anywhere: each wavefront only reads LDS it wrote itself.
//
// Cascade (k_cascade_lower, k_cascade_recompute): troubled cells move to the next
// scheme of the cascade; the troubled cells and their face neighbours are
// recomputed with EDP_1 face orders and re-detected; the new troubled cells are
// appended to the next list.  Both kernels read their item count from device
// memory and return at once when it is zero, so several passes can be queued
// without a host round trip.
#include "gpmood_device.h"
#include "gpmood_launch.h"

namespace gpm {

constexpr int LW = 70;  // LDS columns per ring row: 64 lanes + 3 halo columns each side

// blockIdx -> tile: consecutive tiles go to the same XCD (blocks are dealt to the
// 8 XCDs round robin), so neighbouring strips share halo rows in one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

template <typename real, int RT, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_first_pass(const StageArgs<real> A)
{
    constexpr int q = nodes_of(RT);
    constexpr int NQ = kNQ[RT];
    __shared__ real ring_all[WPB][8][4][LW];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    real(*ring)[4][LW] = ring_all[wv];

    const int nx = A.nx, ny = A.ny, T = A.rows;
    const int nstrip = (nx + 61) / 62, nseg = (ny + T - 1) / T;
    const int wid = xcd_tile(blockIdx.x, gridDim.x) * WPB + wv;
    if (wid >= nstrip * nseg) return;  // whole wavefront leaves together
    const int sx = wid % nstrip, sy = wid / nstrip;
    const int x0 = sx * 62, y0 = sy * T;
    const int yend = min(y0 + T, ny);
    const int i = x0 - 1 + lane;
    const bool own = lane >= 1 && lane <= 62 && i < nx;
    const size_t plane = (size_t)nx * ny;

    const int sc0 = remap(x0 - 4 + lane, nx, A.bcx);
    const bool has1 = lane < LW - 64;
    const int sc1 = remap(x0 - 4 + 64 + (has1 ? lane : 0), nx, A.bcx);
    const real *__restrict__ Us = A.Us;

    auto load_row = [&](int jr, real (&pf)[4][2]) {
        const size_t rowoff = (size_t)remap(jr, ny, A.bcy) * nx;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            pf[v][0] = Us[v * plane + rowoff + sc0];
            pf[v][1] = has1 ? Us[v * plane + rowoff + sc1] : real(0);
        }
    };
    auto store_row = [&](int jr, const real (&pf)[4][2]) {
        const int slot = jr & 7;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            ring[slot][v][lane] = pf[v][0];
            if (has1) ring[slot][v][64 + lane] = pf[v][1];
        }
    };
    for (int jr = y0 - 4; jr <= y0 + 2; ++jr) {
        real pf[4][2];
        load_row(jr, pf);
        store_row(jr, pf);
    }
    wave_lds_sync();

    const real dt = (real)(*A.dt);
    const real g = A.gamma;
    real sypP[q][4];   // y+ states of row j-1
    real Gprev[4];     // flux through face j-3/2
    real dFxP[4];      // x-flux difference of row j-1
    bool rsxP = false, rsymP = false;
#pragma unroll
    for (int v = 0; v < 4; ++v) { Gprev[v] = real(0); dFxP[v] = real(0); }

    for (int j = y0 - 1; j <= yend; ++j) {
        real pf[4][2];
        load_row(j + 4, pf);  // in flight during this row's arithmetic
        const bool doX = j >= y0 && j < yend;
        const bool first = j == y0 - 1;

        real sxm[q][4], sxp[q][4], sym[q][4], syp[q][4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            real Q[NQ];
            build_Q<RT>(Q, [&](int di, int dj) { return ring[(j + dj) & 7][v][lane + 3 + di]; });
            real m_[q], p_[q];
            if (doX) {
                states_dir<RT, 0>(Q, A.W, m_, p_);
#pragma unroll
                for (int k = 0; k < q; ++k) { sxm[k][v] = m_[k]; sxp[k][v] = p_[k]; }
            }
            states_dir<RT, 1>(Q, A.W, m_, p_);
#pragma unroll
            for (int k = 0; k < q; ++k) { sym[k][v] = m_[k]; syp[k][v] = p_[k]; }
        }

        real dFx[4] = {real(0), real(0), real(0), real(0)};
        bool rsx = false;
        if (doX) {
            real F[4] = {real(0), real(0), real(0), real(0)};
            bool badNb = false;
#pragma unroll
            for (int k = 0; k < q; ++k) {
                real ur[4], f[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) ur[v] = __shfl_down(sxm[k][v], 1);
                bool bl, br;
                hllc<0>(g, sxp[k], ur, f, bl, br);
                rsx = rsx || bl;
                badNb = badNb || br;
                const real w = node_weight<RT>(A.W, k);
#pragma unroll
                for (int v = 0; v < 4; ++v) F[v] = fma(w, f[v], F[v]);
            }
            const int badm = __shfl_up((int)badNb, 1);
            rsx = rsx || (badm != 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) dFx[v] = F[v] - __shfl_up(F[v], 1);
        }

        if (!first) {
            real G[4] = {real(0), real(0), real(0), real(0)};
            bool badLy = false, badRy = false;
#pragma unroll
            for (int k = 0; k < q; ++k) {
                real f[4];
                bool bl, br;
                hllc<1>(g, sypP[k], sym[k], f, bl, br);
                badLy = badLy || bl;
                badRy = badRy || br;
                const real w = node_weight<RT>(A.W, k);
#pragma unroll
                for (int v = 0; v < 4; ++v) G[v] = fma(w, f[v], G[v]);
            }
            if (j - 1 >= y0) {
                // cell (i, j-1) is complete
                const int jr = j - 1;
                const int slot = jr & 7;
                real us[4], ust[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    us[v] = ring[slot][v][lane + 3];
                    ust[v] = us[v] - dt * (dFxP[v] / A.dx + (G[v] - Gprev[v]) / A.dy);
                }
                const bool rs = rsxP || rsymP || badLy;
                auto nb = [&](int di, int dj, int v) { return ring[(jr + dj) & 7][v][lane + 3 + di]; };
                const bool tr = own && troubled(A, RT, ust, rs, nb);
                if (own) {
                    const size_t c = (size_t)jr * nx + i;
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const real un = A.s == 0 ? real(0) : A.Un[v * plane + c];
                        A.Uout[v * plane + c] = combine(A.s, un, ust[v]);
                    }
                    A.order[c] = (uint8_t)RT;
                }
                wave_append(tr, jr * nx + i, A.list_out, A.count_out);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) Gprev[v] = G[v];
            rsymP = badRy;
        }
#pragma unroll
        for (int k = 0; k < q; ++k)
#pragma unroll
            for (int v = 0; v < 4; ++v) sypP[k][v] = syp[k][v];
#pragma unroll
        for (int v = 0; v < 4; ++v) dFxP[v] = dFx[v];
        rsxP = rsx;
        store_row(j + 4, pf);
        wave_lds_sync();
    }
}

// ------------------------------------------------------------- cascade pass
struct LowerArgs {
    const int *list_in;
    const int *count_in;
    int *aff;
    int *count_aff;
    uint8_t *order;
    unsigned *stamp;
    unsigned long long *levcnt;
    int nx, ny, bcx, bcy;
    unsigned pass;
    int ncap;       // number of cells: upper bound of every list
    int next[4];    // next radius after r
    int levidx[4];  // cascade level of radius r
};

__device__ __forceinline__ void claim(const LowerArgs &A, int c, bool valid)
{
    bool mine = false;
    if (valid) mine = atomicMax(&A.stamp[c], A.pass) < A.pass;
    wave_append(mine, c, A.aff, A.count_aff);
}

__global__ __launch_bounds__(256) void k_cascade_lower(const LowerArgs A)
{
    int n = *A.count_in;
    n = n < A.ncap ? n : A.ncap;  // a list never holds more than one entry per cell
    if (n <= 0) return;
    const int stride = gridDim.x * blockDim.x;
    const int nround = (n + stride - 1) / stride;
    for (int r = 0; r < nround; ++r) {
        const int idx = r * stride + blockIdx.x * blockDim.x + threadIdx.x;
        const bool valid = idx < n;
        int c = 0, i = 0, j = 0;
        if (valid) {
            c = A.list_in[idx];
            const int o = A.order[c];
            const int o2 = A.next[o];
            A.order[c] = (uint8_t)o2;
            atomicAdd(&A.levcnt[A.levidx[o]], (unsigned long long)-1ll);
            atomicAdd(&A.levcnt[A.levidx[o2]], 1ull);
            i = c % A.nx;
            j = c / A.nx;
        }
        // the cell and its four face neighbours (boundary ghosts map back into the grid)
        claim(A, c, valid);
        const int di[4] = {-1, 1, 0, 0}, dj[4] = {0, 0, -1, 1};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ii = i + di[k], jj = j + dj[k];
            const bool inside_x = A.bcx == 0 || (ii >= 0 && ii < A.nx);
            const bool inside_y = A.bcy == 0 || (jj >= 0 && jj < A.ny);
            const bool ok = valid && inside_x && inside_y;
            const int cc = ok ? remap(jj, A.ny, A.bcy) * A.nx + remap(ii, A.nx, A.bcx) : 0;
            claim(A, cc, ok);
        }
    }
}

// Face states of the cell centred at (ci, cj) (ghost positions allowed) for
// direction DIR at radius R, read from global memory with boundary remaps.
template <typename real, int R, int DIR>
__device__ __forceinline__ void cell_states(const StageArgs<real> &A, int ci, int cj,
                                            real (&sm)[nodes_of(R)][4], real (&sp)[nodes_of(R)][4])
{
    const size_t plane = (size_t)A.nx * A.ny;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const real *U = A.Us + v * plane;
        if constexpr (R == 0) {
            const real x = U[(size_t)remap(cj, A.ny, A.bcy) * A.nx + remap(ci, A.nx, A.bcx)];
            sm[0][v] = x;
            sp[0][v] = x;
        } else {
            real Q[kNQ[R]];
            build_Q<R>(Q, [&](int di, int dj) {
                return U[(size_t)remap(cj + dj, A.ny, A.bcy) * A.nx + remap(ci + di, A.nx, A.bcx)];
            });
            real m_[nodes_of(R)], p_[nodes_of(R)];
            states_dir<R, DIR>(Q, A.W, m_, p_);
#pragma unroll
            for (int k = 0; k < nodes_of(R); ++k) { sm[k][v] = m_[k]; sp[k][v] = p_[k]; }
        }
    }
}

// Flux through the face between cell L = (iL, jL) and cell R (its + neighbour
// along DIR) at radius Rf; same node order and sums as the first pass.
template <typename real, int Rf, int DIR>
__device__ __forceinline__ void face_flux_t(const StageArgs<real> &A, int iL, int jL, real (&F)[4],
                                            bool &badL, bool &badR)
{
    constexpr int q = nodes_of(Rf);
    real lm[q][4], lp[q][4], rm[q][4], rp[q][4];
    cell_states<real, Rf, DIR>(A, iL, jL, lm, lp);
    cell_states<real, Rf, DIR>(A, iL + (DIR == 0), jL + (DIR == 1), rm, rp);
#pragma unroll
    for (int v = 0; v < 4; ++v) F[v] = real(0);
    badL = false;
    badR = false;
#pragma unroll
    for (int k = 0; k < q; ++k) {
        real f[4];
        bool bl, br;
        hllc<DIR>(A.gamma, lp[k], rm[k], f, bl, br);
        badL = badL || bl;
        badR = badR || br;
        const real w = node_weight<Rf>(A.W, k);
#pragma unroll
        for (int v = 0; v < 4; ++v) F[v] = fma(w, f[v], F[v]);
    }
}

// Face flux at a runtime radius.  Everything is inlined into the kernel: device
// function calls are avoided on purpose (a call to a large function also needs
// the scratch stack, and long branches inside such a callee can clobber its return
// address register).
template <typename real, int DIR>
__device__ __forceinline__ void face_flux(const StageArgs<real> &A, int Rf, int iL, int jL, real (&F)[4],
                                          bool &badL, bool &badR)
{
    if (Rf == 3) face_flux_t<real, 3, DIR>(A, iL, jL, F, badL, badR);
    else if (Rf == 2) face_flux_t<real, 2, DIR>(A, iL, jL, F, badL, badR);
    else if (Rf == 1) face_flux_t<real, 1, DIR>(A, iL, jL, F, badL, badR);
    else face_flux_t<real, 0, DIR>(A, iL, jL, F, badL, badR);
}

template <typename real>
__global__ __launch_bounds__(64) void k_cascade_recompute(const StageArgs<real> A, const int *aff,
                                                          const int *count_aff, int ncap)
{
    int n = *count_aff;
    n = n < ncap ? n : ncap;  // a list never holds more than one entry per cell
    if (n <= 0) return;
    const int stride = gridDim.x * blockDim.x;
    const int nround = (n + stride - 1) / stride;
    const int nx = A.nx, ny = A.ny;
    const size_t plane = (size_t)nx * ny;
    const real dt = (real)(*A.dt);
    for (int r = 0; r < nround; ++r) {
        const int idx = r * stride + blockIdx.x * blockDim.x + threadIdx.x;
        const bool valid = idx < n;
        bool tr = false;
        int c = 0;
        if (valid) {
            c = aff[idx];
            const int i = c % nx, j = c / nx;
            const int o = A.order[c];
            const int oW = A.order[(size_t)j * nx + remap(i - 1, nx, A.bcx)];
            const int oE = A.order[(size_t)j * nx + remap(i + 1, nx, A.bcx)];
            const int oS = A.order[(size_t)remap(j - 1, ny, A.bcy) * nx + i];
            const int oN = A.order[(size_t)remap(j + 1, ny, A.bcy) * nx + i];
            real Fm[4], Fp[4], Gm[4], Gp[4];
            bool rs = false;
#pragma unroll 1
            for (int f = 0; f < 4; ++f) {
                real F[4];
                bool bl = false, br = false;
                if (f == 0) face_flux<real, 0>(A, min(o, oW), i - 1, j, F, bl, br);
                else if (f == 1) face_flux<real, 0>(A, min(o, oE), i, j, F, bl, br);
                else if (f == 2) face_flux<real, 1>(A, min(o, oS), i, j - 1, F, bl, br);
                else face_flux<real, 1>(A, min(o, oN), i, j, F, bl, br);
                // the cell owns the right state of its - faces and the left state of its + faces
                rs = rs || ((f & 1) ? bl : br);
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (f == 0) Fm[v] = F[v];
                    else if (f == 1) Fp[v] = F[v];
                    else if (f == 2) Gm[v] = F[v];
                    else Gp[v] = F[v];
                }
            }
            real ust[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const real us = A.Us[v * plane + c];
                const real dFx = Fp[v] - Fm[v];
                ust[v] = us - dt * (dFx / A.dx + (Gp[v] - Gm[v]) / A.dy);
            }
            auto nb = [&](int di, int dj, int v) {
                return A.Us[v * plane + (size_t)remap(j + dj, ny, A.bcy) * nx + remap(i + di, nx, A.bcx)];
            };
            tr = troubled(A, o, ust, rs, nb);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const real un = A.s == 0 ? real(0) : A.Un[v * plane + c];
                A.Uout[v * plane + c] = combine(A.s, un, ust[v]);
            }
        }
        wave_append(tr, c, A.list_out, A.count_out);
    }
}

// -------------------------------------------------------- small kernels
__global__ void k_reset(Ctl *ctl, int top_level, unsigned long long ncell)
{
    const int t = threadIdx.x;
    for (int k = t; k < kMaxPasses + 2; k += blockDim.x) {
        ctl->nlist[k] = 0;
        ctl->naff[k] = 0;
    }
    if (t < 4) ctl->levcnt[t] = t == top_level ? ncell : 0ull;
}

// max over cells of (|u_d| + c) / Delta_d in FP64, as the bit pattern of a
// non-negative double (which orders like the integer).
template <typename real>
__global__ __launch_bounds__(256) void k_dt_reduce(const real *U, size_t ncell, double gamma, double dx,
                                                   double dy, unsigned long long *lam_bits)
{
    __shared__ double red[256];
    double lam = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < ncell; k += (size_t)gridDim.x * blockDim.x) {
        const double r = U[k], mx = U[ncell + k], my = U[2 * ncell + k], E = U[3 * ncell + k];
        const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
        if (!(r > 0.0 && p > 0.0 && __builtin_isfinite(r) && __builtin_isfinite(p))) continue;
        const double cs = sqrt(gamma * p / r);
        const double lx = (fabs(mx / r) + cs) / dx;
        const double ly = (fabs(my / r) + cs) / dy;
        const double l = lx > ly ? lx : ly;
        lam = l > lam ? l : lam;
    }
    red[threadIdx.x] = lam;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] > 0.0) atomicMax(lam_bits, (unsigned long long)__double_as_longlong(red[0]));
}

__global__ void k_dt_finalize(Ctl *ctl, double cfl)
{
    const double lam = __longlong_as_double((long long)ctl->lam_bits);
    ctl->dt = cfl / lam;
}

__global__ void k_dt_set(Ctl *ctl, double dt, int clear_lambda)
{
    if (clear_lambda) ctl->lam_bits = 0ull;
    else ctl->dt = dt;
}

// Compensated totals: per-block double-double partial sums in a fixed order.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void dd_add(double &hi, double &lo, double x)
{
    double s, e;
    two_sum(hi, x, s, e);
    e += lo;
    two_sum(s, e, hi, lo);
}

template <typename real>
__global__ __launch_bounds__(256) void k_totals_partial(const real *U, size_t ncell, double *partial)
{
    __shared__ double sh[256], sl[256];
    const int v = blockIdx.y;
    double hi = 0.0, lo = 0.0;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < ncell; k += (size_t)gridDim.x * blockDim.x)
        dd_add(hi, lo, (double)U[v * ncell + k]);
    sh[threadIdx.x] = hi;
    sl[threadIdx.x] = lo;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            double h = sh[threadIdx.x], l = sl[threadIdx.x];
            dd_add(h, l, sh[threadIdx.x + s]);
            dd_add(h, l, sl[threadIdx.x + s]);
            sh[threadIdx.x] = h;
            sl[threadIdx.x] = l;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[(v * gridDim.x + blockIdx.x) * 2] = sh[0];
        partial[(v * gridDim.x + blockIdx.x) * 2 + 1] = sl[0];
    }
}

__global__ void k_totals_final(const double *partial, int nblk, double area, Ctl *ctl)
{
    const int v = threadIdx.x;
    if (v >= 4) return;
    double hi = 0.0, lo = 0.0;
    for (int b = 0; b < nblk; ++b) {
        dd_add(hi, lo, partial[(v * nblk + b) * 2]);
        dd_add(hi, lo, partial[(v * nblk + b) * 2 + 1]);
    }
    ctl->totals[v] = (hi + lo) * area;
}

// ------------------------------------------------------------- launchers
template <typename real, int RT>
static hipError_t launch_first_pass_rt(const StageArgs<real> &A, hipStream_t st)
{
    constexpr int WPB = sizeof(real) == 8 ? 2 : 4;
    const int nstrip = (A.nx + 61) / 62, nseg = (A.ny + A.rows - 1) / A.rows;
    const int nwave = nstrip * nseg;
    const int nblk = (nwave + WPB - 1) / WPB;
    hipLaunchKernelGGL((k_first_pass<real, RT, WPB>), dim3(nblk), dim3(64 * WPB), 0, st, A);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_first_pass(const StageArgs<real> &A, hipStream_t st)
{
    switch (A.top) {
    case 3: return launch_first_pass_rt<real, 3>(A, st);
    case 2: return launch_first_pass_rt<real, 2>(A, st);
    case 1: return launch_first_pass_rt<real, 1>(A, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_cascade_lower(const LowerArgsHost &h, hipStream_t st)
{
    LowerArgs A;
    A.list_in = h.list_in;
    A.count_in = h.count_in;
    A.aff = h.aff;
    A.count_aff = h.count_aff;
    A.order = h.order;
    A.stamp = h.stamp;
    A.levcnt = h.levcnt;
    A.nx = h.nx;
    A.ny = h.ny;
    A.bcx = h.bcx;
    A.bcy = h.bcy;
    A.pass = h.pass;
    A.ncap = h.nx * h.ny;
    for (int k = 0; k < 4; ++k) {
        A.next[k] = h.next[k];
        A.levidx[k] = h.levidx[k];
    }
    hipLaunchKernelGGL(k_cascade_lower, dim3(h.nblocks), dim3(256), 0, st, A);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_cascade_recompute(const StageArgs<real> &A, const int *aff, const int *count_aff, int nblocks,
                                    hipStream_t st)
{
    hipLaunchKernelGGL(k_cascade_recompute<real>, dim3(nblocks), dim3(64), 0, st, A, aff, count_aff, A.nx * A.ny);
    return hipGetLastError();
}

hipError_t launch_reset(Ctl *ctl, int top_level, unsigned long long ncell, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, st, ctl, top_level, ncell);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_dt(const real *U, size_t ncell, double gamma, double dx, double dy, double cfl, Ctl *ctl,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_dt_set, dim3(1), dim3(1), 0, st, ctl, 0.0, 1);
    size_t nblk = (ncell + 255) / 256;
    if (nblk > 4096) nblk = 4096;
    hipLaunchKernelGGL(k_dt_reduce<real>, dim3((unsigned)nblk), dim3(256), 0, st, U, ncell, gamma, dx, dy,
                       &ctl->lam_bits);
    hipLaunchKernelGGL(k_dt_finalize, dim3(1), dim3(1), 0, st, ctl, cfl);
    return hipGetLastError();
}

hipError_t launch_set_dt(Ctl *ctl, double dt, hipStream_t st)
{
    hipLaunchKernelGGL(k_dt_set, dim3(1), dim3(1), 0, st, ctl, dt, 0);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_totals(const real *U, size_t ncell, double area, double *partial, int nblk, Ctl *ctl,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_totals_partial<real>, dim3(nblk, 4), dim3(256), 0, st, U, ncell, partial);
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, partial, nblk, area, ctl);
    return hipGetLastError();
}

template hipError_t launch_first_pass<float>(const StageArgs<float> &, hipStream_t);
template hipError_t launch_first_pass<double>(const StageArgs<double> &, hipStream_t);
template hipError_t launch_cascade_recompute<float>(const StageArgs<float> &, const int *, const int *, int, hipStream_t);
template hipError_t launch_cascade_recompute<double>(const StageArgs<double> &, const int *, const int *, int, hipStream_t);
template hipError_t launch_dt<float>(const float *, size_t, double, double, double, double, Ctl *, hipStream_t);
template hipError_t launch_dt<double>(const double *, size_t, double, double, double, double, Ctl *, hipStream_t);
template hipError_t launch_totals<float>(const float *, size_t, double, double *, int, Ctl *, hipStream_t);
template hipError_t launch_totals<double>(const double *, size_t, double, double *, int, Ctl *, hipStream_t);

}  // namespace gpm
