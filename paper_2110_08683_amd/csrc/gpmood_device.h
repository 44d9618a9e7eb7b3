// Device-side building blocks of the 2D GP-MOOD stage (internal header, HIP).
//
// Bourgeois & Lee, "GP-MOOD":
//   reconstruction  eq. (gp_reconstructor): state = z^T q over the radius-R diamond,
//                   evaluated in the quarter basis of gpmood_tables.h
//   face quadrature eq. (fvm_F) with the Gauss rules of Table tab:QR-pt-weight
//   Riemann solver  HLLC (the paper cites Toro et al. 1994; textbook form with
//                   Davis wave-speed bounds and Toro's star states)
//   detection       Steps 4-10 of the stepwise algorithm: CAD eq. (CAD) and CAD on
//                   the reconstructed Riemann states, PAD eq. (PAD), CSD eqs. (divV),
//                   (gradP), plateau eq. (plateau), DMP eq. (DMP_RK), u2 eqs.
//                   (u2_curvature), (u2_a), (u2_b) with App. B curvature weights
//   stage combine   eq. (rk3)
//
// Everything here is written with explicit operation order (the library is built
// with -ffp-contract=off and uses fma() only where written), so the first pass
// and the cascade passes produce bit-identical face fluxes for the same face
// order: a face flux is the same number whichever kernel evaluates it, which keeps
// the update exactly conservative.
#ifndef GPMOOD_DEVICE_H
#define GPMOOD_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gpmood_tables.h"

namespace gpm {

constexpr int kMaxPasses = 16384;

// Per-radius quarter-basis weights and Gauss weights, plus the u2 curvature weights.
template <typename real>
struct Weights {
    real w3[2][2][25];
    real w2[2][2][13];
    real w1[2][1][5];
    real qw3[2], qw2[2], qw1;
    real curv[2][3];
};

template <typename real>
struct StageArgs {
    const real *Un;
    const real *Us;
    real *Uout;
    const double *dt;     // device scalar
    const unsigned *stamp0;  // device scalar: claim stamp of the first pass (pass k: + k)
    uint8_t *order;       // GP radius per cell (final after the stage)
    // face fluxes of this stage: x faces [4][ny][nx+1] (face i between cells i-1
    // and i), y faces [4][ny+1][nx]; per face, bit 0 / bit 1: the left (lower) /
    // right (upper) reconstructed state is inadmissible (density or pressure not
    // finite and positive)
    real *FX;
    real *GY;
    uint8_t *FXf;
    uint8_t *GYf;
    unsigned *cstamp;     // claim stamps of cells [nx*ny] and faces [NFX + NFY]
    unsigned *fstamp;
    int nx, ny, bcx, bcy;
    int s;                // RK stage 0..2 of eq. (rk3); 3: general stage (ca, cb, dtf)
    int rows;             // rows per wavefront march (first pass)
    int top;              // top radius
    int iso;              // 1: the y weights are exactly the transposed x weights
    int solver;           // 0 HLLC, 1 HLL
    int slit, si0, si1;   // inflow slit: bit 0 bottom, bit 1 top; its cells si0 <= i < si1
    real slitU[2][4];     // the injected states, bottom and top
    unsigned flags;
    int next[4];          // next radius of the cascade after radius r
    real dx, dy, gamma, sigma_v, sigma_p, plat_thr, delta;
    double dx64, dy64, gamma64;  // the same in FP64 (the dt reduction)
    // general stage (s == 3): U_out = ca B + cb U*, U* = U_s - (dtf dt) F(U_s), B
    // passed as Un; dtf = 1 for the stages of eq. (rk3)
    double dtf;
    real ca, cb;
    Weights<real> W;
    const real *gtab;     // compact cascade weights, kGtabSize values (device)
    const real *gtab_dl;  // their derivative with respect to ell (same layout, no Gauss weights)
};

// Outputs of one evaluation: the troubled count, and the faces and cells that the
// next cascade pass recomputes (claimed with `stamp`, unique per evaluation; the
// kernels set it from the control block).  The counters are updated with
// generic-address atomics and may live in LDS.
struct PassOut {
    int *flist;
    int *fcount;
    int *clist;
    int *ccount;
    int *tcount;
    unsigned stamp;
};

// Device control block (lives in the workspace).
struct Ctl {
    int nface[kMaxPasses + 2];   // faces recomputed by cascade pass k (k >= 1)
    int ncell[kMaxPasses + 2];   // cells re-evaluated by cascade pass k (k >= 1)
    int ntroub[kMaxPasses + 2];  // troubled cells of evaluation k (0: first pass)
    unsigned long long levcnt[4];
    unsigned long long lam_bits;
    double dt;
    double totals[4];
    unsigned long long acc_lev[4];  // instrumentation: summed final-order counts
    unsigned long long acc_iters;   // summed MOOD iterations
    unsigned long long acc_stages;
    // cascade control, written by the pass kernels and the single-workgroup tail
    int nlow;         // cells lowered by the first pass (listed for the deferred claims)
    int tail_end;     // first pass the tail did not run
    int tail_k0;      // first pass left to the tail by the multi-block passes (0: none)
    int tail_back;    // 1: the tail stopped at tail_end because the pass grew large
    int tail_start;   // first pass the tail ran (instrumentation)
    unsigned stamp0;  // claim stamp of this stage's first pass; pass k claims with stamp0 + k
};

// Control of the cascade passes of one stage.  Pass k reads lists [k & 1] with
// counts nface[k], ncell[k] and writes lists [(k + 1) & 1]; its claims carry the
// stamp ctl->stamp0 + k (the first pass: ctl->stamp0).  A multi-block pass whose previous
// evaluation left at most tail_thr troubled cells does nothing and records itself
// in tail_k0: the single-workgroup tail runs from there.  The tail hands back
// (tail_back) at a pass whose previous evaluation left more than back_thr.
struct Cascade {
    int *flist[2];
    int *clist[2];
    Ctl *ctl;
    int tail_thr, back_thr;
};

// ------------------------------------------------------------------ helpers
// Source cell of index i on an axis of n cells with boundary bc: 0 periodic,
// 1 outflow (the edge cell), 2 reflecting wall (the mirror image; an index more
// than n cells outside, which only the unused lanes of a strip reach, is clamped).
__device__ __forceinline__ int remap(int i, int n, int bc)
{
    if (bc == 0) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    if (bc == 2) i = i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// blockIdx -> tile: consecutive tiles go to the same XCD (blocks are dealt to the
// 8 XCDs round robin), so neighbouring strips share halo rows in one L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int per = nb >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// remap() for an index at most one period outside the axis (-n <= i < 2n): the
// cascade reaches at most 4 cells beyond the domain, and periodic and reflecting
// axes have at least 4 cells.  WALLS = false: the build for grids without a
// reflecting axis (or for in-domain indices), which leaves out the mirror branch.
template <bool WALLS = true>
__device__ __forceinline__ int wrap(int i, int n, int bc)
{
    if (bc == 0) return i < 0 ? i + n : (i >= n ? i - n : i);
    if (WALLS && bc == 2) return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Is the gathered cell (i, j) (unwrapped indices) a ghost cell of the inflow slit?
template <typename real>
__device__ __forceinline__ bool in_slit(const StageArgs<real> &A, int i, int j)
{
    return i >= A.si0 && i < A.si1 && (((A.slit & 1) && j < 0) || ((A.slit & 2) && j >= A.ny));
}

// Factor of the momentum normal to an axis in the image of cell index i: -1 when
// a reflecting wall (refl) mirrored the index, which reverses that momentum.
template <typename real>
__device__ __forceinline__ real msign(int i, int n, bool refl)
{
    return refl && (i < 0 || i >= n) ? real(-1) : real(1);
}

// Division of the stage arithmetic: IEEE in FP64 (the parity path), in FP32 the
// hardware reciprocal (1 ulp) times the numerator, about ten times cheaper than a
// correctly rounded division; the FP32 path is checked against the FP64 oracle
// with a stated error, not bitwise.
template <typename real>
__device__ __forceinline__ real dv(real a, real b) { return a / b; }
template <>
__device__ __forceinline__ float dv<float>(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Square root likewise: correctly rounded in FP64, the hardware v_sqrt_f32 (1 ulp)
// in FP32 instead of the compiler's ~12-instruction correctly rounded sequence.
template <typename real>
__device__ __forceinline__ real sq(real a) { return sqrt(a); }
template <>
__device__ __forceinline__ float sq<float>(float a) { return __builtin_amdgcn_sqrtf(a); }

template <typename real>
__device__ __forceinline__ real vmin(real a, real b) { return a < b ? a : b; }
template <typename real>
__device__ __forceinline__ real vmax(real a, real b) { return a > b ? a : b; }
template <typename real>
__device__ __forceinline__ bool finite(real x) { return __builtin_isfinite(x); }
// x is finite and > 0 (a positive normal or subnormal number): one class test
__device__ __forceinline__ bool pos_finite(float x) { return __builtin_amdgcn_classf(x, 0x180); }
__device__ __forceinline__ bool pos_finite(double x) { return __builtin_amdgcn_class(x, 0x180); }

// Ideal-gas pressure from conservative variables (detection form).
template <typename real>
__device__ __forceinline__ real pressure(real g, real r, real mx, real my, real E)
{
    return (g - real(1)) * (E - dv(real(0.5) * (mx * mx + my * my), r));
}

template <int R>
__device__ __forceinline__ constexpr int node_slot(int k)
{
    // table order of nodes: R=3: +g1 +g2 -g2 -g1; R=2: +g 0 -g; R=1: +g -g
    return R == 3 ? ((k == 0 || k == 3) ? 0 : 1) : (R == 2 ? (k == 1 ? 1 : 0) : 0);
}

template <int R, typename real>
__device__ __forceinline__ real node_weight(const Weights<real> &W, int k)
{
    if constexpr (R == 3) return W.qw3[node_slot<3>(k)];
    else if constexpr (R == 2) return W.qw2[node_slot<2>(k)];
    else if constexpr (R == 1) return W.qw1;
    else return real(1);
}

// Pointer into the constant address space (kernel arguments, tables read as such):
// loads through it are scalar and cached in the scalar cache.
template <typename T>
using cptr = const __attribute__((address_space(4))) T *;

template <int R, typename real>
__device__ __forceinline__ real wq(const Weights<real> &W, int dir, int slot, int e)
{
    if constexpr (R == 3) return W.w3[dir][slot][e];
    else if constexpr (R == 2) return W.w2[dir][slot][e];
    else return W.w1[dir][0][e];
}

// The four parity sums of the mirror cells pp = (+a,+b), mp = (-a,+b),
// pm = (+a,-b), mm = (-a,-b), paired along the diagonals so that exchanging the
// axes (pm <-> mp) leaves EE and OO unchanged and swaps OE and EO bit for bit: a
// problem symmetric under x <-> y stays exactly symmetric.
template <typename real>
__device__ __forceinline__ void parity_sums(real pp, real mp, real pm, real mm, real &ee, real &oe, real &eo,
                                            real &oo)
{
    const real s = pp + mm, t = pm + mp, d = pp - mm, u = pm - mp;
    ee = s + t;
    oo = s - t;
    oe = d + u;
    eo = d - u;
}

// Sum of an x and a y term that is not fused with the products that formed them
// (a fused form would round the two axes differently).
template <typename real>
__device__ __forceinline__ real axis_sum(real x, real y)
{
#pragma clang fp contract(off)
    return x + y;
}

// Parity sums Q[e] of one variable's radius-R stencil values; ld(di, dj) returns
// the cell average at offset (di, dj).
template <int R, typename real, typename Load>
__device__ __forceinline__ void build_Q(real (&Q)[kNQ[R]], Load ld)
{
#pragma unroll
    for (int e = 0; e < kNQ[R]; ++e) {
        const int a = kQ[e].a, b = kQ[e].b, c = kQ[e].comp;
        if (a == 0 && b == 0) {
            Q[e] = ld(0, 0);
        } else if (b == 0) {
            if (c == C_EE) Q[e] = ld(a, 0) + ld(-a, 0);
            else Q[e] = ld(a, 0) - ld(-a, 0);
        } else if (a == 0) {
            if (c == C_EE) Q[e] = ld(0, b) + ld(0, -b);
            else Q[e] = ld(0, b) - ld(0, -b);
        } else {
            // four entries per (a, b): EE, OE, EO, OO in that order (see kQ)
            if (c == C_EE) {
                const real pp = ld(a, b), mp = ld(-a, b), pm = ld(a, -b), mm = ld(-a, -b);
                parity_sums(pp, mp, pm, mm, Q[e], Q[e + 1], Q[e + 2], Q[e + 3]);
            }
        }
    }
}

// Index of the transposed entry (b, a) of kQ entry e, with OE and EO exchanged.
constexpr int transposed_entry(int e)
{
    const int c = kQ[e].comp == C_OE ? C_EO : (kQ[e].comp == C_EO ? C_OE : kQ[e].comp);
    for (int k = 0; k < 25; ++k)
        if (kQ[k].a == kQ[e].b && kQ[k].b == kQ[e].a && kQ[k].comp == c) return k;
    return -1;
}

// The 2q face states of one variable for direction DIR (0: x faces, 1: y faces):
// sm[k] on the - face, sp[k] on the + face, node k in table order.  ISO: the grid
// is isotropic (equal spacing and length scale, so the y weights are exactly the
// transposed x weights) and a y face computes what an x face computes on the
// transposed grid: x weight e times the transposed entry, accumulated in the x
// faces' order, so both axes round alike.  Without ISO the y weights are read at
// the transposed entry in the same order (the same bits when they are isotropic).
template <int R, int DIR, bool ISO = false, typename real>
__device__ __forceinline__ void states_dir(const real (&Q)[kNQ[R]], const Weights<real> &W,
                                           real (&sm)[nodes_of(R)], real (&sp)[nodes_of(R)])
{
    constexpr int q = nodes_of(R);
    constexpr int cF = DIR == 0 ? C_OE : C_EO;  // odd across the face
    constexpr int cN = DIR == 0 ? C_EO : C_OE;  // odd along the face (node sign)
#pragma unroll
    for (int p = 0; p < slots_of(R); ++p) {
        real P[4] = {real(0), real(0), real(0), real(0)};
        const bool zero = slot_is_zero(R, p);
#pragma unroll
        for (int e = 0; e < kNQ[R]; ++e) {
            // y faces take the entries in the transposed order in both builds, so an
            // isotropic grid gives the same bits whichever build runs it
            const int et = DIR == 1 ? transposed_entry(e) : e;
            const int c = kQ[et].comp;
            if (zero && (c == cN || c == C_OO)) continue;
            const real w = DIR == 0 ? wq<R>(W, 0, p, e) : (ISO ? wq<R>(W, 0, p, e) : wq<R>(W, 1, p, et));
            P[c] = fma(w, Q[et], P[c]);
        }
        const real A = P[C_EE] + P[cF];
        const real Bm = P[C_EE] - P[cF];
        if (zero) {
            sp[p] = A;
            sm[p] = Bm;
        } else {
            const real C = P[cN] + P[C_OO];
            const real D = P[cN] - P[C_OO];
            sp[p] = A + C;
            sp[q - 1 - p] = A - C;
            sm[p] = Bm + D;
            sm[q - 1 - p] = Bm - D;
        }
    }
}

// Parity sums of the four mirror cells (+-a, +-b) of one variable, as in build_Q.
template <typename real>
__device__ __forceinline__ void parity4(real pp, real mp, real pm, real mm, real (&Q)[4])
{
    parity_sums(pp, mp, pm, mm, Q[C_EE], Q[C_OE], Q[C_EO], Q[C_OO]);
}

// HLLC flux through a face normal to axis DIR.  badL / badR: the density or the
// pressure of the left / right state is not finite and positive (CAD on Riemann
// states: a non-positive value makes the sound speed an invalid square root, and
// either flag troubles both cells of the face).
template <int DIR, typename real>
__device__ __forceinline__ void hllc(real g, const real *UL, const real *UR, real *F, bool &badL, bool &badR)
{
    constexpr int n = 1 + DIR, t = 2 - DIR;
    const real rl = UL[0], irl = dv(real(1), rl), ul = UL[n] * irl, vl = UL[t] * irl, El = UL[3];
    const real rr = UR[0], irr = dv(real(1), rr), ur = UR[n] * irr, vr = UR[t] * irr, Er = UR[3];
    const real pl = (g - real(1)) * (El - real(0.5) * rl * (ul * ul + vl * vl));
    const real pr = (g - real(1)) * (Er - real(0.5) * rr * (ur * ur + vr * vr));
    badL = !(pos_finite(rl) && pos_finite(pl));
    badR = !(pos_finite(rr) && pos_finite(pr));
    const real cl = sq(g * pl * irl), cr = sq(g * pr * irr);
    const real SL = vmin(ul - cl, ur - cr);
    const real SR = vmax(ul + cl, ur + cr);
    const real Ss = dv(pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur), rl * (SL - ul) - rr * (SR - ur));
    const bool useL = Ss >= real(0);
    // star state of the side selected by the sign of S*
    const real rk = useL ? rl : rr, uk = useL ? ul : ur, vk = useL ? vl : vr;
    const real Ek = useL ? El : Er, pk = useL ? pl : pr, Sk = useL ? SL : SR, irk = useL ? irl : irr;
    const real sku = Sk - uk;
    const real fac = dv(rk * sku, Sk - Ss);
    const real fk[4] = {rk * uk, rk * uk * uk + pk, rk * uk * vk, uk * (Ek + pk)};
    const real uc[4] = {rk, rk * uk, rk * vk, Ek};
    const real us[4] = {fac, fac * Ss, fac * vk, fac * (Ek * irk + (Ss - uk) * (Ss + dv(pk, rk * sku)))};
    const real fL[4] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, ul * (El + pl)};
    const real fR[4] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, ur * (Er + pr)};
    const bool takeL = SL >= real(0);
    const bool takeStar = !takeL && (useL || SR > real(0));
    real f[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const real fs = fk[k] + Sk * (us[k] - uc[k]);
        f[k] = takeL ? fL[k] : (takeStar ? fs : fR[k]);
    }
    F[0] = f[0];
    F[n] = f[1];
    F[t] = f[2];
    F[3] = f[3];
}

// HLL flux through a face normal to axis DIR (the solver of the Mach-jet problems,
// after Harten, Lax and van Leer), with HLLC's wave speed bounds: the left or
// right physical flux outside [S_L, S_R], else the flux of the single intermediate
// state, (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L).  badL / badR as
// for hllc.
template <int DIR, typename real>
__device__ __forceinline__ void hll(real g, const real *UL, const real *UR, real *F, bool &badL, bool &badR)
{
    // unfused: the mirrored Riemann problem then gives exactly the mirrored flux,
    // which keeps a mirror-symmetric jet symmetric
#pragma clang fp contract(off)
    constexpr int n = 1 + DIR, t = 2 - DIR;
    const real rl = UL[0], irl = dv(real(1), rl), ul = UL[n] * irl, vl = UL[t] * irl, El = UL[3];
    const real rr = UR[0], irr = dv(real(1), rr), ur = UR[n] * irr, vr = UR[t] * irr, Er = UR[3];
    const real pl = (g - real(1)) * (El - real(0.5) * rl * (ul * ul + vl * vl));
    const real pr = (g - real(1)) * (Er - real(0.5) * rr * (ur * ur + vr * vr));
    badL = !(pos_finite(rl) && pos_finite(pl));
    badR = !(pos_finite(rr) && pos_finite(pr));
    const real cl = sq(g * pl * irl), cr = sq(g * pr * irr);
    const real SL = vmin(ul - cl, ur - cr);
    const real SR = vmax(ul + cl, ur + cr);
    const real fL[4] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, ul * (El + pl)};
    const real fR[4] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, ur * (Er + pr)};
    const real uL[4] = {rl, rl * ul, rl * vl, El};
    const real uR[4] = {rr, rr * ur, rr * vr, Er};
    const real iw = dv(real(1), SR - SL), ss = SL * SR;
    real f[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const real fh = (SR * fL[k] - SL * fR[k] + ss * (uR[k] - uL[k])) * iw;
        f[k] = SL >= real(0) ? fL[k] : (SR <= real(0) ? fR[k] : fh);
    }
    F[0] = f[0];
    F[n] = f[1];
    F[t] = f[2];
    F[3] = f[3];
}

// The scheme's Riemann solver: HLLC, or HLL when HLL is set (a build of its own).
template <int DIR, bool HLL, typename real>
__device__ __forceinline__ void riemann(real g, const real *UL, const real *UR, real *F, bool &badL, bool &badR)
{
    if constexpr (HLL) hll<DIR>(g, UL, UR, F, badL, badR);
    else hllc<DIR>(g, UL, UR, F, badL, badR);
}

// Stage combination of eq. (rk3): U^(1) = U*, hat U^(2) = (3 U^n + U*)/4,
// U^(n+1) = (U^n + 2 U*)/3; s == 3: the general stage ca B + cb U* (ca = 0
// ignores B), un holding B.
template <typename real>
__device__ __forceinline__ real combine(int s, real un, real ust, real ca = real(0), real cb = real(1))
{
    if (s == 0) return ust;
    if (s == 1) return real(0.25) * (real(3) * un + ust);
    if (s == 3) return (ca == real(0) ? real(0) : ca * un) + cb * ust;
    return dv(un + real(2) * ust, real(3));
}

// This lane's index within its wavefront, recomputed where it is used (two
// instructions) rather than kept live, and spilled, across a long loop.
__device__ __forceinline__ int lane_here()
{
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// A value the whole wavefront holds, made scalar.
__device__ __forceinline__ float uniform(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uniform(double x)
{
    const long long b = __builtin_bit_cast(long long, x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll)), hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Detection of one cell (Steps 4-10).  nb(di, dj, v) returns the stage input at
// an offset within radius 2.  Returns true if the candidate is troubled.
template <typename real, typename Nb>
__device__ __forceinline__ bool troubled(const StageArgs<real> &A, int order, const real (&ust)[4],
                                         bool rsbad, Nb nb)
{
    if (order == 0) return false;  // Step 10: the safe scheme is accepted
    const real g = A.gamma;
    const real rho = ust[0];
    const real p = pressure(g, ust[0], ust[1], ust[2], ust[3]);
    if (!(finite(rho) && finite(p))) return true;            // Step 4: CAD
    if ((A.flags & 8u) && rsbad) return true;                // CAD on the Riemann states
    if (!(rho > real(0) && p > real(0))) return true;        // Step 5: PAD
    // DMP bounds over the cell and its face neighbours
    const real rc = nb(0, 0, 0), rW = nb(-1, 0, 0), rE = nb(1, 0, 0), rS = nb(0, -1, 0), rN = nb(0, 1, 0);
    real lo = rc, hi = rc;
    lo = vmin(lo, rW); hi = vmax(hi, rW);
    lo = vmin(lo, rE); hi = vmax(hi, rE);
    lo = vmin(lo, rS); hi = vmax(hi, rS);
    lo = vmin(lo, rN); hi = vmax(hi, rN);
    if (lo <= rho && rho <= hi) return false;                // Step 8: DMP
    if ((A.flags & 2u) && (hi - lo) < A.plat_thr) return false;  // Step 7: plateau
    if (A.flags & 1u) {                                       // Step 6: CSD
        const real pE = pressure(g, rE, nb(1, 0, 1), nb(1, 0, 2), nb(1, 0, 3));
        const real pW = pressure(g, rW, nb(-1, 0, 1), nb(-1, 0, 2), nb(-1, 0, 3));
        const real pN = pressure(g, rN, nb(0, 1, 1), nb(0, 1, 2), nb(0, 1, 3));
        const real pS = pressure(g, rS, nb(0, -1, 1), nb(0, -1, 2), nb(0, -1, 3));
        // 2 dx, 2 dy: the same values in every lane, kept in scalar registers
        const real tdx = uniform(real(2) * A.dx), tdy = uniform(real(2) * A.dy);
        const real divV = dv(dv(nb(1, 0, 1), rE) - dv(nb(-1, 0, 1), rW), tdx) +
                          dv(dv(nb(0, 1, 2), rN) - dv(nb(0, -1, 2), rS), tdy);
        const real gradp = dv(fabs(pE - pW), tdx * vmin(pE, pW)) +
                           dv(fabs(pN - pS), tdy * vmin(pN, pS));
        if (divV >= -A.sigma_v && gradp <= A.sigma_p) return false;
    }
    if (A.flags & 4u) {                                       // Step 9: u2
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const real w0 = A.W.curv[d][0], wa = A.W.curv[d][1], wt = A.W.curv[d][2];
            const int cx[5] = {0, -1, 1, 0, 0}, cy[5] = {0, 0, 0, -1, 1};
            real cmin = real(0), cmax = real(0);
#pragma unroll
            for (int m = 0; m < 5; ++m) {
                const int mi = cx[m], mj = cy[m];
                const real along = d == 0 ? nb(mi - 1, mj, 0) + nb(mi + 1, mj, 0) : nb(mi, mj - 1, 0) + nb(mi, mj + 1, 0);
                const real across = d == 0 ? nb(mi, mj - 1, 0) + nb(mi, mj + 1, 0) : nb(mi - 1, mj, 0) + nb(mi + 1, mj, 0);
                real kap = w0 * nb(mi, mj, 0);
                kap = fma(wa, along, kap);
                kap = fma(wt, across, kap);
                if (m == 0) { cmin = kap; cmax = kap; }
                else { cmin = vmin(cmin, kap); cmax = vmax(cmax, kap); }
            }
            const bool prod = cmin * cmax > -A.delta;
            const bool a = prod && vmax(fabs(cmax), fabs(cmin)) < A.delta;
            const bool b = prod && fabs(cmin) >= real(0.5) * fabs(cmax);
            ok = ok && (a || b);
        }
        if (ok) return false;
    }
    return true;
}

// The cascade's next radius after radius o (n0..n3: the cascade table, held in
// scalar registers; a select chain instead of an indexed load, which would also
// copy the kernel's argument block to the stack).
__device__ __forceinline__ int next_radius(int n0, int n1, int n2, int n3, int o)
{
    return o == 3 ? n3 : (o == 2 ? n2 : (o == 1 ? n1 : n0));
}

// Order this wavefront's LDS writes before its later LDS reads of other lanes'
// data.  The lanes of a wavefront execute in lockstep and LDS serves a wavefront's
// requests in order, so this only keeps the compiler from moving the accesses.
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Add the number of flagged lanes of the wavefront to *count (one atomic per
// wavefront).  Must be reached by all 64 lanes of the wavefront together.
__device__ __forceinline__ void wave_count(bool flag, int *count)
{
    const unsigned long long mask = __ballot(flag);
    if (mask != 0ull && (threadIdx.x & 63) == 0) atomicAdd(count, (int)__popcll(mask));
}

// Reserve n slots per lane (n < 1024) in one list with one atomic per wavefront;
// returns the lane's first slot.  Must be reached by all 64 lanes together.
__device__ __forceinline__ int wave_reserve(int n, int *count)
{
    const int lane = threadIdx.x & 63;
    int incl = n;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
    }
    const int tot = __shfl(incl, 63);
    int b = 0;
    if (lane == 63 && tot != 0) b = atomicAdd(count, tot);
    b = __shfl(b, 63);
    return b + incl - n;
}

// Reserve n slots per lane in two lists at once (n = count0 + 65536 * count1,
// each count below 1024) with one atomic per list and wavefront; returns the
// lane's first slot of each list.  Must be reached by all 64 lanes of the
// wavefront together.
__device__ __forceinline__ void wave_reserve2(int n, int *count0, int *count1, int &base0, int &base1)
{
    const int lane = threadIdx.x & 63;
    int incl = n;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(incl, d);
        if (lane >= d) incl += t;
    }
    const int tot = __shfl(incl, 63);
    int b0 = 0, b1 = 0;
    if (lane == 63 && tot != 0) {  // both issued before either result is used
        b0 = atomicAdd(count0, tot & 0xffff);
        b1 = atomicAdd(count1, tot >> 16);
    }
    b0 = __shfl(b0, 63);
    b1 = __shfl(b1, 63);
    const int excl = incl - n;
    base0 = b0 + (excl & 0xffff);
    base1 = b1 + (excl >> 16);
}

// Device tables of a batch for one stage: per-problem stage arguments, first-pass
// outputs and cascade control, and the block prefixes of the first pass and of
// the dt reduction (problem p owns blocks prefix[p] .. prefix[p+1]-1).
template <typename real>
struct BatchTabs {
    const StageArgs<real> *args;
    const PassOut *pout;
    const Cascade *casc;
    const int *blk;
    const int *dblk;
    int *plan;  // [2][nprob + 1] work-block offsets of the batch's multi-block cascade passes
    int nprob;
    int iso;     // every problem's A.iso is 1
    int walls;   // some problem has a reflecting axis
    int solver;  // the scheme's Riemann solver (shared by the batch)
};

// Arguments of the stage adjoint: A carries U^n, U_s, the frozen final orders of
// the forward stage (A.order), dt and the weights; lam_* are [4][ny][nx] in the
// state precision.  gface: one record per face, the adjoints of both sides'
// quarter accumulators (64 values, state precision) in blocks of 16 per
// (direction, variable), [direction][variable][ny+1][nx+1][16], written by the
// face kernel and gathered by the cells of the faces' stencils; dl64: the FP64 derivative of the compact weight
// table with respect to ell; dl_partial holds one dL/d(ell) partial per tile of
// the cell kernel.
constexpr int kAdjOffsets = 25;  // offsets (da, db) with |da| + |db| <= 3
constexpr int kAdjTile = 16;     // the cell kernel's tiles: kAdjTile x kAdjTile cells
template <typename real>
struct AdjArgs {
    StageArgs<real> A;
    const real *lam_out;
    real *lam_Us;
    real *lam_Un;
    real *gface;
    const double *dl64;
    double *dl_partial;
};

struct LevIdx {
    int v[4];  // cascade level of radius r
};

}  // namespace gpm

#endif
