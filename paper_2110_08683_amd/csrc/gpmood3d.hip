// 3D GP-MOOD stage (GP-MOOD5 and lower) for gfx950, with its C ABI (gpm3_*).
//
// The 3D form of the method (3D is future work in the paper; readings as in the
// 3D oracle): five conservative variables (rho, rho u, rho v, rho w, E), the GP
// stencil of radius R <= 2 is the L1 ball (7 / 25 cells), a face carries the q x q
// tensor Gauss nodes (q = R + 1), EDP_1 face orders, HLLC with two tangential
// momenta, detection with the six face neighbours (DMP, plateau, CSD with the z
// terms, u2 per direction), SSP-RK3 (eq. (rk3)), FP64 CFL dt.
//
// Kernels:
//   k3_faces  one thread per face: both cells' node states at the face's EDP_1
//             radius (dot products with the quad-precision weights), q^2 HLLC
//             solves, the Gauss sum; flux and Riemann-state flags stored.  The
//             first pass runs every face at the top radius, cascade passes the
//             claimed faces.
//   k3_cells  one thread per cell: candidate from the six stored fluxes,
//             detection, RK combination, lowering and claims (stamps, one atomic
//             per wavefront and list) of the faces and cells of the next pass.
// The MOOD loop is the synchronous iteration of the 2D engine: a pass recomputes
// the claimed faces, then re-evaluates the claimed cells, until no cell is
// troubled.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gp_weights.h"
#include "gpmood.h"
#include "gpmood_device.h"

namespace gpm {

constexpr int kZ3 = 6 * 9 * 25;  // weights per radius: [6 faces][9 nodes][25 cells]
constexpr int kPZ3 = 6 * 4 * kNPar3;  // radius-2 parity weights: [6 faces][4 node classes][25 entries]

template <typename real>
struct Stage3 {
    const real *Un;
    const real *Us;
    real *Uout;
    const double *dt;
    uint8_t *order;
    real *F[3];          // per axis a: [5][nz + (a == 2)][ny + (a == 1)][nx + (a == 0)]
    uint8_t *Ff[3];      // bit 0 / 1: the left / right state is inadmissible
    unsigned *cstamp;    // [ncell]
    unsigned *fstamp;    // [all faces, axes concatenated]
    int n[3], bc[3];
    int fofs[4];         // first face id of each axis, total
    int s, top;
    unsigned flags;
    int next[4];
    real d[3], gamma, sigma_v, sigma_p, plat_thr, delta;
    const real *z;       // [R - 1][6][9][25]
    const real *qw;      // [R - 1][9]
    const real *pz;      // [6][4][25]: radius 2 in the parity basis (kPar3)
    real curv[3][4];
    const unsigned *stamp0;
};

struct PassOut3 {
    int *flist, *fcount, *clist, *ccount, *tcount;
    unsigned stamp;
};

__device__ __forceinline__ int w3(int i, int n, int bc)
{
    if (bc == 0) return i < 0 ? i + n : (i >= n ? i - n : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

template <typename real>
__device__ __forceinline__ size_t cell3(const Stage3<real> &S, int i, int j, int k)
{
    return ((size_t)w3(k, S.n[2], S.bc[2]) * S.n[1] + w3(j, S.n[1], S.bc[1])) * S.n[0] + w3(i, S.n[0], S.bc[0]);
}

template <typename real>
__device__ __forceinline__ real p3(real g, const real (&q)[5])
{
    return (g - real(1)) * (q[4] - dv(real(0.5) * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]), q[0]));
}

// HLLC with normal axis a (1 + a is the normal momentum), as the 2D solver with a
// second tangential momentum.
template <typename real>
__device__ __forceinline__ void hllc3(real g, int a, const real (&UL)[5], const real (&UR)[5], real (&F)[5],
                                      bool &badL, bool &badR)
{
    const int n = 1 + a, t1 = 1 + (a + 1) % 3, t2 = 1 + (a + 2) % 3;
    const real rl = UL[0], irl = dv(real(1), rl), ul = UL[n] * irl, vl = UL[t1] * irl, wl = UL[t2] * irl, El = UL[4];
    const real rr = UR[0], irr = dv(real(1), rr), ur = UR[n] * irr, vr = UR[t1] * irr, wr = UR[t2] * irr, Er = UR[4];
    const real pl = (g - real(1)) * (El - real(0.5) * rl * (ul * ul + vl * vl + wl * wl));
    const real pr = (g - real(1)) * (Er - real(0.5) * rr * (ur * ur + vr * vr + wr * wr));
    badL = !(pos_finite(rl) && pos_finite(pl));
    badR = !(pos_finite(rr) && pos_finite(pr));
    const real cl = sq(g * pl * irl), cr = sq(g * pr * irr);
    const real SL = vmin(ul - cl, ur - cr);
    const real SR = vmax(ul + cl, ur + cr);
    const real Ss = dv(pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur), rl * (SL - ul) - rr * (SR - ur));
    const bool useL = Ss >= real(0);
    const real rk = useL ? rl : rr, uk = useL ? ul : ur, vk = useL ? vl : vr, wk = useL ? wl : wr;
    const real Ek = useL ? El : Er, pk = useL ? pl : pr, Sk = useL ? SL : SR, irk = useL ? irl : irr;
    const real sku = Sk - uk;
    const real fac = dv(rk * sku, Sk - Ss);
    const real fk[5] = {rk * uk, rk * uk * uk + pk, rk * uk * vk, rk * uk * wk, uk * (Ek + pk)};
    const real uc[5] = {rk, rk * uk, rk * vk, rk * wk, Ek};
    const real us[5] = {fac, fac * Ss, fac * vk, fac * wk, fac * (Ek * irk + (Ss - uk) * (Ss + dv(pk, rk * sku)))};
    const real fL[5] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, rl * ul * wl, ul * (El + pl)};
    const real fR[5] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, rr * ur * wr, ur * (Er + pr)};
    const bool takeL = SL >= real(0);
    const bool takeStar = !takeL && (useL || SR > real(0));
    real f[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) {
        const real fs = fk[m] + Sk * (us[m] - uc[m]);
        f[m] = takeL ? fL[m] : (takeStar ? fs : fR[m]);
    }
    F[0] = f[0];
    F[4] = f[4];
#pragma unroll
    for (int m = 1; m < 4; ++m) F[m] = m == n ? f[1] : (m == t1 ? f[2] : f[3]);
}

// Decode a face id: axis a, and the cell (i, j, k) on its + side (the left cell is
// one step back along a).
template <typename real>
__device__ __forceinline__ void face3_decode(const Stage3<real> &S, int f, int &a, int &i, int &j, int &k, int &loc)
{
    a = f < S.fofs[1] ? 0 : (f < S.fofs[2] ? 1 : 2);
    loc = f - S.fofs[a];
    const int m0 = S.n[0] + (a == 0), m1 = S.n[1] + (a == 1);
    i = loc % m0;
    const int r = loc / m0;
    j = r % m1;
    k = r / m1;
}

template <typename real>
__device__ __forceinline__ void face3_flux(const Stage3<real> &S, int f)
{
    int a, i, j, k, loc;
    face3_decode(S, f, a, i, j, k, loc);
    const int iL = i - (a == 0), jL = j - (a == 1), kL = k - (a == 2);
    const int R = min((int)S.order[cell3(S, iL, jL, kL)], (int)S.order[cell3(S, i, j, k)]);
    const size_t plane = (size_t)S.n[0] * S.n[1] * S.n[2];
    real Fs[5] = {real(0), real(0), real(0), real(0), real(0)};
    bool bl = false, br = false;
    if (R <= 0) {
        real UL[5], UR[5];
        const size_t cl = cell3(S, iL, jL, kL), cr = cell3(S, i, j, k);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            UL[v] = S.Us[v * plane + cl];
            UR[v] = S.Us[v * plane + cr];
        }
        real fl[5];
        hllc3(S.gamma, a, UL, UR, fl, bl, br);
#pragma unroll
        for (int v = 0; v < 5; ++v) Fs[v] = fma(real(1), fl[v], real(0));
    } else {
        const int ns = R == 1 ? 7 : 25, nq = R == 1 ? 4 : 9;
        const real *zL = S.z + ((size_t)(R - 1) * 6 + 2 * a + 1) * 9 * 25;  // + face of the left cell
        const real *zR = S.z + ((size_t)(R - 1) * 6 + 2 * a) * 9 * 25;      // - face of the right cell
        real st[9][2][5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            real qL[25], qR[25];
#pragma unroll
            for (int m = 0; m < 25; ++m) {
                if (m < ns) {
                    qL[m] = S.Us[v * plane + cell3(S, iL + kBall[m][0], jL + kBall[m][1], kL + kBall[m][2])];
                    qR[m] = S.Us[v * plane + cell3(S, i + kBall[m][0], j + kBall[m][1], k + kBall[m][2])];
                } else {
                    qL[m] = qR[m] = real(0);
                }
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                real sl = real(0), sr = real(0);
                if (q < nq) {
#pragma unroll
                    for (int m = 0; m < 25; ++m)
                        if (m < ns) {
                            sl = fma(zL[q * 25 + m], qL[m], sl);
                            sr = fma(zR[q * 25 + m], qR[m], sr);
                        }
                }
                st[q][0][v] = sl;
                st[q][1][v] = sr;
            }
        }
        const real *w = S.qw + (size_t)(R - 1) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            if (q < nq) {
                real fl[5];
                bool b1, b2;
                hllc3(S.gamma, a, st[q][0], st[q][1], fl, b1, b2);
                bl = bl || b1;
                br = br || b2;
#pragma unroll
                for (int v = 0; v < 5; ++v) Fs[v] = fma(w[q], fl[v], Fs[v]);
            }
        }
    }
    const int m0 = S.n[0] + (a == 0), m1 = S.n[1] + (a == 1), m2 = S.n[2] + (a == 2);
    const size_t nfa = (size_t)m0 * m1 * m2;
#pragma unroll
    for (int v = 0; v < 5; ++v) S.F[a][v * nfa + loc] = Fs[v];
    S.Ff[a][loc] = (uint8_t)((bl ? 1 : 0) | (br ? 2 : 0));
}

template <typename real>
__global__ __launch_bounds__(128) void k3_faces(const Stage3<real> S, const int *list, const int *count, int all)
{
    const int cap = S.fofs[3];
    int n = all ? cap : *count;
    n = n < cap ? n : cap;
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x)
        face3_flux(S, all ? t : list[t]);
}

// First evaluation: every face of axis A at the top radius R (every cell starts the
// stage at the top order), with the products and sums of face3_flux in the same
// order.  All 2 x 5 stencils are loaded once into registers; the node loop is
// rolled and reads each node's 2 x 25 weights through the scalar path (R and A
// are uniform), so no lane loads a weight.
template <typename real, int R, int A>
__global__ __launch_bounds__(128, 1) void k3_faces_top(const Stage3<real> S)
{
    constexpr int ns = R == 1 ? 7 : 25, nq = R == 1 ? 4 : 9;
    const int m0 = S.n[0] + (A == 0), m1 = S.n[1] + (A == 1), m2 = S.n[2] + (A == 2);
    const int nfa = m0 * m1 * m2;
    const int loc = blockIdx.x * blockDim.x + threadIdx.x;
    if (loc >= nfa) return;
    const size_t plane = (size_t)S.n[0] * S.n[1] * S.n[2];
    const int i = loc % m0, rr = loc / m0, j = rr % m1, k = rr / m1;
    const int iL = i - (A == 0), jL = j - (A == 1), kL = k - (A == 2);
    real qL[5][ns], qR[5][ns];
#pragma unroll
    for (int m = 0; m < ns; ++m) {
        const size_t cl = cell3(S, iL + kBall[m][0], jL + kBall[m][1], kL + kBall[m][2]);
        const size_t cr = cell3(S, i + kBall[m][0], j + kBall[m][1], k + kBall[m][2]);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            qL[v][m] = S.Us[v * plane + cl];
            qR[v][m] = S.Us[v * plane + cr];
        }
    }
    const cptr<real> zL = (cptr<real>)S.z + ((R - 1) * 6 + 2 * A + 1) * 9 * 25;  // + face of the left cell
    const cptr<real> zR = (cptr<real>)S.z + ((R - 1) * 6 + 2 * A) * 9 * 25;      // - face of the right cell
    const cptr<real> w = (cptr<real>)S.qw + (R - 1) * 9;
    real Fs[5] = {real(0), real(0), real(0), real(0), real(0)};
    bool bl = false, br = false;
#pragma unroll 1
    for (int q = 0; q < nq; ++q) {
        real sl[5], sr[5];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            real a = real(0), b = real(0);
#pragma unroll
            for (int m = 0; m < ns; ++m) {
                a = fma(zL[q * 25 + m], qL[v][m], a);
                b = fma(zR[q * 25 + m], qR[v][m], b);
            }
            sl[v] = a;
            sr[v] = b;
        }
        real fl[5];
        bool b1, b2;
        hllc3(S.gamma, A, sl, sr, fl, b1, b2);
        bl = bl || b1;
        br = br || b2;
#pragma unroll
        for (int v = 0; v < 5; ++v) Fs[v] = fma(w[q], fl[v], Fs[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) S.F[A][(size_t)v * nfa + loc] = Fs[v];
    S.Ff[A][loc] = (uint8_t)((bl ? 1 : 0) | (br ? 2 : 0));
}

// Radius 2 in the parity basis: one thread per face; per variable, each side's 25
// ball values are folded into the 25 parity entries of the face axis (kPar3) and
// the nine node states come from the four node classes' weights: 14 products for
// the centre, 19 for each pair on a tangential axis, 25 for the four corners (77,
// against 225 for nine 25-term dot products).  The weights are the orbit
// averages of the quad-precision prediction vectors; the node states agree with
// the plain dot products to rounding.
template <int A>
__device__ __forceinline__ constexpr int par_member(int e, int s1, int s2)
{
    const int t1 = A == 0 ? 1 : 0, t2 = A == 2 ? 1 : 2;
    int d[3] = {0, 0, 0};
    d[A] = kPar3[e].dn;
    d[t1] = s1 * kPar3[e].a1;
    d[t2] = s2 * kPar3[e].a2;
    return ball_index(d[0], d[1], d[2]);
}

template <int A, typename real>
__device__ __forceinline__ void par3_entries(const real (&q)[25], real (&P)[kNPar3])
{
#pragma unroll
    for (int e = 0; e < kNPar3; ++e) {
        const int a1 = kPar3[e].a1, a2 = kPar3[e].a2, c = kPar3[e].comp;
        const real pp = q[par_member<A>(e, 1, 1)];
        if (a1 == 0 && a2 == 0) {
            P[e] = pp;
        } else if (a2 == 0) {
            const real mp = q[par_member<A>(e, -1, 1)];
            P[e] = c == 0 ? pp + mp : pp - mp;
        } else if (a1 == 0) {
            const real pm = q[par_member<A>(e, 1, -1)];
            P[e] = c == 0 ? pp + pm : pp - pm;
        } else {
            const real mp = q[par_member<A>(e, -1, 1)], pm = q[par_member<A>(e, 1, -1)];
            const real mm = q[par_member<A>(e, -1, -1)];
            P[e] = c == 0 ? (pp + mp) + (pm + mm)
                 : c == 1 ? (pp - mp) + (pm - mm)
                 : c == 2 ? (pp + mp) - (pm + mm)
                          : (pp - mp) - (pm - mm);
        }
    }
}

// The nine node states (table order) of one face side from its parity entries.
template <typename real>
__device__ __forceinline__ void par3_states(const real (&P)[kNPar3], cptr<real> W, real (&s)[9])
{
    real c0 = real(0), a1 = real(0), a2 = real(0), a3 = real(0);
#pragma unroll
    for (int e = 0; e < kPar3EE; ++e) {
        c0 = fma(W[e], P[e], c0);
        a1 = fma(W[kNPar3 + e], P[e], a1);
        a2 = fma(W[2 * kNPar3 + e], P[e], a2);
        a3 = fma(W[3 * kNPar3 + e], P[e], a3);
    }
    real b1 = real(0), b3 = real(0);
#pragma unroll
    for (int e = kPar3EE; e < kPar3EE + kPar3OE; ++e) {
        b1 = fma(W[kNPar3 + e], P[e], b1);
        b3 = fma(W[3 * kNPar3 + e], P[e], b3);
    }
    real c2 = real(0), c3 = real(0);
#pragma unroll
    for (int e = kPar3EE + kPar3OE; e < kNPar3 - 1; ++e) {
        c2 = fma(W[2 * kNPar3 + e], P[e], c2);
        c3 = fma(W[3 * kNPar3 + e], P[e], c3);
    }
    const real d3 = W[3 * kNPar3 + kNPar3 - 1] * P[kNPar3 - 1];
    s[4] = c0;
    s[1] = a1 + b1;
    s[7] = a1 - b1;
    s[3] = a2 + c2;
    s[5] = a2 - c2;
    s[0] = (a3 + b3) + (c3 + d3);
    s[2] = (a3 + b3) - (c3 + d3);
    s[6] = (a3 - b3) + (c3 - d3);
    s[8] = (a3 - b3) - (c3 - d3);
}

// Node states of both sides of face (i, j, k) of axis A (left cell (iL, jL, kL)).
// IN: both balls lie inside the grid (offsets from the cell index, no mapping).
template <int A, bool IN, typename real>
__device__ __forceinline__ void top2_states(const Stage3<real> &S, int i, int j, int k, real (&sl)[9][5],
                                            real (&sr)[9][5])
{
    const size_t plane = (size_t)S.n[0] * S.n[1] * S.n[2];
    const int iL = i - (A == 0), jL = j - (A == 1), kL = k - (A == 2);
    const int sy = S.n[0], sz = S.n[0] * S.n[1];
    const cptr<real> WL = (cptr<real>)S.pz + (2 * A + 1) * 4 * kNPar3;  // + face of the left cell
    const cptr<real> WR = (cptr<real>)S.pz + (2 * A) * 4 * kNPar3;      // - face of the right cell
#pragma unroll
    for (int v = 0; v < 5; ++v) {
        // one variable's loads at a time: the node states of all five stay live
        __builtin_amdgcn_sched_barrier(0);
        const real *U = S.Us + v * plane;
        // the weights are reloaded (scalar loads) for each variable rather than
        // held in scalar registers across all five
        cptr<real> WLv = WL, WRv = WR;
        asm volatile("" : "+s"(WLv), "+s"(WRv));
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int ci = side == 0 ? iL : i, cj = side == 0 ? jL : j, ck = side == 0 ? kL : k;
            real q[25], P[kNPar3], st[9];
            if constexpr (IN) {
                const real *c0 = U + ((size_t)ck * S.n[1] + cj) * S.n[0] + ci;
#pragma unroll
                for (int m = 0; m < 25; ++m) q[m] = c0[kBall[m][2] * sz + kBall[m][1] * sy + kBall[m][0]];
            } else {
#pragma unroll
                for (int m = 0; m < 25; ++m) q[m] = U[cell3(S, ci + kBall[m][0], cj + kBall[m][1], ck + kBall[m][2])];
            }
            par3_entries<A>(q, P);
            par3_states(P, side == 0 ? WLv : WRv, st);
#pragma unroll
            for (int n = 0; n < 9; ++n) {
                if (side == 0) sl[n][v] = st[n];
                else sr[n][v] = st[n];
            }
        }
    }
}

template <typename real, int A>
__global__ __launch_bounds__(128) void k3_faces_top2(const Stage3<real> S)
{
    const int m0 = S.n[0] + (A == 0), m1 = S.n[1] + (A == 1), m2 = S.n[2] + (A == 2);
    const int nfa = m0 * m1 * m2;
    const int loc = blockIdx.x * blockDim.x + threadIdx.x;
    if (loc >= nfa) return;
    const int i = loc % m0, rr = loc / m0, j = rr % m1, k = rr / m1;
    const int lo[3] = {i - (A == 0), j - (A == 1), k - (A == 2)}, hi[3] = {i, j, k};
    bool inside = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) inside = inside && lo[d] >= 2 && hi[d] + 2 < S.n[d];
    real sl[9][5], sr[9][5];
    if (inside) top2_states<A, true>(S, i, j, k, sl, sr);
    else top2_states<A, false>(S, i, j, k, sl, sr);
    const cptr<real> w = (cptr<real>)S.qw + 9;
    real Fs[5] = {real(0), real(0), real(0), real(0), real(0)};
    bool bl = false, br = false;
#pragma unroll
    for (int n = 0; n < 9; ++n) {
        real fl[5];
        bool b1, b2;
        hllc3(S.gamma, A, sl[n], sr[n], fl, b1, b2);
        bl = bl || b1;
        br = br || b2;
#pragma unroll
        for (int v = 0; v < 5; ++v) Fs[v] = fma(w[n], fl[v], Fs[v]);
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) S.F[A][(size_t)v * nfa + loc] = Fs[v];
    S.Ff[A][loc] = (uint8_t)((bl ? 1 : 0) | (br ? 2 : 0));
}

template <typename real, int R>
static void launch_faces_top(const Stage3<real> &S, hipStream_t st)
{
    for (int a = 0; a < 3; ++a) {
        const long long nfa = (long long)(S.n[0] + (a == 0)) * (S.n[1] + (a == 1)) * (S.n[2] + (a == 2));
        const dim3 g((unsigned)((nfa + 127) / 128)), t(128);
        if constexpr (R == 2) {
            if (a == 0) hipLaunchKernelGGL((k3_faces_top2<real, 0>), g, t, 0, st, S);
            if (a == 1) hipLaunchKernelGGL((k3_faces_top2<real, 1>), g, t, 0, st, S);
            if (a == 2) hipLaunchKernelGGL((k3_faces_top2<real, 2>), g, t, 0, st, S);
        } else {
            if (a == 0) hipLaunchKernelGGL((k3_faces_top<real, R, 0>), g, t, 0, st, S);
            if (a == 1) hipLaunchKernelGGL((k3_faces_top<real, R, 1>), g, t, 0, st, S);
            if (a == 2) hipLaunchKernelGGL((k3_faces_top<real, R, 2>), g, t, 0, st, S);
        }
    }
}

// Face id of axis a at cell (i, j, k) (the - face; + face: the next index along a).
template <typename real>
__device__ __forceinline__ int face3_id(const Stage3<real> &S, int a, int i, int j, int k)
{
    const int m0 = S.n[0] + (a == 0), m1 = S.n[1] + (a == 1);
    return S.fofs[a] + (k * m1 + j) * m0 + i;
}

template <typename real>
__device__ __forceinline__ void claims3(const Stage3<real> &S, const PassOut3 &P, int i, int j, int k, bool act)
{
    int fid[9];
    bool fok[9];
    const int c3[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int ip = i + (a == 0), jp = j + (a == 1), kp = k + (a == 2);
        fid[2 * a] = face3_id(S, a, i, j, k);
        fid[2 * a + 1] = face3_id(S, a, ip, jp, kp);
        fok[2 * a] = fok[2 * a + 1] = true;
        // periodic axis: the boundary face has a second copy at the other end
        const bool lo = c3[a] == 0, hi = c3[a] == S.n[a] - 1;
        fok[6 + a] = S.bc[a] == 0 && (lo || hi);
        const int e = lo ? S.n[a] : 0;
        fid[6 + a] = fok[6 + a] ? face3_id(S, a, a == 0 ? e : i, a == 1 ? e : j, a == 2 ? e : k) : fid[2 * a];
    }
    int cid[7];
    bool cok[7];
#pragma unroll
    for (int m = 0; m < 7; ++m) {
        const int ii = i + kBall[m][0], jj = j + kBall[m][1], kk = k + kBall[m][2];
        cok[m] = (S.bc[0] == 0 || (ii >= 0 && ii < S.n[0])) && (S.bc[1] == 0 || (jj >= 0 && jj < S.n[1])) &&
                 (S.bc[2] == 0 || (kk >= 0 && kk < S.n[2]));
        cid[m] = cok[m] ? (int)cell3(S, ii, jj, kk) : (int)cell3(S, i, j, k);
    }
    bool fmine[9], cmine[7];
    int nmine = 0;
    if (act) {
        unsigned fo[9], co[7];
#pragma unroll
        for (int m = 0; m < 9; ++m) fo[m] = atomicMax(&S.fstamp[fid[m]], fok[m] ? P.stamp : 0u);
#pragma unroll
        for (int m = 0; m < 7; ++m) co[m] = atomicMax(&S.cstamp[cid[m]], cok[m] ? P.stamp : 0u);
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            fmine[m] = fok[m] && fo[m] < P.stamp;
            nmine += fmine[m] ? 1 : 0;
        }
#pragma unroll
        for (int m = 0; m < 7; ++m) {
            cmine[m] = cok[m] && co[m] < P.stamp;
            nmine += cmine[m] ? 65536 : 0;
        }
    } else {
#pragma unroll
        for (int m = 0; m < 9; ++m) fmine[m] = false;
#pragma unroll
        for (int m = 0; m < 7; ++m) cmine[m] = false;
    }
    int fb, cb;
    wave_reserve2(nmine, P.fcount, P.ccount, fb, cb);
    if (nmine != 0) {
#pragma unroll
        for (int m = 0; m < 9; ++m)
            if (fmine[m]) P.flist[fb++] = fid[m];
#pragma unroll
        for (int m = 0; m < 7; ++m)
            if (cmine[m]) P.clist[cb++] = cid[m];
    }
}

template <typename real>
__device__ __forceinline__ bool troubled3(const Stage3<real> &S, int o, const real (&ust)[5], bool rs, int i, int j,
                                          int k)
{
    if (o == 0) return false;
    const size_t plane = (size_t)S.n[0] * S.n[1] * S.n[2];
    const real g = S.gamma;
    const real rho = ust[0], p = p3(g, ust);
    if (!(finite(rho) && finite(p))) return true;
    if ((S.flags & 8u) && rs) return true;
    if (!(rho > real(0) && p > real(0))) return true;
    real r25[25];
#pragma unroll
    for (int m = 0; m < 25; ++m) r25[m] = S.Us[cell3(S, i + kBall[m][0], j + kBall[m][1], k + kBall[m][2])];
    real lo = r25[0], hi = r25[0];
#pragma unroll
    for (int m = 1; m < 7; ++m) {
        lo = vmin(lo, r25[m]);
        hi = vmax(hi, r25[m]);
    }
    if (lo <= rho && rho <= hi) return false;                   // DMP
    if ((S.flags & 2u) && (hi - lo) < S.plat_thr) return false;  // plateau
    if (S.flags & 1u) {                                          // CSD
        real divV = real(0), gradp = real(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            real qp[5], qm[5];
            const size_t cp = cell3(S, i + (a == 0), j + (a == 1), k + (a == 2));
            const size_t cm = cell3(S, i - (a == 0), j - (a == 1), k - (a == 2));
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                qp[v] = S.Us[v * plane + cp];
                qm[v] = S.Us[v * plane + cm];
            }
            divV = divV + (qp[1 + a] / qp[0] - qm[1 + a] / qm[0]) / (real(2) * S.d[a]);
            const real pp = p3(g, qp), pm = p3(g, qm);
            gradp = gradp + fabs(pp - pm) / (real(2) * S.d[a] * vmin(pp, pm));
        }
        if (divV >= -S.sigma_v && gradp <= S.sigma_p) return false;
    }
    if (S.flags & 4u) {  // u2
        // index in kBall of the offset (di, dj, dk) with |di|+|dj|+|dk| <= 2
        auto at = [&](int di, int dj, int dk) {
            int r = 0;
#pragma unroll
            for (int m = 0; m < 25; ++m)
                if (kBall[m][0] == di && kBall[m][1] == dj && kBall[m][2] == dk) r = m;
            return r25[r];
        };
        bool ok = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            real cmin = real(0), cmax = real(0);
#pragma unroll
            for (int m = 0; m < 7; ++m) {
                const int mi = kBall[m][0], mj = kBall[m][1], mk = kBall[m][2];
                real kap = S.curv[d][0] * at(mi, mj, mk);
                int slot = 2;
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    const int ex = e == 0, ey = e == 1, ez = e == 2;
                    const real pair = at(mi + ex, mj + ey, mk + ez) + at(mi - ex, mj - ey, mk - ez);
                    if (e == d) kap = fma(S.curv[d][1], pair, kap);
                    else kap = fma(S.curv[d][slot++], pair, kap);
                }
                if (m == 0) {
                    cmin = kap;
                    cmax = kap;
                } else {
                    cmin = vmin(cmin, kap);
                    cmax = vmax(cmax, kap);
                }
            }
            const bool pr = cmin * cmax > -S.delta;
            const bool a_ = pr && vmax(fabs(cmax), fabs(cmin)) < S.delta;
            const bool b_ = pr && fabs(cmin) >= real(0.5) * fabs(cmax);
            ok = ok && (a_ || b_);
        }
        if (ok) return false;
    }
    return true;
}

template <typename real>
__global__ __launch_bounds__(128) void k3_cells(const Stage3<real> S, const int *list, const int *count, int all,
                                                PassOut3 P)
{
    const int nc = S.n[0] * S.n[1] * S.n[2];
    int n = all ? nc : *count;
    n = n < nc ? n : nc;
    if (n <= (int)(blockIdx.x * blockDim.x)) return;
    P.stamp = *S.stamp0 + P.stamp;  // P.stamp carries the pass index
    const size_t plane = (size_t)nc;
    const real dt = (real)(*S.dt);
    const int stride = gridDim.x * blockDim.x;
    const int nround = (n + stride - 1) / stride;
    for (int r = 0; r < nround; ++r) {
        const int idx = r * stride + blockIdx.x * blockDim.x + threadIdx.x;
        bool tr = false;
        int i = 0, j = 0, k = 0;
        if (idx < n) {
            const int c = all ? idx : list[idx];
            i = c % S.n[0];
            j = (c / S.n[0]) % S.n[1];
            k = c / (S.n[0] * S.n[1]);
            real ust[5];
            real div[5] = {real(0), real(0), real(0), real(0), real(0)};
            // every flux, flag and state value of the cell loaded first, then one
            // wait (the flag tests and the divisions had split the loads by axis)
            real fpv[3][5], fmv[3][5], us[5];
            int fl = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int m0 = S.n[0] + (a == 0), m1 = S.n[1] + (a == 1), m2 = S.n[2] + (a == 2);
                const size_t nfa = (size_t)m0 * m1 * m2;
                const int fm = (k * m1 + j) * m0 + i;
                const int fp = ((k + (a == 2)) * m1 + j + (a == 1)) * m0 + i + (a == 0);
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    fpv[a][v] = S.F[a][v * nfa + fp];
                    fmv[a][v] = S.F[a][v * nfa + fm];
                }
                fl |= S.Ff[a][fm] | S.Ff[a][fp];  // either side of either face
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) us[v] = S.Us[v * plane + c];
            const int o = S.order[c];
            __builtin_amdgcn_sched_barrier(0);
            const bool rs = fl != 0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int v = 0; v < 5; ++v) div[v] = div[v] + (fpv[a][v] - fmv[a][v]) / S.d[a];
#pragma unroll
            for (int v = 0; v < 5; ++v) ust[v] = us[v] - dt * div[v];
            tr = troubled3(S, o, ust, rs, i, j, k);
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const real un = S.s == 0 ? real(0) : S.Un[v * plane + c];
                S.Uout[v * plane + c] = combine(S.s, un, ust[v]);
            }
            if (tr) S.order[c] = (uint8_t)next_radius(S.next[0], S.next[1], S.next[2], S.next[3], o);
        }
        wave_count(tr, P.tcount);
        claims3(S, P, i, j, k, tr);
    }
}

__global__ void k3_fill_order(uint8_t *order, size_t n, int top)
{
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x)
        order[t] = (uint8_t)top;
}

__global__ void k3_reset(Ctl *ctl, int nzero, unsigned stamp0)
{
    for (int k = threadIdx.x; k < nzero && k < kMaxPasses + 2; k += blockDim.x) {
        ctl->nface[k] = 0;
        ctl->ncell[k] = 0;
        ctl->ntroub[k] = 0;
    }
    if (threadIdx.x == 0) ctl->stamp0 = stamp0;
}

template <typename real>
__global__ __launch_bounds__(256) void k3_dt(const real *U, size_t n, double gamma, double dx, double dy, double dz,
                                             unsigned long long *lam_bits)
{
    __shared__ double red[256];
    double lam = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double r = U[t], mx = U[n + t], my = U[2 * n + t], mz = U[3 * n + t], E = U[4 * n + t];
        const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my + mz * mz) / r);
        if (!(r > 0.0 && p > 0.0 && __builtin_isfinite(r) && __builtin_isfinite(p))) continue;
        const double cs = sqrt(gamma * p / r);
        const double lx = (fabs(mx / r) + cs) / dx, ly = (fabs(my / r) + cs) / dy, lz = (fabs(mz / r) + cs) / dz;
        double l = lx > ly ? lx : ly;
        l = lz > l ? lz : l;
        lam = l > lam ? l : lam;
    }
    red[threadIdx.x] = lam;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] > 0.0) {
        // as in 2D: no atomic from a block whose value cannot raise the maximum
        const unsigned long long b = (unsigned long long)__double_as_longlong(red[0]);
        if (b > __hip_atomic_load(lam_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(lam_bits, b);
    }
}

__global__ void k3_dt_begin(Ctl *ctl) { ctl->lam_bits = 0ull; }
__global__ void k3_dt_end(Ctl *ctl, double cfl) { ctl->dt = cfl / __longlong_as_double((long long)ctl->lam_bits); }

__global__ __launch_bounds__(256) void k3_hist(const uint8_t *order, size_t n, int l0, int l1, int l2,
                                               unsigned long long *cnt)
{
    __shared__ unsigned long long c[3];
    if (threadIdx.x < 3) c[threadIdx.x] = 0ull;
    __syncthreads();
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const int o = order[t];
        const int l = o == 2 ? l2 : (o == 1 ? l1 : l0);
        atomicAdd(&c[l], 1ull);
    }
    __syncthreads();
    if (threadIdx.x < 3 && c[threadIdx.x]) atomicAdd(&cnt[threadIdx.x], c[threadIdx.x]);
}

// Compensated (double-double) totals, block partials then a fixed-order sum.
template <typename real>
__global__ __launch_bounds__(256) void k3_tot_partial(const real *U, size_t n, double *partial)
{
    __shared__ double sh[256], sl[256];
    const int v = blockIdx.y;
    double hi = 0.0, lo = 0.0;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (size_t)gridDim.x * blockDim.x) {
        const double x = (double)U[v * n + t];
        const double s = hi + x, bb = s - hi, e = (hi - (s - bb)) + (x - bb);
        lo += e;
        hi = s;
    }
    sh[threadIdx.x] = hi;
    sl[threadIdx.x] = lo;
    __syncthreads();
    if (threadIdx.x == 0) {
        double H = 0.0, L = 0.0;
        for (int k = 0; k < 256; ++k) {
            const double s = H + sh[k], bb = s - H, e = (H - (s - bb)) + (sh[k] - bb);
            L += e + sl[k];
            H = s;
        }
        partial[(size_t)v * gridDim.x * 2 + 2 * blockIdx.x] = H;
        partial[(size_t)v * gridDim.x * 2 + 2 * blockIdx.x + 1] = L;
    }
}

__global__ void k3_tot_final(const double *partial, int nblk, double vol, double *tot)
{
    const int v = threadIdx.x;
    if (v >= 5) return;
    double H = 0.0, L = 0.0;
    for (int b = 0; b < nblk; ++b) {
        const double x = partial[(size_t)v * nblk * 2 + 2 * b];
        const double s = H + x, bb = s - H, e = (H - (s - bb)) + (x - bb);
        L += e + partial[(size_t)v * nblk * 2 + 2 * b + 1];
        H = s;
    }
    tot[v] = (H + L) * vol;
}

}  // namespace gpm

using namespace gpm;

// ------------------------------------------------------------------- host side
namespace {

constexpr size_t kAl = 256;
size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }
constexpr int kTot3Blocks = 1024;

}  // namespace

struct gpm3_ctx {
    gpm_grid grid;
    int prec;
    hipStream_t stream;
    int n[3];
    size_t ncell, nface[3], nfaces;
    double d[3];
    bool have_scheme = false;
    gpm_scheme scheme;
    int top = 0, next[4] = {0, 0, 0, 0}, levidx[3] = {0, 0, 0};
    std::vector<double> z64, qw64, pz64;
    std::vector<float> z32, qw32, pz32;
    double curv64[3][4];
    float curv32[3][4];
    char *state = nullptr, *work = nullptr;
    int cur = 0;
    uint8_t *order = nullptr;
    unsigned *cstamp = nullptr, *fstamp = nullptr;
    int *flist[2] = {nullptr, nullptr}, *clist[2] = {nullptr, nullptr};
    void *F[3] = {nullptr, nullptr, nullptr};
    uint8_t *Ff[3] = {nullptr, nullptr, nullptr};
    Ctl *ctl = nullptr;
    double *partial = nullptr;
    void *wtab = nullptr;  // z then qw, context precision
    unsigned pass = 0;
    int last_npass = 0;
    bool fresh = true;
    int *pinned = nullptr;
    std::string err;
};

static gpm_status f3(gpm3_ctx *c, gpm_status st, const std::string &m)
{
    if (c) c->err = m;
    return st;
}

#define H3(c, expr)                                                                        \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess) return f3((c), GPM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

static size_t esz3(const gpm3_ctx *c) { return c->prec == GPM_F64 ? 8 : 4; }
static size_t slot3(const gpm3_ctx *c) { return al(5 * c->ncell * esz3(c)); }

enum { X_ORDER, X_CST, X_FST, X_FL0, X_FL1, X_CL0, X_CL1, X_F0, X_F1, X_F2, X_FF0, X_FF1, X_FF2, X_CTL, X_PART, X_W, X_N };

static size_t layout3(const gpm3_ctx *c, size_t off[X_N])
{
    const size_t e = esz3(c);
    const size_t sz[X_N] = {c->ncell, 4 * c->ncell, 4 * c->nfaces, 4 * c->nfaces, 4 * c->nfaces, 4 * c->ncell,
                            4 * c->ncell, 5 * e * c->nface[0], 5 * e * c->nface[1], 5 * e * c->nface[2],
                            c->nface[0], c->nface[1], c->nface[2], sizeof(Ctl),
                            ((size_t)kTot3Blocks * 5 * 2 + 8) * sizeof(double), (size_t)(2 * kZ3 + 2 * 9 + kPZ3) * e};
    size_t o = 0;
    for (int k = 0; k < X_N; ++k) {
        off[k] = o;
        o = al(o + sz[k]);
    }
    return o;
}

static void *slotp(gpm3_ctx *c, int s) { return c->state + (size_t)s * slot3(c); }

template <typename real>
static Stage3<real> args3(gpm3_ctx *c, int s, const void *Un, const void *Us, void *Uout)
{
    Stage3<real> S;
    S.Un = (const real *)Un;
    S.Us = (const real *)Us;
    S.Uout = (real *)Uout;
    S.dt = &c->ctl->dt;
    S.order = c->order;
    for (int a = 0; a < 3; ++a) {
        S.F[a] = (real *)c->F[a];
        S.Ff[a] = c->Ff[a];
        S.n[a] = c->n[a];
        S.bc[a] = c->grid.bc[a];
        S.d[a] = (real)c->d[a];
    }
    S.fofs[0] = 0;
    S.fofs[1] = (int)c->nface[0];
    S.fofs[2] = (int)(c->nface[0] + c->nface[1]);
    S.fofs[3] = (int)c->nfaces;
    S.cstamp = c->cstamp;
    S.fstamp = c->fstamp;
    S.s = s;
    S.top = c->top;
    S.flags = c->scheme.flags;
    for (int r = 0; r < 4; ++r) S.next[r] = c->next[r];
    S.gamma = (real)c->grid.gamma;
    S.sigma_v = (real)c->scheme.sigma_v;
    S.sigma_p = (real)c->scheme.sigma_p;
    double d3 = 1e300, dm = 1e300;
    for (int a = 0; a < 3; ++a) {
        d3 = c->d[a] * c->d[a] * c->d[a] < d3 ? c->d[a] * c->d[a] * c->d[a] : d3;
        dm = c->d[a] < dm ? c->d[a] : dm;
    }
    S.plat_thr = (real)d3;
    S.delta = (real)dm;
    S.z = (const real *)c->wtab;
    S.qw = (const real *)c->wtab + 2 * kZ3;
    S.pz = (const real *)c->wtab + 2 * kZ3 + 18;
    for (int d = 0; d < 3; ++d)
        for (int k = 0; k < 4; ++k) S.curv[d][k] = sizeof(real) == 8 ? (real)c->curv64[d][k] : (real)c->curv32[d][k];
    S.stamp0 = &c->ctl->stamp0;
    return S;
}

template <typename real>
static gpm_status stage3(gpm3_ctx *c, int s, const void *Un, const void *Us, void *Uout)
{
    Stage3<real> S = args3<real>(c, s, Un, Us, Uout);
    if (c->pass >= 0xffffffffu - (unsigned)(2 * kMaxPasses + 8)) {
        H3(c, hipMemsetAsync(c->cstamp, 0, 4 * c->ncell, c->stream));
        H3(c, hipMemsetAsync(c->fstamp, 0, 4 * c->nfaces, c->stream));
        c->pass = 0;
    }
    const unsigned stamp0 = c->pass + 1;
    c->pass += (unsigned)kMaxPasses + 2;
    const int nzero = c->fresh ? kMaxPasses + 2 : (c->last_npass + 3 < kMaxPasses + 2 ? c->last_npass + 3 : kMaxPasses + 2);
    c->fresh = false;
    hipLaunchKernelGGL(k3_reset, dim3(1), dim3(256), 0, c->stream, c->ctl, nzero, stamp0);
    hipLaunchKernelGGL(k3_fill_order, dim3(1024), dim3(256), 0, c->stream, c->order, c->ncell, c->top);
    // first evaluation: every face at the top radius, then every cell
    int nbf = (int)((c->nfaces + 127) / 128);
    if (nbf > 65536) nbf = 65536;
    int nbc = (int)((c->ncell + 127) / 128);
    if (nbc > 65536) nbc = 65536;
    if (c->top == 2) launch_faces_top<real, 2>(S, c->stream);
    else if (c->top == 1) launch_faces_top<real, 1>(S, c->stream);
    else hipLaunchKernelGGL(k3_faces<real>, dim3(nbf), dim3(128), 0, c->stream, S, (const int *)nullptr, (const int *)nullptr, 1);
    PassOut3 P;
    P.flist = c->flist[1];
    P.clist = c->clist[1];
    P.fcount = &c->ctl->nface[1];
    P.ccount = &c->ctl->ncell[1];
    P.tcount = &c->ctl->ntroub[0];
    P.stamp = 0;
    hipLaunchKernelGGL(k3_cells<real>, dim3(nbc), dim3(128), 0, c->stream, S, (const int *)nullptr, (const int *)nullptr, 1, P);
    H3(c, hipGetLastError());
    // cascade passes in batches, with a host check of the counts per batch
    int nb = (int)((c->ncell + 127) / 128);
    if (nb > 2048) nb = 2048;
    int k = 1, batch = 4;
    for (;;) {
        H3(c, hipMemcpyAsync(c->pinned, &c->ctl->ntroub[k - 1], sizeof(int), hipMemcpyDeviceToHost, c->stream));
        H3(c, hipStreamSynchronize(c->stream));
        if (*c->pinned == 0) break;
        if (k + batch > kMaxPasses) {
            c->last_npass = k - 1;
            return f3(c, GPM_ENOTCONV, "MOOD loop exceeded the pass limit");
        }
        for (int b = 0; b < batch; ++b, ++k) {
            hipLaunchKernelGGL(k3_faces<real>, dim3(nb), dim3(128), 0, c->stream, S, c->flist[k & 1], &c->ctl->nface[k], 0);
            PassOut3 Q;
            Q.flist = c->flist[(k + 1) & 1];
            Q.clist = c->clist[(k + 1) & 1];
            Q.fcount = &c->ctl->nface[k + 1];
            Q.ccount = &c->ctl->ncell[k + 1];
            Q.tcount = &c->ctl->ntroub[k];
            Q.stamp = (unsigned)k;
            hipLaunchKernelGGL(k3_cells<real>, dim3(nb), dim3(128), 0, c->stream, S, c->clist[k & 1], &c->ctl->ncell[k], 0, Q);
        }
        H3(c, hipGetLastError());
        if (batch < 32) batch *= 2;
    }
    c->last_npass = k - 1;
    return GPM_OK;
}

template <typename real>
static gpm_status dt3(gpm3_ctx *c, const void *U, double cfl)
{
    hipLaunchKernelGGL(k3_dt_begin, dim3(1), dim3(1), 0, c->stream, c->ctl);
    size_t nblk = (c->ncell + 255) / 256;
    if (nblk > 8192) nblk = 8192;
    hipLaunchKernelGGL(k3_dt<real>, dim3((unsigned)nblk), dim3(256), 0, c->stream, (const real *)U, c->ncell,
                       c->grid.gamma, c->d[0], c->d[1], c->d[2], &c->ctl->lam_bits);
    hipLaunchKernelGGL(k3_dt_end, dim3(1), dim3(1), 0, c->stream, c->ctl, cfl);
    H3(c, hipGetLastError());
    return GPM_OK;
}

extern "C" {

gpm_status gpm3_create(const gpm_grid *grid, int prec, void *hip_stream, gpm3_ctx **out)
{
    if (!grid || !out) return GPM_EINVAL;
    *out = nullptr;
    if (grid->dim != 3) return GPM_EUNSUPPORTED;
    if (prec != GPM_F32 && prec != GPM_F64) return GPM_EINVAL;
    size_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        if (grid->n[a] < 1 || grid->n[a] > 4096) return GPM_EINVAL;
        if (!(grid->hi[a] > grid->lo[a])) return GPM_EINVAL;
        if (grid->bc[a] == GPM_BC_REFLECT || grid->slit != 0) return GPM_EUNSUPPORTED;  // 2D only
        if (grid->bc[a] != GPM_BC_PERIODIC && grid->bc[a] != GPM_BC_OUTFLOW) return GPM_EINVAL;
        if (grid->bc[a] == GPM_BC_PERIODIC && grid->n[a] < 3) return GPM_EUNSUPPORTED;
        ncell *= (size_t)grid->n[a];
    }
    if (!(grid->gamma > 1.0)) return GPM_EINVAL;
    if (3 * ncell + 3 * 4096 * 4096 > 0x7fffffffull) return GPM_EUNSUPPORTED;  // 32-bit face ids
    gpm3_ctx *c = new (std::nothrow) gpm3_ctx;
    if (!c) return GPM_ENOMEM;
    c->grid = *grid;
    c->prec = prec;
    c->stream = (hipStream_t)hip_stream;
    for (int a = 0; a < 3; ++a) {
        c->n[a] = grid->n[a];
        c->d[a] = (grid->hi[a] - grid->lo[a]) / grid->n[a];
    }
    c->ncell = ncell;
    c->nfaces = 0;
    for (int a = 0; a < 3; ++a) {
        c->nface[a] = (size_t)(c->n[0] + (a == 0)) * (c->n[1] + (a == 1)) * (c->n[2] + (a == 2));
        c->nfaces += c->nface[a];
    }
    if (hipHostMalloc((void **)&c->pinned, 64, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return GPM_EHIP;
    }
    *out = c;
    return GPM_OK;
}

void gpm3_destroy(gpm3_ctx *c)
{
    if (!c) return;
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
}

const char *gpm3_last_error(const gpm3_ctx *c) { return c ? c->err.c_str() : ""; }

static gpm_status upload3(gpm3_ctx *c)
{
    if (!c->wtab || !c->have_scheme) return GPM_OK;
    const size_t e = esz3(c);
    std::vector<char> buf((2 * kZ3 + 18 + kPZ3) * e);
    if (e == 8) {
        std::memcpy(buf.data(), c->z64.data(), 2 * kZ3 * 8);
        std::memcpy(buf.data() + 2 * kZ3 * 8, c->qw64.data(), 18 * 8);
        std::memcpy(buf.data() + (2 * kZ3 + 18) * 8, c->pz64.data(), kPZ3 * 8);
    } else {
        std::memcpy(buf.data(), c->z32.data(), 2 * kZ3 * 4);
        std::memcpy(buf.data() + 2 * kZ3 * 4, c->qw32.data(), 18 * 4);
        std::memcpy(buf.data() + (2 * kZ3 + 18) * 4, c->pz32.data(), kPZ3 * 4);
    }
    H3(c, hipMemcpyAsync(c->wtab, buf.data(), buf.size(), hipMemcpyHostToDevice, c->stream));
    H3(c, hipStreamSynchronize(c->stream));
    return GPM_OK;
}

gpm_status gpm3_set_scheme(gpm3_ctx *c, const gpm_scheme *s)
{
    if (!c || !s) return GPM_EINVAL;
    if (s->nlev < 1 || s->nlev > 3) return f3(c, GPM_EINVAL, "nlev must be 1..3");
    if (s->stencil != GPM_STENCIL_DIAMOND) return f3(c, GPM_EUNSUPPORTED, "the 3D engine uses the L1-ball stencil");
    if (s->solver != GPM_SOLVER_HLLC) return f3(c, GPM_EUNSUPPORTED, "the 3D engine uses HLLC");
    for (int l = 0; l < s->nlev; ++l) {
        if (s->radius[l] < 0 || s->radius[l] > 2) return f3(c, GPM_EINVAL, "3D radius must be 0..2");
        if (l > 0 && !(s->radius[l] < s->radius[l - 1])) return f3(c, GPM_EINVAL, "cascade must strictly decrease");
    }
    if (s->radius[s->nlev - 1] != 0) return f3(c, GPM_EINVAL, "cascade must end at radius 0 (FOG)");
    if (s->radius[0] == 0) return f3(c, GPM_EINVAL, "top scheme must have radius >= 1");
    if (!(s->ell >= 0.0)) return f3(c, GPM_EINVAL, "ell must be >= 0");
    double dmin = c->d[0] < c->d[1] ? c->d[0] : c->d[1];
    dmin = c->d[2] < dmin ? c->d[2] : dmin;
    const double ell = s->ell > 0.0 ? s->ell : 12.0 * dmin;
    c->z64.assign(2 * kZ3, 0.0);
    c->z32.assign(2 * kZ3, 0.0f);
    c->qw64.assign(18, 0.0);
    c->qw32.assign(18, 0.0f);
    c->pz64.assign(kPZ3, 0.0);
    c->pz32.assign(kPZ3, 0.0f);
    for (int R = 1; R <= 2; ++R) {
        bool used = false;
        for (int l = 0; l < s->nlev; ++l) used = used || s->radius[l] == R;
        if (!used) continue;
        Gpw3Level L;
        if (gpw3_level(R, ell / c->d[0], ell / c->d[1], ell / c->d[2], &L) != 0)
            return f3(c, GPM_EINVAL, "GP covariance matrix not positive definite");
        for (int f = 0; f < 6; ++f)
            for (int k = 0; k < L.nq; ++k)
                for (int m = 0; m < kNBall[R]; ++m) {
                    const size_t o = ((size_t)(R - 1) * 6 + f) * 9 * 25 + k * 25 + m;
                    c->z64[o] = L.z64[f][k][m];
                    c->z32[o] = L.z32[f][k][m];
                }
        for (int k = 0; k < L.nq; ++k) {
            c->qw64[(R - 1) * 9 + k] = L.qw64[k];
            c->qw32[(R - 1) * 9 + k] = L.qw32[k];
        }
        if (R == 2)
            for (int f = 0; f < 6; ++f)
                for (int cls = 0; cls < 4; ++cls)
                    for (int e = 0; e < kNPar3; ++e) {
                        c->pz64[((size_t)f * 4 + cls) * kNPar3 + e] = L.pz64[f][cls][e];
                        c->pz32[((size_t)f * 4 + cls) * kNPar3 + e] = L.pz32[f][cls][e];
                    }
    }
    Gpw3Curv K;
    if (gpw3_curvature(ell / c->d[0], ell / c->d[1], ell / c->d[2], ell, &K) != 0)
        return f3(c, GPM_EINVAL, "GP-R1 covariance matrix not positive definite");
    std::memcpy(c->curv64, K.w64, sizeof(c->curv64));
    std::memcpy(c->curv32, K.w32, sizeof(c->curv32));
    c->scheme = *s;
    c->scheme.ell = ell;
    c->top = s->radius[0];
    for (int r = 0; r < 4; ++r) c->next[r] = 0;
    for (int l = 0; l < s->nlev; ++l) {
        c->levidx[s->radius[l]] = l;
        c->next[s->radius[l]] = l + 1 < s->nlev ? s->radius[l + 1] : 0;
    }
    c->have_scheme = true;
    return upload3(c);
}

gpm_status gpm3_workspace_size(const gpm3_ctx *c, size_t *state_bytes, size_t *work_bytes)
{
    if (!c) return GPM_EINVAL;
    size_t off[X_N];
    if (state_bytes) *state_bytes = 3 * slot3(c);
    if (work_bytes) *work_bytes = layout3(c, off);
    return GPM_OK;
}

gpm_status gpm3_bind(gpm3_ctx *c, void *state, void *work)
{
    if (!c || !state || !work) return GPM_EINVAL;
    if (((uintptr_t)state % kAl) || ((uintptr_t)work % kAl)) return f3(c, GPM_EINVAL, "buffers must be 256-byte aligned");
    size_t off[X_N];
    const size_t wb = layout3(c, off);
    c->state = (char *)state;
    c->work = (char *)work;
    c->order = (uint8_t *)(c->work + off[X_ORDER]);
    c->cstamp = (unsigned *)(c->work + off[X_CST]);
    c->fstamp = (unsigned *)(c->work + off[X_FST]);
    c->flist[0] = (int *)(c->work + off[X_FL0]);
    c->flist[1] = (int *)(c->work + off[X_FL1]);
    c->clist[0] = (int *)(c->work + off[X_CL0]);
    c->clist[1] = (int *)(c->work + off[X_CL1]);
    for (int a = 0; a < 3; ++a) {
        c->F[a] = c->work + off[X_F0 + a];
        c->Ff[a] = (uint8_t *)(c->work + off[X_FF0 + a]);
    }
    c->ctl = (Ctl *)(c->work + off[X_CTL]);
    c->partial = (double *)(c->work + off[X_PART]);
    c->wtab = c->work + off[X_W];
    c->cur = 0;
    c->pass = 0;
    c->fresh = true;
    H3(c, hipMemsetAsync(c->work, 0, wb, c->stream));
    H3(c, hipStreamSynchronize(c->stream));
    return upload3(c);
}

gpm_status gpm3_init_state(gpm3_ctx *c, const double *U)
{
    if (!c || !U) return GPM_EINVAL;
    if (!c->state) return f3(c, GPM_ESTATE, "not bound");
    const size_t n = 5 * c->ncell;
    if (c->prec == GPM_F64) {
        H3(c, hipMemcpyAsync(slotp(c, c->cur), U, n * 8, hipMemcpyHostToDevice, c->stream));
        H3(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> t(n);
        for (size_t k = 0; k < n; ++k) t[k] = (float)U[k];
        H3(c, hipMemcpyAsync(slotp(c, c->cur), t.data(), n * 4, hipMemcpyHostToDevice, c->stream));
        H3(c, hipStreamSynchronize(c->stream));
    }
    return GPM_OK;
}

gpm_status gpm3_get_state(gpm3_ctx *c, double *U)
{
    if (!c || !U) return GPM_EINVAL;
    if (!c->state) return f3(c, GPM_ESTATE, "not bound");
    const size_t n = 5 * c->ncell;
    if (c->prec == GPM_F64) {
        H3(c, hipMemcpyAsync(U, slotp(c, c->cur), n * 8, hipMemcpyDeviceToHost, c->stream));
        H3(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> t(n);
        H3(c, hipMemcpyAsync(t.data(), slotp(c, c->cur), n * 4, hipMemcpyDeviceToHost, c->stream));
        H3(c, hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < n; ++k) U[k] = t[k];
    }
    return GPM_OK;
}

gpm_status gpm3_compute_dt(gpm3_ctx *c, double cfl, double *dt_host)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return f3(c, GPM_ESTATE, "not bound");
    if (!(cfl > 0.0)) return f3(c, GPM_EINVAL, "cfl must be > 0");
    gpm_status st = c->prec == GPM_F64 ? dt3<double>(c, slotp(c, c->cur), cfl) : dt3<float>(c, slotp(c, c->cur), cfl);
    if (st != GPM_OK) return st;
    if (dt_host) {
        H3(c, hipMemcpyAsync(dt_host, &c->ctl->dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        H3(c, hipStreamSynchronize(c->stream));
    }
    return GPM_OK;
}

gpm_status gpm3_step(gpm3_ctx *c, double cfl, int nsteps)
{
    if (!c || nsteps < 0) return GPM_EINVAL;
    if (!c->have_scheme) return f3(c, GPM_ESTATE, "no scheme set");
    if (!c->state) return f3(c, GPM_ESTATE, "not bound");
    if (!(cfl > 0.0)) return f3(c, GPM_EINVAL, "cfl must be > 0");
    for (int n = 0; n < nsteps; ++n) {
        const int u0 = c->cur, a = (c->cur + 1) % 3, b = (c->cur + 2) % 3;
        const bool dbl = c->prec == GPM_F64;
        gpm_status st = dbl ? dt3<double>(c, slotp(c, u0), cfl) : dt3<float>(c, slotp(c, u0), cfl);
        if (st == GPM_OK) st = dbl ? stage3<double>(c, 0, slotp(c, u0), slotp(c, u0), slotp(c, a))
                                   : stage3<float>(c, 0, slotp(c, u0), slotp(c, u0), slotp(c, a));
        if (st == GPM_OK) st = dbl ? stage3<double>(c, 1, slotp(c, u0), slotp(c, a), slotp(c, b))
                                   : stage3<float>(c, 1, slotp(c, u0), slotp(c, a), slotp(c, b));
        if (st == GPM_OK) st = dbl ? stage3<double>(c, 2, slotp(c, u0), slotp(c, b), slotp(c, a))
                                   : stage3<float>(c, 2, slotp(c, u0), slotp(c, b), slotp(c, a));
        if (st != GPM_OK) return st;
        c->cur = a;
    }
    return GPM_OK;
}

gpm_status gpm3_troubled_counts(gpm3_ctx *c, long long counts[3], int *mood_iters)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return f3(c, GPM_ESTATE, "not bound");
    H3(c, hipMemsetAsync(c->ctl->levcnt, 0, sizeof(c->ctl->levcnt), c->stream));
    hipLaunchKernelGGL(k3_hist, dim3(1024), dim3(256), 0, c->stream, c->order, c->ncell, c->levidx[0], c->levidx[1],
                       c->levidx[2], c->ctl->levcnt);
    unsigned long long lc[3];
    H3(c, hipMemcpyAsync(lc, c->ctl->levcnt, sizeof(lc), hipMemcpyDeviceToHost, c->stream));
    // passes are queued in batches: count those that had cells to re-evaluate
    std::vector<int> nc(c->last_npass + 2);
    H3(c, hipMemcpyAsync(nc.data(), c->ctl->ncell, sizeof(int) * nc.size(), hipMemcpyDeviceToHost, c->stream));
    H3(c, hipStreamSynchronize(c->stream));
    if (counts)
        for (int l = 0; l < 3; ++l) counts[l] = (long long)lc[l];
    if (mood_iters) {
        int it = 1;
        for (size_t k = 1; k < nc.size(); ++k)
            if (nc[k] > 0) ++it;
        *mood_iters = it;
    }
    return GPM_OK;
}

gpm_status gpm3_get_order_mask(gpm3_ctx *c, unsigned char *out)
{
    if (!c || !out) return GPM_EINVAL;
    if (!c->state) return f3(c, GPM_ESTATE, "not bound");
    H3(c, hipMemcpyAsync(out, c->order, c->ncell, hipMemcpyDeviceToHost, c->stream));
    H3(c, hipStreamSynchronize(c->stream));
    return GPM_OK;
}

gpm_status gpm3_totals(gpm3_ctx *c, double totals[5])
{
    if (!c || !totals) return GPM_EINVAL;
    if (!c->state) return f3(c, GPM_ESTATE, "not bound");
    const int nblk = kTot3Blocks;
    if (c->prec == GPM_F64)
        hipLaunchKernelGGL(k3_tot_partial<double>, dim3(nblk, 5), dim3(256), 0, c->stream,
                           (const double *)slotp(c, c->cur), c->ncell, c->partial);
    else
        hipLaunchKernelGGL(k3_tot_partial<float>, dim3(nblk, 5), dim3(256), 0, c->stream,
                           (const float *)slotp(c, c->cur), c->ncell, c->partial);
    double *tot = c->partial + (size_t)kTot3Blocks * 5 * 2;
    hipLaunchKernelGGL(k3_tot_final, dim3(1), dim3(64), 0, c->stream, c->partial, nblk, c->d[0] * c->d[1] * c->d[2],
                       tot);
    double t[5];
    H3(c, hipMemcpyAsync(t, tot, sizeof(t), hipMemcpyDeviceToHost, c->stream));
    H3(c, hipStreamSynchronize(c->stream));
    for (int v = 0; v < 5; ++v) totals[v] = t[v];
    return GPM_OK;
}

}  // extern "C"
