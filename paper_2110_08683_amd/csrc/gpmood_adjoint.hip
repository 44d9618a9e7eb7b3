// Adjoint (vector-Jacobian product) of one SSP-RK3 stage with the cell orders of
// the forward stage and its dt held fixed.
//
// With the orders frozen the stage is U_out = combine(s, U^n, U*), U* = U_s - dt
// (F_{i+1/2} - F_{i-1/2}) / dx - dt (G_{j+1/2} - G_{j-1/2}) / dy (eq. (fvm_discrete)),
// every face flux a Gauss sum of HLLC fluxes of GP-reconstructed states at the
// face's EDP_1 radius (eq. (fvm_F), eq. (gp_reconstructor)).  Given lambda_out =
// dL/dU_out this returns dL/dU_s, adds dL/dU^n, and sums dL/d(ell) through the
// ell-dependence of the GP weights.  Per face (k_adj_faces):
//   1. lambda_F = (alpha lambda_out(R) - alpha lambda_out(L)) dt / Delta, from the
//      cells whose update uses this copy of the face (alpha = 1, 1/4, 2/3);
//   2. the node states are rebuilt in the quarter basis (as in the cascade);
//   3. per Gauss node, J^T (w_g lambda_F) for both states, by reverse mode
//      through the HLLC flux with the forward's branches;
//   4. node adjoints -> the adjoints of both sides' quarter accumulators, stored
//      as the face's record (no atomics).
// Per cell (k_adj_cells): the transposed reconstruction, gathered in a fixed
// order from the records of the faces whose stencils hold the cell (stencil cells
// remapped exactly as the forward gathers them), gives dL/dU_s = alpha lambda_out
// + that sum, and beta lambda_out is added to dL/dU^n (beta = 3/4, 1/3); in stage
// 0, where U^n is also U_s, a given dL/dU^n from the later stages is added to
// dL/dU_s instead.  Per cell again (k_adj_dl): dL/d(ell), the records times the
// ell-derivatives of the weights times the parity sums of the state, for the face
// sides centred on the cell, summed per block and then in a fixed order.
#include "gpmood_device.h"
#include "gpmood_launch.h"

namespace gpm {

// ------------------------------------------------- reverse-mode HLLC
// Reverse mode through the x-face HLLC flux: given weights w (the adjoint of the
// flux), gl = w^T dF/dUL and gr = w^T dF/dUR, with every branch (the wave-speed
// minimum and maximum, the sign of S*, the side of the fan) taken as the flux
// takes it.  One pass recomputes the flux's intermediates, a second runs the
// chain rule backwards through them: about three times the cost of the flux
// itself, where eight forward-mode (dual-number) passes cost about twenty.
// Adjoints of the primitive values (density r, normal and tangential velocity
// u, v, energy E, pressure p, inverse density ir) are held per side (0 = left,
// 1 = right) and mapped to the conserved variables at the end.
template <typename real>
struct SideAdj {
    real r, u, v, E, p, ir;
    __device__ void zero() { r = u = v = E = p = ir = real(0); }
};

// w . (physical flux of (r, u, v, E, p)), back to the primitives.
template <typename real>
__device__ __forceinline__ void flux_adj(const real (&w)[4], real r, real u, real v, real E, real p, SideAdj<real> &a)
{
    a.r += w[0] * u + w[1] * u * u + w[2] * u * v;
    a.u += w[0] * r + real(2) * w[1] * r * u + w[2] * r * v + w[3] * (E + p);
    a.v += w[2] * r * u;
    a.E += w[3] * u;
    a.p += w[1] + w[3] * u;
}

template <typename real>
__device__ __forceinline__ void hllc_vjp(real g, const real (&UL)[4], const real (&UR)[4], const real (&w)[4],
                                         real (&gl)[4], real (&gr)[4])
{
    // forward: the intermediates of hllc<0>
    const real rl = UL[0], irl = dv(real(1), rl), ul = UL[1] * irl, vl = UL[2] * irl, El = UL[3];
    const real rr = UR[0], irr = dv(real(1), rr), ur = UR[1] * irr, vr = UR[2] * irr, Er = UR[3];
    const real pl = (g - real(1)) * (El - real(0.5) * rl * (ul * ul + vl * vl));
    const real pr = (g - real(1)) * (Er - real(0.5) * rr * (ur * ur + vr * vr));
    const real cl = sq(g * pl * irl), cr = sq(g * pr * irr);
    const bool minL = (ul - cl) < (ur - cr), maxL = (ul + cl) > (ur + cr);
    const real SL = minL ? ul - cl : ur - cr;
    const real SR = maxL ? ul + cl : ur + cr;
    const real dL = SL - ul, dR = SR - ur;
    const real den = rl * dL - rr * dR;
    const real Ss = dv(pr - pl + rl * ul * dL - rr * ur * dR, den);
    const bool useL = Ss >= real(0);
    const bool takeL = SL >= real(0);
    const bool takeStar = !takeL && (useL || SR > real(0));
    // backward
    SideAdj<real> a[2];
    a[0].zero();
    a[1].zero();
    real aSL = real(0), aSR = real(0);
    if (takeL) {
        flux_adj(w, rl, ul, vl, El, pl, a[0]);
    } else if (!takeStar) {
        flux_adj(w, rr, ur, vr, Er, pr, a[1]);
    } else {
        SideAdj<real> &k = useL ? a[0] : a[1];
        const real r = useL ? rl : rr, u = useL ? ul : ur, v = useL ? vl : vr, E = useL ? El : Er;
        const real p = useL ? pl : pr, ir = useL ? irl : irr, S = useL ? SL : SR;
        const real sku = S - u, den2 = S - Ss, rs = r * sku;
        const real fac = dv(rs, den2), q = dv(p, rs);
        const real Y = Ss + q, Z = Ss - u, X = E * ir + Z * Y;
        // F* = F_k + S (U* - U_k), U* = fac (1, Ss, v, X)
        flux_adj(w, r, u, v, E, p, k);
        const real us[4] = {fac, fac * Ss, fac * v, fac * X};
        const real uc[4] = {r, r * u, r * v, E};
        real aS = real(0);
#pragma unroll
        for (int i = 0; i < 4; ++i) aS += w[i] * (us[i] - uc[i]);
        // U_k = (r, r u, r v, E)
        k.r -= S * (w[0] + w[1] * u + w[2] * v);
        k.u -= S * w[1] * r;
        k.v -= S * w[2] * r;
        k.E -= S * w[3];
        const real afac = S * (w[0] + w[1] * Ss + w[2] * v + w[3] * X);
        real aSs = S * w[1] * fac;
        k.v += S * w[2] * fac;
        const real aX = S * w[3] * fac;
        k.E += aX * ir;
        k.ir += aX * E;
        const real aZ = aX * Y, aY = aX * Z;
        aSs += aZ + aY;
        k.u -= aZ;
        k.p += dv(aY, rs);
        const real ars = dv(afac, den2) - dv(aY * q, rs);  // rs enters fac and q
        const real aden2 = -dv(afac * fac, den2);
        k.r += ars * sku;
        const real asku = ars * r;
        aS += aden2 + asku;
        aSs -= aden2;
        k.u -= asku;
        if (useL) aSL += aS;
        else aSR += aS;
        // S* = num / den
        const real anum = dv(aSs, den), aden = -dv(aSs * Ss, den);
        a[1].p += anum;
        a[0].p -= anum;
        a[0].r += anum * ul * dL + aden * dL;
        a[0].u += anum * rl * (dL - ul) - aden * rl;
        aSL += anum * rl * ul + aden * rl;
        a[1].r -= anum * ur * dR + aden * dR;
        a[1].u -= anum * rr * (dR - ur) - aden * rr;
        aSR -= anum * rr * ur + aden * rr;
    }
    // wave-speed bounds: S_L = u - c and S_R = u + c of the side each takes
    real acl = real(0), acr = real(0);
    if (minL) { a[0].u += aSL; acl -= aSL; }
    else { a[1].u += aSL; acr -= aSL; }
    if (maxL) { a[0].u += aSR; acl += aSR; }
    else { a[1].u += aSR; acr += aSR; }
    // c = sqrt(g p ir), then p = (g - 1) (E - r (u^2 + v^2) / 2), u = m ir, v = n ir, ir = 1 / r
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        SideAdj<real> &b = a[sd];
        const real c = sd ? cr : cl, p = sd ? pr : pl, ir = sd ? irr : irl, r = sd ? rr : rl;
        const real u = sd ? ur : ul, v = sd ? vr : vl;
        const real ax = dv(sd ? acr : acl, real(2) * c);
        b.p += ax * g * ir;
        b.ir += ax * g * p;
        const real gp = (g - real(1)) * b.p;
        b.E += gp;
        b.r -= gp * real(0.5) * (u * u + v * v);
        b.u -= gp * r * u;
        b.v -= gp * r * v;
        const real *U = sd ? UR : UL;
        b.ir += b.u * U[1] + b.v * U[2];
        real *out = sd ? gr : gl;
        out[0] = b.r - b.ir * ir * ir;
        out[1] = b.u * ir;
        out[2] = b.v * ir;
        out[3] = b.E;
    }
}

// ------------------------------------------------ per-face adjoint layout
// Offsets (da, db) of a stencil cell from its face side's centre, |da| + |db| <= 3,
// in the fixed order of the gather.
constexpr int kAdjDa[kAdjOffsets] = {0, -1, 0, 1, -2, -1, 0, 1, 2, -3, -2, -1, 0, 1, 2, 3, -2, -1, 0, 1, 2, -1, 0, 1, 0};
constexpr int kAdjDb[kAdjOffsets] = {-3, -2, -2, -2, -1, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 2, 2, 2, 3};

__host__ __device__ constexpr int iabs_c(int x) { return x < 0 ? -x : x; }
// Index of position (a, b) = (|da|, |db|) in the compact weight table, and the
// smallest face radius whose stencil holds it.
__host__ __device__ constexpr int pos_of(int a, int b)
{
    return a == 0 && b == 0 ? 0 : a == 1 && b == 0 ? 1 : a == 0 && b == 1 ? 2 : a == 2 && b == 0 ? 3
         : a == 0 && b == 2 ? 4 : a == 1 && b == 1 ? 5 : a == 3 && b == 0 ? 6 : a == 0 && b == 3 ? 7
         : a == 2 && b == 1 ? 8 : 9;
}
__host__ __device__ constexpr int min_radius(int e) { return e == 0 ? 0 : (e <= 2 ? 1 : (e <= 5 ? 2 : 3)); }

// The per-face record: the adjoints of both sides' quarter accumulators, 64
// values per face in blocks of 16 per (direction, variable): block (dir, v) of
// face (i, j) holds side * 8 + p * 4 + c contiguously, at [dir][v][ny+1][nx+1][16],
// so that a face writes, and a gather reads, whole 16-byte quads.
template <typename real>
__device__ __forceinline__ real *record_block(const AdjArgs<real> &J, int dir, int v, int i, int j)
{
    const size_t FX = (size_t)J.A.nx + 1, FY = (size_t)J.A.ny + 1;
    return J.gface + ((((size_t)dir * 4 + v) * FY + (size_t)j) * FX + (size_t)i) * 16;
}

// Four values moved together (one 16-byte access per four floats).
template <typename real>
struct alignas(16) Quad {
    real x[4];
};

// ------------------------------------------------------------ per-face adjoint
template <typename real>
__global__ __launch_bounds__(128) void k_adj_faces(const AdjArgs<real> J)
{
    const StageArgs<real> &A = J.A;
    const int nx = A.nx, ny = A.ny;
    const size_t plane = (size_t)nx * ny;
    // a periodic axis has one face per cell along it (the face at the wrap joins
    // cells n-1 and 0), an outflow axis n + 1
    const int fxn = A.bcx == 0 ? nx : nx + 1, fyn = A.bcy == 0 ? ny : ny + 1;
    const int nfx = fxn * ny, nft = nfx + nx * fyn;
    const real alpha = A.s == 0 ? real(1) : (A.s == 1 ? real(0.25) : real(2) / real(3));
    const real dt = (real)(*A.dt);
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nft; f += gridDim.x * blockDim.x) {
        int dir, iL, jL, i, j;
        bool hasL, hasR;
        if (f < nfx) {
            dir = 0;
            j = f / fxn;
            i = f - j * fxn;  // between cells i-1 and i
            iL = i - 1;
            jL = j;
            hasL = A.bcx == 0 || i >= 1;
            hasR = A.bcx == 0 || i < nx;
        } else {
            dir = 1;
            const int g = f - nfx;
            j = g / nx;
            i = g - j * nx;  // between cells (i, j-1) and (i, j)
            iL = i;
            jL = j - 1;
            hasL = A.bcy == 0 || j >= 1;
            hasR = A.bcy == 0 || j < ny;
        }
        const int iR = iL + (dir == 0), jR = jL + (dir == 1);
        const int cL = wrap(jL, ny, A.bcy) * nx + wrap(iL, nx, A.bcx);
        const int cR = wrap(jR, ny, A.bcy) * nx + wrap(iR, nx, A.bcx);
        const real inv = dt / (dir == 0 ? A.dx : A.dy);
        real lF[4];
        bool any = false;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const real lr = hasR ? J.lam_out[v * plane + cR] : real(0);
            const real ll = hasL ? J.lam_out[v * plane + cL] : real(0);
            lF[v] = (alpha * lr - alpha * ll) * inv;
            any = any || lF[v] != real(0);
        }
        if (!any) {
            // nothing flows through this face: its record holds zeros
            const Quad<real> z = {{real(0), real(0), real(0), real(0)}};
            for (int v = 0; v < 4; ++v) {
                Quad<real> *blk = reinterpret_cast<Quad<real> *>(record_block(J, dir, v, i, j));
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) blk[k4] = z;
            }
            continue;
        }
        const int R = min((int)A.order[cL], (int)A.order[cR]);
        const int np = R <= 0 ? 1 : (R == 1 ? 3 : (R == 2 ? 6 : 10));
        const int q = R <= 0 ? 1 : R + 1;
        const real *wt = A.gtab + (R * 2 + dir) * kGtabPerDir;
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
            // the position's 32 values and 8 weights, all loads issued before the
            // arithmetic that waits for them
            real u[4][8], wq[2][4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const real *U = A.Us + v * plane;
                u[v][0] = U[yLp + xLp];
                u[v][1] = U[yLp + xLm];
                u[v][2] = U[yLm + xLp];
                u[v][3] = U[yLm + xLm];
                u[v][4] = U[yRp + xRp];
                u[v][5] = U[yRp + xRm];
                u[v][6] = U[yRm + xRp];
                u[v][7] = U[yRm + xRm];
            }
#pragma unroll
            for (int p = 0; p < 2; ++p)
#pragma unroll
                for (int c = 0; c < 4; ++c) wq[p][c] = wt[p * (kNPos * 4) + e * 4 + c];
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                real ql[4], qr[4];
                parity4(u[v][0], u[v][1], u[v][2], u[v][3], ql);
                parity4(u[v][4], u[v][5], u[v][6], u[v][7], qr);
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        PL[v][p][c] = fma(wq[p][c], ql[c], PL[v][p][c]);
                        PR[v][p][c] = fma(wq[p][c], qr[c], PR[v][p][c]);
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
            // d(w_g lambda_F . F) / d(UL, UR), momenta rotated into the x-face form
            const real wx[4] = {wq_ * lF[0], wq_ * (dir ? lF[2] : lF[1]), wq_ * (dir ? lF[1] : lF[2]), wq_ * lF[3]};
            const real L4[4] = {UL[0], dir ? UL[2] : UL[1], dir ? UL[1] : UL[2], UL[3]};
            const real R4[4] = {UR[0], dir ? UR[2] : UR[1], dir ? UR[1] : UR[2], UR[3]};
            real gxl[4], gxr[4];
            hllc_vjp(A.gamma, L4, R4, wx, gxl, gxr);
            const real gs[8] = {gxl[0], dir ? gxl[2] : gxl[1], dir ? gxl[1] : gxl[2], gxl[3],
                                gxr[0], dir ? gxr[2] : gxr[1], dir ? gxr[1] : gxr[2], gxr[3]};
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
        // 4. the face's record (the transposed reconstruction, and the ell terms,
        // are applied by the cells that gather it)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Quad<real> *blk = reinterpret_cast<Quad<real> *>(record_block(J, dir, v, i, j));
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                Quad<real> l, r;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    l.x[c] = gL[v][p][c];
                    r.x[c] = gR[v][p][c];
                }
                blk[p] = l;
                blk[2 + p] = r;
            }
        }
    }
}

// ------------------------------------------------------------ per-cell gather
// A 16 x 16 tile of cells gathers from the faces whose stencils reach it: face
// indices [t0 - 3, t0 + 19] on both axes (a 23 x 23 window), staged in LDS one
// (direction, variable) at a time with the faces' radii and the direction's
// compact weights.  Each cell sums, in a fixed order, over its unwrapped images
// (its own index, and on an outflow axis the ghost indices that copy an edge cell)
// and over the 2 sides x 25 offsets of each direction, the contribution of the
// face side centred at image - offset: the weighted accumulator adjoints
// (h_c = sum_p w[p][e][c] g[p][c] at position e = (|da|, |db|)), combined with
// the signs of the mirror image (+-a, +-b) that reads this cell, both mirrors
// when a or b is 0.
constexpr int kTile = kAdjTile;
constexpr int kWin = kTile + 7;
template <typename real>
struct GatherLds {
    static constexpr int kStride = sizeof(real) == 4 ? 20 : 18;  // 16 values, padded against bank conflicts
    alignas(16) real g[kWin * kWin * kStride];
    alignas(16) real w[4 * kGtabPerDir];
    signed char r[kWin * kWin];
};

// Contribution of the face side whose LDS record is g (8 values: p, c) to the
// stencil cell at offset (DA, DB) from the side's centre, with the compact
// weights w0 = w[0][e][.], w1 = w[1][e][.] of its position e:
// h_c = w0_c g0_c + w1_c g1_c, combined with the signs of the mirror image
// (+-a, +-b) that reads the cell: x-odd parts carry sign(DA), y-odd parts
// sign(DB), and a zero offset takes both mirrors, doubling the even part and
// cancelling the odd one.
template <typename real, int DA, int DB>
__device__ __forceinline__ real side_term(const Quad<real> &w0, const Quad<real> &w1, const real *g)
{
#pragma clang fp contract(fast)
    const Quad<real> g0 = *reinterpret_cast<const Quad<real> *>(g);
    const Quad<real> g1 = *reinterpret_cast<const Quad<real> *>(g + 4);
    real h[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) h[c] = w0.x[c] * g0.x[c] + w1.x[c] * g1.x[c];
    if constexpr (DA == 0 && DB == 0) {
        return real(4) * h[C_EE];
    } else if constexpr (DA == 0) {
        return real(2) * (DB > 0 ? h[C_EE] + h[C_EO] : h[C_EE] - h[C_EO]);
    } else if constexpr (DB == 0) {
        return real(2) * (DA > 0 ? h[C_EE] + h[C_OE] : h[C_EE] - h[C_OE]);
    } else {
        const real x = DA > 0 ? h[C_EE] + h[C_OE] : h[C_EE] - h[C_OE];
        const real y = DA > 0 ? h[C_EO] + h[C_OO] : h[C_EO] - h[C_OO];
        return DB > 0 ? x + y : x - y;
    }
}

// The 25 offsets in gather order: grouped by stencil position e, so that one
// position's weights serve consecutive terms.
constexpr int kGatherDa[kAdjOffsets] = {0, 1, -1, 0, 0, 2, -2, 0, 0, 1, -1, 1, -1, 3, -3, 0, 0, 2, -2, 2, -2, 1, -1, 1, -1};
constexpr int kGatherDb[kAdjOffsets] = {0, 0, 0, 1, -1, 0, 0, 2, -2, 1, 1, -1, -1, 0, 0, 3, -3, 1, 1, -1, -1, 2, 2, -2, -2};

// The contributions to one cell image at window coordinates (bx, by) from the
// faces of direction DIR, summed over (offset, side) in a fixed order, with the
// weights of each face's radius from the LDS table (all lanes read the same
// entries).  TOP: every face of the window has the top radius 3 or does not exist
// (then its record is zero), so no radius test is needed: the sum has the same
// bits as the general path's.  CHECK: the image may reach outside the window
// (ghost images of edge cells).
template <typename real, int DIR, bool CHECK, bool TOP, int O = 0>
__device__ __forceinline__ void gather_sides(const GatherLds<real> &L, int bx, int by, real &sum)
{
    if constexpr (O < 2 * kAdjOffsets) {
        constexpr int o = O / 2, side = O % 2;
        constexpr int da = kGatherDa[o], db = kGatherDb[o];
        constexpr int e = pos_of(iabs_c(da), iabs_c(db));
        const int wx = bx - da + (DIR == 0 && side == 0 ? 1 : 0);
        const int wy = by - db + (DIR == 1 && side == 0 ? 1 : 0);
        const int f = wy * kWin + wx;
        const real *g = L.g + f * GatherLds<real>::kStride + side * 8;
        if constexpr (TOP) {
            const real *w = L.w + 3 * kGtabPerDir + e * 4;
            sum += side_term<real, da, db>(*reinterpret_cast<const Quad<real> *>(w),
                                           *reinterpret_cast<const Quad<real> *>(w + kNPos * 4), g);
        } else {
            if (!CHECK || (wx >= 0 && wx < kWin && wy >= 0 && wy < kWin)) {
                const int R = L.r[f];
                if (R >= min_radius(e)) {  // not: no face (-1), or beyond its radius
                    const real *w = L.w + R * kGtabPerDir + e * 4;
                    sum += side_term<real, da, db>(*reinterpret_cast<const Quad<real> *>(w),
                                                   *reinterpret_cast<const Quad<real> *>(w + kNPos * 4), g);
                }
            }
        }
        gather_sides<real, DIR, CHECK, TOP, O + 1>(L, bx, by, sum);
    }
}

__device__ __forceinline__ int mod_n(int i, int n)
{
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// Unwrapped images of index m on an axis of n cells: m, and on an outflow axis
// the ghost indices that copy an edge cell (face-side centres run from -1 to n,
// so radius-3 stencils read ghosts -1..-4 and n..n+3).  Count, and image q.
__device__ __forceinline__ int n_images(int m, int n, int bc)
{
    return 1 + (bc != 0 && m == 0 ? 4 : 0) + (bc != 0 && m == n - 1 ? 4 : 0);
}
__device__ __forceinline__ int image(int m, int n, int bc, int q)
{
    if (q == 0) return m;
    if (bc != 0 && m == 0 && q <= 4) return -q;
    return n - 1 + (q - (m == 0 ? 4 : 0));
}

// Window face q of direction dir: its face indices (periodic axes wrapped) and
// whether it exists.
struct WinFace {
    int fi, fj;
    bool ok;
};
__device__ __forceinline__ WinFace win_face(int q, int dir, int i0, int j0, int nx, int ny, int bcx, int bcy)
{
    WinFace w;
    w.fi = i0 - 3 + q % kWin;
    w.fj = j0 - 3 + q / kWin;
    w.ok = true;
    const int fxn = dir == 0 ? (bcx == 0 ? nx : nx + 1) : nx;
    const int fyn = dir == 1 ? (bcy == 0 ? ny : ny + 1) : ny;
    if (bcx == 0) w.fi = mod_n(w.fi, nx);
    else w.ok = w.ok && w.fi >= 0 && w.fi < fxn;
    if (bcy == 0) w.fj = mod_n(w.fj, ny);
    else w.ok = w.ok && w.fj >= 0 && w.fj < fyn;
    return w;
}

constexpr int kWinPerThread = (kWin * kWin + 255) / 256;

// This thread's share of the window records of round r (direction r / 4,
// variable r % 4): 16 values (side, p, c) per face, zero for absent faces.
template <typename real>
__device__ __forceinline__ void fetch_round(const AdjArgs<real> &J, int r, int i0, int j0,
                                            Quad<real> (&pre)[kWinPerThread][4])
{
    const int dir = r >> 2, v = r & 3;
#pragma unroll
    for (int t = 0; t < kWinPerThread; ++t) {
        const int q = threadIdx.x + t * 256;
        const WinFace w = win_face(q, dir, i0, j0, J.A.nx, J.A.ny, J.A.bcx, J.A.bcy);
        const bool ok = q < kWin * kWin && w.ok;
        const Quad<real> *blk = reinterpret_cast<const Quad<real> *>(record_block(J, dir, v, ok ? w.fi : 0, ok ? w.fj : 0));
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4) {  // side * 2 + p; an absent face (block of face 0) reads as zeros
            const Quad<real> r = blk[k4];
#pragma unroll
            for (int c = 0; c < 4; ++c) pre[t][k4].x[c] = ok ? r.x[c] : real(0);
        }
    }
}

template <typename real>
__global__ __launch_bounds__(256, 2) void k_adj_cells(const AdjArgs<real> J)
{
    __shared__ GatherLds<real> L;
    const StageArgs<real> &A = J.A;
    const int nx = A.nx, ny = A.ny;
    const size_t n = (size_t)nx * ny;
    // tiles in row-major order, dealt so that the workgroups of one XCD take a
    // contiguous run of them: neighbouring tiles, whose windows overlap by seven
    // faces on each side, share the records in that XCD's L2
    const int ntx = (nx + kTile - 1) / kTile, t = xcd_tile(blockIdx.x, gridDim.x);
    const int i0 = (t % ntx) * kTile, j0 = (t / ntx) * kTile;
    const int tx = threadIdx.x % kTile, ty = threadIdx.x / kTile;
    const int mi = i0 + tx, mj = j0 + ty;
    const bool own = mi < nx && mj < ny;
    const int nix = own ? n_images(mi, nx, A.bcx) : 0, niy = own ? n_images(mj, ny, A.bcy) : 0;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    constexpr int KS = GatherLds<real>::kStride;
    // eight rounds (direction, variable); the next round's records are fetched
    // into registers while this round's are gathered
    Quad<real> pre[kWinPerThread][4];
    fetch_round(J, 0, i0, j0, pre);
    bool top = false;
    for (int r = 0; r < 8; ++r) {
        const int dir = r >> 2, v = r & 3;
        __syncthreads();  // the previous round's readers are done
#pragma unroll
        for (int t = 0; t < kWinPerThread; ++t) {
            const int q = threadIdx.x + t * 256;
            if (q < kWin * kWin) {
                Quad<real> *dst = reinterpret_cast<Quad<real> *>(L.g + q * KS);
#pragma unroll
                for (int k4 = 0; k4 < 4; ++k4) dst[k4] = pre[t][k4];
            }
        }
        if (v == 0) {
            // this direction's face radii and weights
            bool notop = false;
            for (int q = threadIdx.x; q < kWin * kWin; q += blockDim.x) {
                const WinFace w = win_face(q, dir, i0, j0, nx, ny, A.bcx, A.bcy);
                int R = -1;
                if (w.ok) {
                    const int iL = w.fi - (dir == 0), jL = w.fj - (dir == 1);
                    const int cL = wrap(jL, ny, A.bcy) * nx + wrap(iL, nx, A.bcx);
                    const int cR = wrap(w.fj, ny, A.bcy) * nx + wrap(w.fi, nx, A.bcx);
                    R = min((int)A.order[cL], (int)A.order[cR]);
                }
                L.r[q] = (signed char)R;
                notop = notop || (R >= 0 && R != 3);
            }
            {
                // every load issued before the first store
                constexpr int per = (4 * kGtabPerDir + kTile * kTile - 1) / (kTile * kTile);
                real wv[per];
#pragma unroll
                for (int m = 0; m < per; ++m) {
                    const int q = (int)threadIdx.x + m * kTile * kTile;
                    wv[m] = q < 4 * kGtabPerDir ? A.gtab[((q / kGtabPerDir) * 2 + dir) * kGtabPerDir + q % kGtabPerDir]
                                                : real(0);
                }
#pragma unroll
                for (int m = 0; m < per; ++m) {
                    const int q = (int)threadIdx.x + m * kTile * kTile;
                    if (q < 4 * kGtabPerDir) L.w[q] = wv[m];
                }
            }
            // every face of the window at the top radius (or absent): no radius tests
            top = __syncthreads_and(!notop) != 0;
        } else {
            __syncthreads();
        }
        if (r + 1 < 8) fetch_round(J, r + 1, i0, j0, pre);
        if (own) {
            // the cell's own image, then (edge cells of an outflow axis) its ghosts
            real sum = real(0);
            if (top) {
                if (dir == 0) gather_sides<real, 0, false, true>(L, tx + 3, ty + 3, sum);
                else gather_sides<real, 1, false, true>(L, tx + 3, ty + 3, sum);
            } else {
                if (dir == 0) gather_sides<real, 0, false, false>(L, tx + 3, ty + 3, sum);
                else gather_sides<real, 1, false, false>(L, tx + 3, ty + 3, sum);
            }
            for (int qy = 0; qy < niy; ++qy)
                for (int qx = (qy == 0 ? 1 : 0); qx < nix; ++qx) {
                    const int bx = image(mi, nx, A.bcx, qx) - (i0 - 3), by = image(mj, ny, A.bcy, qy) - (j0 - 3);
                    if (dir == 0) gather_sides<real, 0, true, false>(L, bx, by, sum);
                    else gather_sides<real, 1, true, false>(L, bx, by, sum);
                }
            acc[v] += (double)sum;
        }
    }
    if (!own) return;
    const size_t k = (size_t)mj * nx + mi;
    const real alpha = A.s == 0 ? real(1) : (A.s == 1 ? real(0.25) : real(2) / real(3));
    const real beta = A.s == 0 ? real(0) : (A.s == 1 ? real(0.75) : real(1) / real(3));
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const size_t q = v * n + k;
        const real lo = J.lam_out[q];
        const real ls = (real)((double)(alpha * lo) + acc[v]);
        if (A.s > 0) {
            J.lam_Us[q] = ls;
            J.lam_Un[q] += beta * lo;
        } else {
            // U^n feeds both arguments of stage 0: fold in its other adjoint if given
            J.lam_Us[q] = J.lam_Un ? ls + J.lam_Un[q] : ls;
        }
    }
}

// ------------------------------------------------------------ dL/d(ell)
// The ell terms, in FP64, cell by cell.  Each face side is centred on a cell (or,
// on an outflow axis, on the ghost cell beyond a boundary face); the term of a
// side of radius R is the sum over its stencil positions e within R of
// d(w[p][e][c])/d(ell) x record[p][c] x the parity sum q[e][c] of the state
// around the centre (eq. (gp_reconstructor) differentiated in ell through the
// weights).  A cell forms the parity sums of each variable once and uses them for
// the four sides centred on it: in each direction the right side of its face
// below and the left side of its face above, one sum over e when the two faces
// have the same radius.  An edge cell of an outflow axis also takes the outer
// side of its boundary face.  Each block sums its cells' terms in a fixed order.

// Parity sums of variable plane U around (ci, cj) (unwrapped) at the kNPos
// stencil positions, in FP64.
template <typename real>
__device__ __forceinline__ void parity_sums(const StageArgs<real> &A, const real *U, int ci, int cj,
                                            double (&q)[kNPos][4])
{
    const int nx = A.nx, ny = A.ny;
    // the seven columns and rows around the centre, then every load, then the sums
    int xs[7];
    size_t ys[7];
#pragma unroll
    for (int d = 0; d < 7; ++d) {
        xs[d] = wrap(ci + d - 3, nx, A.bcx);
        ys[d] = (size_t)wrap(cj + d - 3, ny, A.bcy) * nx;
    }
    real u[kNPos][4];
#pragma unroll
    for (int e = 0; e < kNPos; ++e) {
        const int a = (int)((kPosA >> (4 * e)) & 15u), b = (int)((kPosB >> (4 * e)) & 15u);
        u[e][0] = U[ys[3 + b] + xs[3 + a]];
        u[e][1] = U[ys[3 + b] + xs[3 - a]];
        u[e][2] = U[ys[3 - b] + xs[3 + a]];
        u[e][3] = U[ys[3 - b] + xs[3 - a]];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int e = 0; e < kNPos; ++e)
        parity4((double)u[e][0], (double)u[e][1], (double)u[e][2], (double)u[e][3], q[e]);
}

// Sum over the positions e within radius R of dw[p][e][c] q[e][c] g[p][c] (dw:
// the ell derivatives of the weights of R and the face direction; g: the records
// of the sides, summed).  TOP: R is the top radius 3.
template <bool TOP>
__device__ __forceinline__ double ell_term(const double *dw, const double (&q)[kNPos][4], const double (&g)[2][4],
                                           int R)
{
    const int np = TOP ? kNPos : (R <= 0 ? 1 : (R == 1 ? 3 : (R == 2 ? 6 : 10)));
    double t = 0.0;
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            double sq = 0.0;
#pragma unroll
            for (int e = 0; e < kNPos; ++e)
                if (e < np) sq = fma(dw[p * (kNPos * 4) + e * 4 + c], q[e][c], sq);
            t = fma(g[p][c], sq, t);
        }
    return t;
}

// A side's record of variable v (8 values p, c) at face (fi, fj) of direction
// dir, added in FP64 to g.
template <typename real>
__device__ __forceinline__ void add_record(const AdjArgs<real> &J, int dir, int side, int v, int fi, int fj,
                                           double (&g)[2][4])
{
    const Quad<real> *blk = reinterpret_cast<const Quad<real> *>(record_block(J, dir, v, fi, fj)) + side * 2;
#pragma unroll
    for (int p = 0; p < 2; ++p) {
        const Quad<real> r = blk[p];
#pragma unroll
        for (int c = 0; c < 4; ++c) g[p][c] += (double)r.x[c];
    }
}

// dlw: J.dl64 again, as a restricted pointer the kernel never writes through, so
// that the block-uniform reads of the top-radius path are scalar loads.
template <typename real>
__global__ __launch_bounds__(256) void k_adj_dl(const AdjArgs<real> J, const double *__restrict__ dlw)
{
    __shared__ double red[256];
    __shared__ double dwl[4 * 2 * kGtabPerDir];  // the ell derivatives of the weights, [R][dir][.]
    for (int q = threadIdx.x; q < 4 * 2 * kGtabPerDir; q += blockDim.x) dwl[q] = J.dl64[q];
    __syncthreads();
    const StageArgs<real> &A = J.A;
    const int nx = A.nx, ny = A.ny;
    const size_t n = (size_t)nx * ny;
    const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dl = 0.0;
    if (k < n) {
        const int mj = (int)(k / nx), mi = (int)(k - (size_t)mj * nx);
        // the radii of the cell's faces (EDP_1: the smaller order of the two cells)
        const size_t row = (size_t)mj * nx;
        const int o = A.order[k], oxm = A.order[row + wrap(mi - 1, nx, A.bcx)], oxp = A.order[row + wrap(mi + 1, nx, A.bcx)];
        const int oym = A.order[(size_t)wrap(mj - 1, ny, A.bcy) * nx + mi], oyp = A.order[(size_t)wrap(mj + 1, ny, A.bcy) * nx + mi];
        const int R[2][2] = {{min(oxm, o), min(o, oxp)}, {min(oym, o), min(o, oyp)}};
        // face indices: below (fi, fj) = (mi, mj) in both directions; above, the
        // next index (on a periodic axis the face at the wrap is face 0)
        const int hx = A.bcx == 0 && mi + 1 == nx ? 0 : mi + 1, hy = A.bcy == 0 && mj + 1 == ny ? 0 : mj + 1;
        const bool top = __all(R[0][0] == 3 && R[0][1] == 3 && R[1][0] == 3 && R[1][1] == 3) != 0;
        for (int v = 0; v < 4; ++v) {
            const real *U = A.Us + (size_t)v * n;
            double q[kNPos][4];
            parity_sums(A, U, mi, mj, q);
#pragma unroll
            for (int dir = 0; dir < 2; ++dir) {
                double g[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
                add_record(J, dir, 1, v, mi, mj, g);  // right side of the face below
                if (top) {
                    add_record(J, dir, 0, v, dir == 0 ? hx : mi, dir == 0 ? mj : hy, g);
                    dl += ell_term<true>(dlw + (3 * 2 + dir) * kGtabPerDir, q, g, 3);
                } else {
                    const int R0 = R[dir][0], R1 = R[dir][1];
                    if (R0 == R1) add_record(J, dir, 0, v, dir == 0 ? hx : mi, dir == 0 ? mj : hy, g);
                    dl += ell_term<false>(dwl + (R0 * 2 + dir) * kGtabPerDir, q, g, R0);
                    if (R0 != R1) {
                        double h[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
                        add_record(J, dir, 0, v, dir == 0 ? hx : mi, dir == 0 ? mj : hy, h);
                        dl += ell_term<false>(dwl + (R1 * 2 + dir) * kGtabPerDir, q, h, R1);
                    }
                }
            }
            // outer sides of the boundary faces of an outflow axis, centred on ghosts
#pragma unroll 1
            for (int gk = 0; gk < 4; ++gk) {
                const int dir = gk >> 1, hi = gk & 1;
                const int m = dir == 0 ? mi : mj, nd = dir == 0 ? nx : ny;
                if ((dir == 0 ? A.bcx : A.bcy) == 0 || m != (hi ? nd - 1 : 0)) continue;
                const int ci = mi + (dir == 0 ? (hi ? 1 : -1) : 0), cj = mj + (dir == 1 ? (hi ? 1 : -1) : 0);
                double qg[kNPos][4];
                parity_sums(A, U, ci, cj, qg);
                double g[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
                // the left side of face 0, or the right side of face nd
                add_record(J, dir, hi ? 1 : 0, v, dir == 0 && hi ? nx : mi, dir == 1 && hi ? ny : mj, g);
                const int Rg = R[dir][hi];
                dl += ell_term<false>(dwl + (Rg * 2 + dir) * kGtabPerDir, qg, g, Rg);
            }
        }
    }
    red[threadIdx.x] = dl;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) J.dl_partial[blockIdx.x] = red[0];
}

// Fixed-order sum of the per-block partials into *out, or added to *out when
// accumulate is set (one block of 256 threads): thread t sums the contiguous
// chunk t in order, then a pairwise tree in LDS.  The order does not depend on
// timing, so the result is the same on every run.
__global__ __launch_bounds__(256) void k_adj_dl_final(const double *partial, int n, double *out, int accumulate)
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
    if (t == 0) *out = accumulate ? *out + red[0] : red[0];
}

template <typename real>
hipError_t launch_stage_vjp(const AdjArgs<real> &J, int nblk_faces, double *dl_out, bool accumulate, hipStream_t st)
{
    hipLaunchKernelGGL(k_adj_faces<real>, dim3(nblk_faces), dim3(128), 0, st, J);
    const int tiles = ((J.A.nx + kTile - 1) / kTile) * ((J.A.ny + kTile - 1) / kTile);
    hipLaunchKernelGGL(k_adj_cells<real>, dim3((unsigned)tiles), dim3(kTile * kTile), 0, st, J);
    // one thread per cell: ceil(nx ny / 256) <= tiles blocks, one partial each
    const int nblk_dl = (int)(((size_t)J.A.nx * J.A.ny + 255) / 256);
    hipLaunchKernelGGL(k_adj_dl<real>, dim3((unsigned)nblk_dl), dim3(256), 0, st, J, J.dl64);
    hipLaunchKernelGGL(k_adj_dl_final, dim3(1), dim3(256), 0, st, J.dl_partial, nblk_dl, dl_out, (int)accumulate);
    return hipGetLastError();
}

template hipError_t launch_stage_vjp<float>(const AdjArgs<float> &, int, double *, bool, hipStream_t);
template hipError_t launch_stage_vjp<double>(const AdjArgs<double> &, int, double *, bool, hipStream_t);

}  // namespace gpm
