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
// RK combine.  Every face flux (and its Riemann-state CAD flags) is stored for the
// cascade.  A troubled cell takes the next scheme of the cascade at once and is
// listed; a follow-up kernel claims its four faces and the five cells whose
// candidates they change.  No block barrier is needed: each wavefront only reads
// LDS it wrote itself.
//
// Cascade pass k (k_faces, then k_cells): recompute the claimed faces at their new
// EDP_1 order (min of the two cells' radii), then re-evaluate the claimed cells
// from the stored fluxes, re-detect, lower the troubled ones and claim the faces
// and cells of pass k+1.  Each face flux is computed once and read by both of its
// cells, so the update stays exactly conservative.  Every list holds each face or
// cell at most once (claim stamps), and both kernels read their item count from
// device memory and return at once when it is zero, so passes can be queued
// without a host round trip.
#include "gpmood_device.h"
#include "gpmood_launch.h"

namespace gpm {

constexpr int LW = 70;  // LDS columns per ring row: 64 lanes + 3 halo columns each side

// Claims after lowering cell (i, j) (act = this lane lowered it): its four faces
// (and, on periodic axes, the duplicate copy of a boundary face) are listed for
// recomputation in the next pass, and the cell with its four face neighbours for
// re-evaluation.  A stamp per face and per cell keeps each list duplicate-free.
// Must be reached by all 64 lanes of the wavefront together.
template <typename real>
__device__ __forceinline__ void claim_ids(const StageArgs<real> &A, int i, int j, int (&fid)[6], bool (&fok)[6],
                                          int (&cid)[5], bool (&cok)[5])
{
    const int nx = A.nx, ny = A.ny;
    const int nfx = (nx + 1) * ny;
    // faces: x faces i, i+1 of row j; y faces j, j+1 of column i; periodic duplicates
    fid[0] = j * (nx + 1) + i;
    fid[1] = j * (nx + 1) + i + 1;
    fid[2] = nfx + j * nx + i;
    fid[3] = nfx + (j + 1) * nx + i;
    fok[0] = fok[1] = fok[2] = fok[3] = true;
    fok[4] = A.bcx == 0 && (i == 0 || i == nx - 1);
    fid[4] = fok[4] ? (i == 0 ? j * (nx + 1) + nx : j * (nx + 1)) : fid[0];  // copy of face 0 / face nx
    fok[5] = A.bcy == 0 && (j == 0 || j == ny - 1);
    fid[5] = fok[5] ? (j == 0 ? nfx + ny * nx + i : nfx + i) : fid[2];      // copy of face 0 / face ny
    const int di[5] = {0, -1, 1, 0, 0}, dj[5] = {0, 0, 0, -1, 1};
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        const int ii = i + di[k], jj = j + dj[k];
        cok[k] = (A.bcx == 0 || (ii >= 0 && ii < nx)) && (A.bcy == 0 || (jj >= 0 && jj < ny));
        // (on a non-periodic axis only in-domain indices get here: no mirror needed)
        cid[k] = cok[k] ? wrap<false>(jj, ny, A.bcy) * nx + wrap<false>(ii, nx, A.bcx) : j * nx + i;
    }
}

template <typename real>
__device__ __forceinline__ void claim_after_lowering(const StageArgs<real> &A, const PassOut &P, int i, int j,
                                                     bool act)
{
    int fid[6], cid[5];
    bool fok[6], cok[5];
    claim_ids(A, i, j, fid, fok, cid, cok);
    bool fmine[6], cmine[5];
    int nmine = 0;
    if (act) {
        // all eleven stamp updates are issued back to back; an entry that does not
        // apply updates its own cell or face with 0, which changes nothing
        unsigned fo[6], co[5];
#pragma unroll
        for (int k = 0; k < 6; ++k) fo[k] = atomicMax(&A.fstamp[fid[k]], fok[k] ? P.stamp : 0u);
#pragma unroll
        for (int k = 0; k < 5; ++k) co[k] = atomicMax(&A.cstamp[cid[k]], cok[k] ? P.stamp : 0u);
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            fmine[k] = fok[k] && fo[k] < P.stamp;
            nmine += fmine[k] ? 1 : 0;
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            cmine[k] = cok[k] && co[k] < P.stamp;
            nmine += cmine[k] ? 65536 : 0;
        }
    } else {
#pragma unroll
        for (int k = 0; k < 6; ++k) fmine[k] = false;
#pragma unroll
        for (int k = 0; k < 5; ++k) cmine[k] = false;
    }
    int fb, cb;
    wave_reserve2(nmine, P.fcount, P.ccount, fb, cb);
    if (nmine != 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k)
            if (fmine[k]) P.flist[fb++] = fid[k];
#pragma unroll
        for (int k = 0; k < 5; ++k)
            if (cmine[k]) P.clist[cb++] = cid[k];
    }
}

// One wavefront's strip (tile wid of the problem) of the first pass; ring is the
// wavefront's LDS ring.  ISO: A.iso is 1 (the y states read the x weights).
// A lowered cell is only appended to P.clist (count P.ccount); its claims are
// made after the pass (k_claims_first, or k_claims_first_batch in a batch), which keeps
// the claim atomics, and the wait for their results, out of the march.
template <typename real, int RT, bool ISO, bool HLL, bool BND>
__device__ __forceinline__ void first_pass_wave(const StageArgs<real> &A, const PassOut &P, int wid,
                                                real (*ring)[4][LW])
{
    constexpr int q = nodes_of(RT);
    constexpr int NQ = kNQ[RT];
    const int lane = threadIdx.x & 63;

    const int nx = A.nx, ny = A.ny, T = A.rows;
    const int nstrip = (nx + 61) / 62, nseg = (ny + T - 1) / T;
    if (wid >= nstrip * nseg) return;  // whole wavefront leaves together
    const int sx = wid % nstrip, sy = wid / nstrip;
    const int x0 = sx * 62, y0 = sy * T;
    const int yend = min(y0 + T, ny);
    const int i = x0 - 1 + lane;
    const bool own_col = lane >= 1 && lane <= 62 && i < nx;
    const bool own = own_col;
    const size_t plane = (size_t)nx * ny;
    const size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);

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
    // Reflecting walls reverse the x momentum of mirrored columns and the y
    // momentum of mirrored rows; applied here, not at the load, which stays in flight.
    auto store_row = [&](int jr, real (&pf)[4][2]) {
        const int slot = jr & 7;
        // (BND: the build for grids with a reflecting axis or an inflow slit)
        if (BND && A.bcx == 2) {
            const int c0 = x0 - 4 + lane, c1 = c0 + 64;
            if (c0 < 0 || c0 >= nx) pf[1][0] = -pf[1][0];
            if (c1 >= nx) pf[1][1] = -pf[1][1];
        }
        if (BND && A.bcy == 2 && (jr < 0 || jr >= ny)) {
            pf[2][0] = -pf[2][0];
            pf[2][1] = -pf[2][1];
        }
        if (BND && A.slit && (((A.slit & 1) && jr < 0) || ((A.slit & 2) && jr >= ny))) {
            // ghost rows of an inflow slit hold the injected state
            const int c0 = x0 - 4 + lane, c1 = c0 + 64;
            const int side = jr < 0 ? 0 : 1;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                if (c0 >= A.si0 && c0 < A.si1) pf[v][0] = A.slitU[side][v];
                if (c1 >= A.si0 && c1 < A.si1) pf[v][1] = A.slitU[side][v];
            }
        }
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

    const real dt = uniform((real)(*A.dt * A.dtf));  // in a scalar register
    const real g = A.gamma;
    real sypP[q][4];   // y+ states of row j-1
    real Gprev[4];     // flux through face j-3/2
    real dFxP[4];      // x-flux difference of row j-1
    bool rsxP = false, rsymP = false;
    unsigned long long tmask = 0ull;  // this lane's lowered cells, bit (row - y0) mod 64
#pragma unroll
    for (int v = 0; v < 4; ++v) { Gprev[v] = real(0); dFxP[v] = real(0); }

    for (int j = y0 - 1; j <= yend; ++j) {
        // U^n of the cell this row completes, (i, j-1), issued before the row
        // prefetch: waiting for it later leaves the prefetch in flight
        real unp[4] = {real(0), real(0), real(0), real(0)};
        if (A.s != 0 && own && j - 1 >= y0) {
            const unsigned c = (unsigned)(j - 1) * (unsigned)nx + (unsigned)(x0 - 1 + lane_here());
#pragma unroll
            for (int v = 0; v < 4; ++v) unp[v] = (A.Un + v * plane)[c];
        }
        __builtin_amdgcn_sched_barrier(0);
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
            // x states also on the two rows that do not use them: no branch here
            states_dir<RT, 0, ISO>(Q, A.W, m_, p_);
#pragma unroll
            for (int k = 0; k < q; ++k) { sxm[k][v] = m_[k]; sxp[k][v] = p_[k]; }
            states_dir<RT, 1, ISO>(Q, A.W, m_, p_);
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
                riemann<0, HLL>(g, sxp[k], ur, f, bl, br);
                rsx = rsx || bl;
                badNb = badNb || br;
                const real w = node_weight<RT>(A.W, k);
#pragma unroll
                for (int v = 0; v < 4; ++v) F[v] = fma(w, f[v], F[v]);
            }
            // store face i+1/2: lanes of the strip's own cells, plus the domain's left face
            if ((own || (lane == 0 && x0 == 0)) && j < ny) {
                // 32-bit lane offsets from block-uniform bases (fewer live registers)
                const unsigned fi = (unsigned)j * (unsigned)(nx + 1) + (unsigned)(x0 + lane_here());  // face i + 1/2
#pragma unroll
                for (int v = 0; v < 4; ++v) (A.FX + v * nfx)[fi] = F[v];
                A.FXf[fi] = (uint8_t)((rsx ? 1 : 0) | (badNb ? 2 : 0));
            }
            // an inadmissible state on either side of the face troubles both of its
            // cells: this lane's cell takes faces i+1/2 and i-1/2 (the lane below's)
            const bool fbad = rsx || badNb;
            const int badm = __shfl_up((int)fbad, 1);
            rsx = fbad || (badm != 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) dFx[v] = F[v] - __shfl_up(F[v], 1);
        }

        if (!first) {
            real G[4] = {real(0), real(0), real(0), real(0)};
            bool badLy = false, badRy = false;
            real fh[q / 2 > 0 ? q / 2 : 1][4];  // HLL builds: fluxes of nodes 0 .. q/2-1, paired below
#pragma unroll
            for (int k = 0; k < q; ++k) {
                real f[4];
                bool bl, br;
                riemann<1, HLL>(g, sypP[k], sym[k], f, bl, br);
                badLy = badLy || bl;
                badRy = badRy || br;
                const real w = node_weight<RT>(A.W, k);
                if constexpr (HLL) {
                    // mirror-paired quadrature, (f_k + f_{q-1-k}) w_k: a mirror in x
                    // reverses the nodes of a y face, and the pairs keep the sum exact
                    if (2 * k + 1 < q) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) fh[k < q / 2 ? k : 0][v] = f[v];
                    } else if (2 * k + 1 == q) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) G[v] = fma(w, f[v], G[v]);
                    } else {
                        const int m = q - 1 - k;
#pragma unroll
                        for (int v = 0; v < 4; ++v) G[v] = fma(w, f[v] + fh[m < q / 2 ? m : 0][v], G[v]);
                    }
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) G[v] = fma(w, f[v], G[v]);
                }
            }
            // store face j-1/2 (y index j): the segment's faces above its first row,
            // plus the domain's bottom face
            if (own_col && (j > y0 || y0 == 0)) {
                const unsigned gi = (unsigned)j * (unsigned)nx + (unsigned)(x0 - 1 + lane_here());
#pragma unroll
                for (int v = 0; v < 4; ++v) (A.GY + v * nfy)[gi] = G[v];
                A.GYf[gi] = (uint8_t)((badLy ? 1 : 0) | (badRy ? 2 : 0));
            }
            if (j - 1 >= y0) {
                // cell (i, j-1) is complete
                const int jr = j - 1;
                const int slot = jr & 7;
                real us[4], ust[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    us[v] = ring[slot][v][lane + 3];
                    ust[v] = us[v] - dt * axis_sum(dv(dFxP[v], A.dx), dv(G[v] - Gprev[v], A.dy));
                }
                const bool rs = rsxP || rsymP || badLy || badRy;
                auto nb = [&](int di, int dj, int v) { return ring[(jr + dj) & 7][v][lane + 3 + di]; };
                const bool tr = own && troubled(A, RT, ust, rs, nb);
                if (own) {
                    const unsigned c = (unsigned)jr * (unsigned)nx + (unsigned)(x0 - 1 + lane_here());
#pragma unroll
                    for (int v = 0; v < 4; ++v) (A.Uout + v * plane)[c] = combine(A.s, unp[v], ust[v], A.ca, A.cb);
                    A.order[c] = (uint8_t)(tr ? A.next[RT] : RT);
                }
                // lowered cells are listed once per 64 rows of the march (once per
                // march at the default lengths), not row by row: the wait for the
                // slot an atomic returns would stall the march
                const int rb = (jr - y0) & 63;
                if (tr) tmask |= 1ull << rb;
                if (rb == 63 || jr == yend - 1) {  // the same in every lane
                    const int nt = __popcll(tmask);  // at most 64
                    int b, bt;
                    wave_reserve2(nt | (nt << 16), P.ccount, P.tcount, b, bt);
                    const int row0 = jr - rb;
                    for (unsigned long long m = tmask; m != 0ull; m &= m - 1ull)
                        P.clist[b++] = (row0 + __ffsll((long long)m) - 1) * nx + (x0 - 1 + lane_here());
                    tmask = 0ull;
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) Gprev[v] = G[v];
            rsymP = badLy || badRy;
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

template <typename real, int RT, int WPB, bool ISO, bool HLL, bool BND>
__global__ __launch_bounds__(64 * WPB, sizeof(real) == 4 ? 2 : 1) void k_first_pass(const StageArgs<real> A, const PassOut P)
{
    __shared__ real ring_all[WPB][8][4][LW];
    const int wv = threadIdx.x >> 6;
    first_pass_wave<real, RT, ISO, HLL, BND>(A, P, xcd_tile(blockIdx.x, gridDim.x) * WPB + wv, ring_all[wv]);
}

// The claims of the cells the first pass lowered (listed in low, count *nlow):
// the same claims, stamps and lists as if they had been made in the pass.
template <typename real>
__global__ __launch_bounds__(256) void k_claims_first(const StageArgs<real> A, const PassOut P, const int *low,
                                                      const int *nlow)
{
    const int n = *nlow;
    PassOut Q = P;
    Q.stamp = *A.stamp0;
    const int stride = gridDim.x * blockDim.x;
    const int nround = (n + stride - 1) / stride;
    for (int r = 0; r < nround; ++r) {
        const int t = r * stride + blockIdx.x * blockDim.x + threadIdx.x;
        const bool act = t < n;
        int i = 0, j = 0;
        if (act) {
            const int c = low[t];
            j = c / A.nx;
            i = c - j * A.nx;
        }
        claim_after_lowering(A, Q, i, j, act);
    }
}

// ------------------------------------------------------------- cascade pass
// The Riemann solver through a face normal to axis dir (runtime): the momenta are
// swapped into the x-face form and back, so the arithmetic is that of riemann<dir>.
template <bool HLL, typename real>
__device__ __forceinline__ void hllc_rt(real g, int dir, const real (&UL)[4], const real (&UR)[4], real (&F)[4],
                                        bool &badL, bool &badR)
{
    const real L[4] = {UL[0], dir ? UL[2] : UL[1], dir ? UL[1] : UL[2], UL[3]};
    const real Rr[4] = {UR[0], dir ? UR[2] : UR[1], dir ? UR[1] : UR[2], UR[3]};
    real f[4];
    riemann<0, HLL>(g, L, Rr, f, badL, badR);
    F[0] = f[0];
    F[1] = dir ? f[2] : f[1];
    F[2] = dir ? f[1] : f[2];
    F[3] = f[3];
}

// Per-wavefront LDS of the cascade's face work: 16 faces x 4 lanes, each lane with
// the 4 left and 4 right node states of its variable (later: one node's flux),
// and one flag word per lane.
template <typename real>
struct FaceXchg {
    real s[64][8];
    int fl[64];
};

// Copy the compact weight table into LDS (all NT threads of the block, every
// load issued before the first store; a block barrier must follow before it is
// read).
template <int NT, typename real>
__device__ __forceinline__ void load_gtab(const real *gtab, real *wl)
{
    constexpr int per = (kGtabSize + NT - 1) / NT;
    real v[per];
#pragma unroll
    for (int m = 0; m < per; ++m) {
        const int t = (int)threadIdx.x + m * NT;
        v[m] = t < kGtabSize ? gtab[t] : real(0);
    }
#pragma unroll
    for (int m = 0; m < per; ++m) {
        const int t = (int)threadIdx.x + m * NT;
        if (t < kGtabSize) wl[t] = v[m];
    }
}

// Cascade pass, part 1: recompute the listed faces at their EDP_1 order (the
// smaller radius of the two cells), four lanes per face.  Lane v of a quad
// gathers variable v of both cells' quarter positions (all loads issued at once),
// forms that variable's states at every Gauss node, and after an LDS transpose
// lane k solves the HLLC problem of node k; lane v then sums variable v of the
// node fluxes with the Gauss weights (eq. (fvm_F)).  The products and sums are
// those of the first pass (build_Q, states_dir, hllc), in the same order, with
// the multiplicity of on-axis positions folded into the table weights.
//
// A listed face borders a cell lowered in the previous evaluation, so its radius
// is below the top radius: at most 2 for GP-MOOD7.  Radius 3 (positions 6..9) is
// still handled, by a rolled loop.  The number of rounds is uniform across the
// wavefront (LDS exchange); wl is the LDS copy of the compact weight table.
// pre: when use_pre, this thread's list entry of round 0, loaded by the caller
// (while the count was still unknown).
template <bool WALLS, bool HLL, typename real>
__device__ __forceinline__ void faces_phase(const StageArgs<real> &A, const real *wl, FaceXchg<real> &X,
                                            const int *flist, int n, int t0, int stride, int pre = 0,
                                            bool use_pre = false)
{
    const int nx = A.nx, ny = A.ny;
    const int nfx = (nx + 1) * ny, nfy = nx * (ny + 1);
    const size_t plane = (size_t)nx * ny;
    const int lane = threadIdx.x & 63, v = lane & 3, q0 = lane & ~3;
    const int nround = (4 * n + stride - 1) / stride;
    for (int r = 0; r < nround; ++r) {
        const int idx = (r * stride + t0) >> 2;
        const bool valid = idx < n;
        int dir = 0, R = 0, fo = 0;
        bool tr = false;
        real PL[2][4], PR[2][4];  // [slot][component] of variable v, left and right cell
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int c = 0; c < 4; ++c) PL[p][c] = PR[p][c] = real(0);
        if (valid) {
            const int f = (use_pre && r == 0) ? pre : flist[idx];
            int iL, jL, cL, cR;
            if (f < nfx) {
                const int j = f / (nx + 1), i = f - j * (nx + 1);  // between cells i-1 and i
                dir = 0;
                fo = f;
                iL = i - 1;
                jL = j;
                cL = j * nx + wrap<WALLS>(i - 1, nx, A.bcx);
                cR = j * nx + wrap<WALLS>(i, nx, A.bcx);
            } else {
                const int g = f - nfx;
                const int j = g / nx, i = g - j * nx;  // between cells (i, j-1) and (i, j)
                dir = 1;
                fo = g;
                iL = i;
                jL = j - 1;
                cL = wrap<WALLS>(j - 1, ny, A.bcy) * nx + i;
                cR = wrap<WALLS>(j, ny, A.bcy) * nx + i;
            }
            const int iR = iL + (dir == 0), jR = jL + (dir == 1);
            const int oL = A.order[cL], oR = A.order[cR];  // issued ahead of the stencil loads
            // an isotropic y face computes what an x face computes on the transposed
            // grid: position (a, b) is gathered at offset (b, a) and the x table used
            tr = dir == 1 && A.iso;
            const real *U = A.Us + v * plane;
            // a gathered cell (xr, yr) (unwrapped) at wrapped offset yo + xo, sign sg;
            // the walls build also puts an inflow slit's state in its ghost cells
            const real slitb = A.slitU[0][v], slitt = A.slitU[1][v];
            auto gv = [&](int xr, int yr, size_t yo, int xo, real sg) -> real {
                return (WALLS && A.slit && in_slit(A, xr, yr)) ? (yr < 0 ? slitb : slitt) : sg * U[yo + xo];
            };
            // reflecting walls reverse the normal momentum of mirrored cells (WALLS:
            // the variant built for grids with a reflecting axis)
            const bool fx = WALLS && v == 1 && A.bcx == 2, fy = WALLS && v == 2 && A.bcy == 2;
            // quarter positions 0..5 (radius <= 2) of both cells: 48 independent loads
            constexpr int pa[6] = {0, 1, 0, 2, 0, 1}, pb[6] = {0, 0, 1, 0, 2, 1};
            real QL[6][4], QR[6][4];
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                const int xLp = wrap<WALLS>(iL + pa[e], nx, A.bcx), xLm = wrap<WALLS>(iL - pa[e], nx, A.bcx);
                const int xRp = wrap<WALLS>(iR + pa[e], nx, A.bcx), xRm = wrap<WALLS>(iR - pa[e], nx, A.bcx);
                const size_t yLp = (size_t)wrap<WALLS>(jL + pb[e], ny, A.bcy) * nx;
                const size_t yLm = (size_t)wrap<WALLS>(jL - pb[e], ny, A.bcy) * nx;
                const size_t yRp = (size_t)wrap<WALLS>(jR + pb[e], ny, A.bcy) * nx;
                const size_t yRm = (size_t)wrap<WALLS>(jR - pb[e], ny, A.bcy) * nx;
                const real sLp = msign<real>(iL + pa[e], nx, fx), sLm = msign<real>(iL - pa[e], nx, fx);
                const real sRp = msign<real>(iR + pa[e], nx, fx), sRm = msign<real>(iR - pa[e], nx, fx);
                const real tLp = msign<real>(jL + pb[e], ny, fy), tLm = msign<real>(jL - pb[e], ny, fy);
                const real tRp = msign<real>(jR + pb[e], ny, fy), tRm = msign<real>(jR - pb[e], ny, fy);
                const int a = pa[e], b = pb[e];
                parity4(gv(iL + a, jL + b, yLp, xLp, sLp * tLp), gv(iL - a, jL + b, yLp, xLm, sLm * tLp),
                        gv(iL + a, jL - b, yLm, xLp, sLp * tLm), gv(iL - a, jL - b, yLm, xLm, sLm * tLm), QL[e]);
                parity4(gv(iR + a, jR + b, yRp, xRp, sRp * tRp), gv(iR - a, jR + b, yRp, xRm, sRm * tRp),
                        gv(iR + a, jR - b, yRm, xRp, sRp * tRm), gv(iR - a, jR - b, yRm, xRm, sRm * tRm), QR[e]);
            }
            // a transposed y face takes position (a, b) from the gathered (b, a), OE and
            // EO exchanged: with the diagonal pairing these are the bits a transposed
            // gather would give
            constexpr int T6[6] = {0, 2, 1, 4, 3, 5};
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                if (T6[e] == e) {
                    const real lo = QL[e][C_OE], ro = QR[e][C_OE];
                    QL[e][C_OE] = tr ? QL[e][C_EO] : lo;
                    QL[e][C_EO] = tr ? lo : QL[e][C_EO];
                    QR[e][C_OE] = tr ? QR[e][C_EO] : ro;
                    QR[e][C_EO] = tr ? ro : QR[e][C_EO];
                } else if (T6[e] > e) {
                    const int f = T6[e];
                    real l0[4], l1[4], r0[4], r1[4];
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        l0[c] = QL[e][c]; l1[c] = QL[f][c];
                        r0[c] = QR[e][c]; r1[c] = QR[f][c];
                    }
                    QL[e][C_EE] = tr ? l1[C_EE] : l0[C_EE];
                    QL[e][C_OO] = tr ? l1[C_OO] : l0[C_OO];
                    QL[e][C_OE] = tr ? l1[C_EO] : l0[C_OE];
                    QL[e][C_EO] = tr ? l1[C_OE] : l0[C_EO];
                    QL[f][C_EE] = tr ? l0[C_EE] : l1[C_EE];
                    QL[f][C_OO] = tr ? l0[C_OO] : l1[C_OO];
                    QL[f][C_OE] = tr ? l0[C_EO] : l1[C_OE];
                    QL[f][C_EO] = tr ? l0[C_OE] : l1[C_EO];
                    QR[e][C_EE] = tr ? r1[C_EE] : r0[C_EE];
                    QR[e][C_OO] = tr ? r1[C_OO] : r0[C_OO];
                    QR[e][C_OE] = tr ? r1[C_EO] : r0[C_OE];
                    QR[e][C_EO] = tr ? r1[C_OE] : r0[C_EO];
                    QR[f][C_EE] = tr ? r0[C_EE] : r1[C_EE];
                    QR[f][C_OO] = tr ? r0[C_OO] : r1[C_OO];
                    QR[f][C_OE] = tr ? r0[C_EO] : r1[C_OE];
                    QR[f][C_EO] = tr ? r0[C_OE] : r1[C_EO];
                }
            }
            R = min(oL, oR);
            const real *wt = wl + (R * 2 + (tr ? 0 : dir)) * kGtabPerDir;
            const int np = R <= 0 ? 1 : (R == 1 ? 3 : (R == 2 ? 6 : 10));
#pragma unroll
            for (int e = 0; e < 6; ++e) {
                if (e < np) {
#pragma unroll
                    for (int p = 0; p < 2; ++p)
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            const real w = wt[p * (kNPos * 4) + e * 4 + c];
                            PL[p][c] = fma(w, QL[e][c], PL[p][c]);
                            PR[p][c] = fma(w, QR[e][c], PR[p][c]);
                        }
                }
            }
#pragma unroll 1
            for (int e = 6; e < np; ++e) {
                const int a0 = (int)((kPosA >> (4 * e)) & 15u), b0 = (int)((kPosB >> (4 * e)) & 15u);
                const int a = tr ? b0 : a0, b = tr ? a0 : b0;  // x and y offsets
                const int xLp = wrap<WALLS>(iL + a, nx, A.bcx), xLm = wrap<WALLS>(iL - a, nx, A.bcx);
                const int xRp = wrap<WALLS>(iR + a, nx, A.bcx), xRm = wrap<WALLS>(iR - a, nx, A.bcx);
                const size_t yLp = (size_t)wrap<WALLS>(jL + b, ny, A.bcy) * nx, yLm = (size_t)wrap<WALLS>(jL - b, ny, A.bcy) * nx;
                const size_t yRp = (size_t)wrap<WALLS>(jR + b, ny, A.bcy) * nx, yRm = (size_t)wrap<WALLS>(jR - b, ny, A.bcy) * nx;
                const real sLp = msign<real>(iL + a, nx, fx), sLm = msign<real>(iL - a, nx, fx);
                const real sRp = msign<real>(iR + a, nx, fx), sRm = msign<real>(iR - a, nx, fx);
                const real tLp = msign<real>(jL + b, ny, fy), tLm = msign<real>(jL - b, ny, fy);
                const real tRp = msign<real>(jR + b, ny, fy), tRm = msign<real>(jR - b, ny, fy);
                const real Lpp = gv(iL + a, jL + b, yLp, xLp, sLp * tLp), Lmm = gv(iL - a, jL - b, yLm, xLm, sLm * tLm);
                const real Lx = gv(iL - a, jL + b, yLp, xLm, sLm * tLp), Ly = gv(iL + a, jL - b, yLm, xLp, sLp * tLm);
                const real Lpm = tr ? Lx : Ly, Lmp = tr ? Ly : Lx;
                const real Rpp = gv(iR + a, jR + b, yRp, xRp, sRp * tRp), Rmm = gv(iR - a, jR - b, yRm, xRm, sRm * tRm);
                const real Rx = gv(iR - a, jR + b, yRp, xRm, sRm * tRp), Ry = gv(iR + a, jR - b, yRm, xRp, sRp * tRm);
                const real Rpm = tr ? Rx : Ry, Rmp = tr ? Ry : Rx;
                real ql[4], qr[4];
                parity4(Lpp, Lmp, Lpm, Lmm, ql);
                parity4(Rpp, Rmp, Rpm, Rmm, qr);
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        const real w = wt[p * (kNPos * 4) + e * 4 + c];
                        PL[p][c] = fma(w, ql[c], PL[p][c]);
                        PR[p][c] = fma(w, qr[c], PR[p][c]);
                    }
            }
        }
        const int q = R <= 0 ? 1 : R + 1;
        // states of variable v at node k (table order; slot 1 is the inner pair for
        // R = 3 and the centre node for R = 2; a single node has no +- partner)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int slot = (R >= 2 && k >= 1 && k <= q - 2) ? 1 : 0;
            const bool single = R <= 0 || (R == 2 && k == 1);
            const bool plus = k < (q >> 1);
            const real lee = slot ? PL[1][C_EE] : PL[0][C_EE], loe = slot ? PL[1][C_OE] : PL[0][C_OE];
            const real leo = slot ? PL[1][C_EO] : PL[0][C_EO], loo = slot ? PL[1][C_OO] : PL[0][C_OO];
            const real ree = slot ? PR[1][C_EE] : PR[0][C_EE], roe = slot ? PR[1][C_OE] : PR[0][C_OE];
            const real reo = slot ? PR[1][C_EO] : PR[0][C_EO], roo = slot ? PR[1][C_OO] : PR[0][C_OO];
            // odd across / along the face (a transposed y face is in the x-face frame)
            const bool yframe = dir == 1 && !tr;
            const real lF = yframe ? leo : loe, lN = yframe ? loe : leo;
            const real rF = yframe ? reo : roe, rN = yframe ? roe : reo;
            const real Ap = lee + lF, Cp = lN + loo;  // + face of the left cell
            const real Bm = ree - rF, Dm = rN - roo;  // - face of the right cell
            X.s[lane][k] = single ? Ap : (plus ? Ap + Cp : Ap - Cp);
            X.s[lane][4 + k] = single ? Bm : (plus ? Bm + Dm : Bm - Dm);
        }
        wave_lds_sync();
        real fk[4] = {real(0), real(0), real(0), real(0)};
        int flg = 0;
        if (valid && v < q) {  // lane v solves node k = v
            real UL[4], UR[4];
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                UL[w] = X.s[q0 + w][v];
                UR[w] = X.s[q0 + w][4 + v];
            }
            bool bl, br;
            hllc_rt<HLL>(A.gamma, dir, UL, UR, fk, bl, br);
            flg = (bl ? 1 : 0) | (br ? 2 : 0);
        }
        wave_lds_sync();
#pragma unroll
        for (int w = 0; w < 4; ++w) X.s[lane][w] = fk[w];
        X.fl[lane] = flg;
        wave_lds_sync();
        if (valid) {
            real F = real(0);
            int fl = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (k < q) {
                    const int slot = (R >= 2 && k >= 1 && k <= q - 2) ? 1 : 0;
                    if constexpr (HLL) {
                        // mirror-paired quadrature (see the first pass's y faces)
                        if (2 * k + 1 == q) F = fma(wl[kGtabNodeOff + R * 2 + slot], X.s[q0 + k][v], F);
                        else if (2 * k + 1 > q)
                            F = fma(wl[kGtabNodeOff + R * 2 + slot], X.s[q0 + k][v] + X.s[q0 + q - 1 - k][v], F);
                    } else {
                        F = fma(wl[kGtabNodeOff + R * 2 + slot], X.s[q0 + k][v], F);
                    }
                    fl |= X.fl[q0 + k];
                }
            }
            if (dir == 0) {
                A.FX[(size_t)v * nfx + fo] = F;
                if (v == 0) A.FXf[fo] = (uint8_t)fl;
            } else {
                A.GY[(size_t)v * nfy + fo] = F;
                if (v == 0) A.GYf[fo] = (uint8_t)fl;
            }
        }
        wave_lds_sync();  // the next round overwrites X
    }
}

// Cascade pass, part 2: re-evaluate the listed cells from the stored fluxes,
// re-detect, lower the troubled ones and claim the faces and cells of the next
// pass.  Detection reads no other cell's order, so lowering in place is safe.
// Everything a cell needs (fluxes, flags, its radius-2 neighbourhood) is loaded
// at once, up front.  The number of rounds is uniform across the wavefront.
//
// cell_load gathers what does not depend on this pass's fluxes (the stage input
// around the cell, U^n and its order); cell_finish reads the fluxes and flags,
// forms the candidate, detects, writes the result and lowers.  The tail issues
// cell_load while other wavefronts still recompute the faces.
constexpr int kDi13[13] = {0, -1, 1, 0, 0, -2, 2, 0, 0, -1, 1, -1, 1};
constexpr int kDj13[13] = {0, 0, 0, -1, 1, 0, 0, -2, 2, -1, -1, 1, 1};

template <typename real>
struct CellIn {
    int c, i, j, o;
    real rho[13];     // radius-2 diamond of densities (kDi13, kDj13)
    real mom[5][3];   // the other variables of the cell and its face neighbours
    real un[4];       // U^n of the cell (stages 1, 2)
};

template <bool WALLS, typename real>
__device__ __forceinline__ void cell_load(const StageArgs<real> &A, int c, CellIn<real> &X)
{
    const int nx = A.nx, ny = A.ny;
    const size_t plane = (size_t)nx * ny;
    X.c = c;
    X.j = c / nx;
    X.i = c - X.j * nx;
    size_t yr[5];
    int xc[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) {
        yr[d] = (size_t)wrap<WALLS>(X.j + d - 2, ny, A.bcy) * nx;
        xc[d] = wrap<WALLS>(X.i + d - 2, nx, A.bcx);
    }
#pragma unroll
    for (int m = 0; m < 13; ++m) X.rho[m] = A.Us[yr[kDj13[m] + 2] + xc[kDi13[m] + 2]];
#pragma unroll
    for (int m = 0; m < 5; ++m)
#pragma unroll
        for (int w = 1; w < 4; ++w) X.mom[m][w - 1] = A.Us[w * plane + yr[kDj13[m] + 2] + xc[kDi13[m] + 2]];
    // reflecting walls reverse the normal momentum of a mirrored face neighbour;
    // an inflow slit's ghost cells hold the injected state
    if (WALLS) {
#pragma unroll
        for (int m = 1; m < 5; ++m) {
            X.mom[m][0] *= msign<real>(X.i + kDi13[m], nx, A.bcx == 2);
            X.mom[m][1] *= msign<real>(X.j + kDj13[m], ny, A.bcy == 2);
        }
        if (A.slit) {
#pragma unroll
            for (int m = 1; m < 13; ++m) {
                const bool s = in_slit(A, X.i + kDi13[m], X.j + kDj13[m]);
                const int side = X.j + kDj13[m] < 0 ? 0 : 1;
                X.rho[m] = s ? A.slitU[side][0] : X.rho[m];
                if (m < 5)
#pragma unroll
                    for (int w = 1; w < 4; ++w) X.mom[m][w - 1] = s ? A.slitU[side][w] : X.mom[m][w - 1];
            }
        }
    }
#pragma unroll
    for (int w = 0; w < 4; ++w) X.un[w] = A.s == 0 ? real(0) : A.Un[w * plane + c];
    X.o = A.order[c];
}

// The stored fluxes and Riemann-state flags of a cell's four faces (faces i-1/2,
// i+1/2, j-1/2, j+1/2; fid: their face ids as the claims list them).
template <typename real>
struct CellFlux {
    real f[4][4];  // [face][variable]
    int fl[4];
    int fid[4];
};

template <typename real>
__device__ __forceinline__ void cell_fetch(const StageArgs<real> &A, const CellIn<real> &X, CellFlux<real> &F)
{
    const int nx = A.nx, ny = A.ny;
    const size_t nfx = (size_t)(nx + 1) * ny, nfy = (size_t)nx * (ny + 1);
    const size_t fxm = (size_t)X.j * (nx + 1) + X.i, gym = (size_t)X.j * nx + X.i;  // faces i-1/2, j-1/2
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        F.f[0][w] = A.FX[w * nfx + fxm];
        F.f[1][w] = A.FX[w * nfx + fxm + 1];
        F.f[2][w] = A.GY[w * nfy + gym];
        F.f[3][w] = A.GY[w * nfy + gym + nx];
    }
    F.fl[0] = A.FXf[fxm];
    F.fl[1] = A.FXf[fxm + 1];
    F.fl[2] = A.GYf[gym];
    F.fl[3] = A.GYf[gym + nx];
    F.fid[0] = (int)fxm;
    F.fid[1] = (int)fxm + 1;
    F.fid[2] = (int)(nfx + gym);
    F.fid[3] = (int)(nfx + gym + nx);
    // every flux and flag is consumed here: the flag loads are issued with the
    // flux loads (not sunk into the branch of the detection that reads them), and
    // the cell waits once for all of them
    asm volatile("" ::"v"(F.fl[0]), "v"(F.fl[1]), "v"(F.fl[2]), "v"(F.fl[3]), "v"(F.f[0][0]), "v"(F.f[0][1]),
                 "v"(F.f[0][2]), "v"(F.f[0][3]), "v"(F.f[1][0]), "v"(F.f[1][1]), "v"(F.f[1][2]), "v"(F.f[1][3]),
                 "v"(F.f[2][0]), "v"(F.f[2][1]), "v"(F.f[2][2]), "v"(F.f[2][3]), "v"(F.f[3][0]), "v"(F.f[3][1]),
                 "v"(F.f[3][2]), "v"(F.f[3][3]));
}

// Returns whether the cell is troubled (it has then been lowered).
template <typename real>
__device__ __forceinline__ bool cell_finish_flux(const StageArgs<real> &A, const CellIn<real> &X,
                                                 const CellFlux<real> &F, real dt)
{
    const size_t plane = (size_t)A.nx * A.ny;
    // an inadmissible state on either side of any of the cell's faces
    const bool rs = (F.fl[0] | F.fl[1] | F.fl[2] | F.fl[3]) != 0;
    real ust[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const real us = w == 0 ? X.rho[0] : X.mom[0][w - 1];
        const real dFx = F.f[1][w] - F.f[0][w];
        ust[w] = us - dt * axis_sum(dv(dFx, A.dx), dv(F.f[3][w] - F.f[2][w], A.dy));
    }
    auto nb = [&](int di, int dj, int w) -> real {
        int m = 0;
#pragma unroll
        for (int t = 0; t < 13; ++t)
            if (kDi13[t] == di && kDj13[t] == dj) m = t;
        return w == 0 ? X.rho[m] : X.mom[m < 5 ? m : 0][w - 1];
    };
    const bool tr = troubled(A, X.o, ust, rs, nb);
#pragma unroll
    for (int w = 0; w < 4; ++w) A.Uout[w * plane + X.c] = combine(A.s, X.un[w], ust[w], A.ca, A.cb);
    if (tr) A.order[X.c] = (uint8_t)next_radius(A.next[0], A.next[1], A.next[2], A.next[3], X.o);
    return tr;
}

template <typename real>
__device__ __forceinline__ bool cell_finish(const StageArgs<real> &A, const CellIn<real> &X, real dt)
{
    CellFlux<real> F;
    cell_fetch(A, X, F);
    return cell_finish_flux(A, X, F, dt);
}

template <bool WALLS, typename real>
__device__ __forceinline__ void cells_phase(const StageArgs<real> &A, const int *clist, int n, int t0, int stride,
                                            const PassOut &P, real dt, int pre = 0, bool use_pre = false)
{
    const int nround = (n + stride - 1) / stride;
    for (int r = 0; r < nround; ++r) {
        const int idx = r * stride + t0;
        const bool valid = idx < n;
        bool tr = false;
        int i = 0, j = 0;
        if (valid) {
            CellIn<real> X;
            cell_load<WALLS>(A, (use_pre && r == 0) ? pre : clist[idx], X);
            tr = cell_finish(A, X, dt);
            i = X.i;
            j = X.j;
        }
        wave_count(tr, P.tcount);
        claim_after_lowering(A, P, i, j, tr);
    }
}

// Outputs of cascade pass k.
__device__ __forceinline__ PassOut pass_out(const Cascade &C, int k, unsigned stamp0)
{
    PassOut P;
    P.flist = C.flist[(k + 1) & 1];
    P.fcount = &C.ctl->nface[k + 1];
    P.clist = C.clist[(k + 1) & 1];
    P.ccount = &C.ctl->ncell[k + 1];
    P.tcount = &C.ctl->ntroub[k];
    P.stamp = stamp0 + (unsigned)k;
    return P;
}

// Does multi-block pass k run?  Not when it has nothing to do, nor when the
// previous evaluation left few troubled cells (the tail takes over from k).
__device__ __forceinline__ bool pass_runs(const Cascade &C, int k)
{
    return C.ctl->ncell[k] > 0 && C.ctl->ntroub[k - 1] > C.tail_thr;
}

template <typename real, bool WALLS, bool HLL>
__global__ __launch_bounds__(256) void k_faces(const StageArgs<real> A, const Cascade C, int k)
{
    __shared__ real wl[kGtabSize];
    __shared__ FaceXchg<real> xch[4];
    const int cap = (A.nx + 1) * A.ny + A.nx * (A.ny + 1);
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    // issued together, before the counts are known: this thread's first list
    // entry (in bounds; used only if the pass runs and covers it) and the weights
    const int i0 = t0 >> 2;
    const int pre = C.flist[k & 1][i0 < cap ? i0 : cap - 1];
    load_gtab<256>(A.gtab, wl);
    if (!pass_runs(C, k)) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && C.ctl->ncell[k] > 0) C.ctl->tail_k0 = k;
        return;
    }
    int n = C.ctl->nface[k];
    n = n < cap ? n : cap;  // a list holds each face at most once
    if (4 * n <= (int)(blockIdx.x * blockDim.x)) return;  // no face for this block
    __syncthreads();
    faces_phase<WALLS, HLL>(A, wl, xch[threadIdx.x >> 6], C.flist[k & 1], n, t0, gridDim.x * blockDim.x, pre, true);
}

template <typename real, bool WALLS>
__global__ __launch_bounds__(64) void k_cells(const StageArgs<real> A, const Cascade C, int k)
{
    const int cap = A.nx * A.ny;
    const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
    // this thread's first list entry, issued before the counts are known (in bounds)
    const int pre = C.clist[k & 1][t0 < cap ? t0 : cap - 1];
    const real dt = (real)(*A.dt * A.dtf);
    if (!pass_runs(C, k)) return;
    int n = C.ctl->ncell[k];
    n = n < cap ? n : cap;  // a list holds each cell at most once
    if (n <= (int)(blockIdx.x * blockDim.x)) return;
    cells_phase<WALLS>(A, C.clist[k & 1], n, t0, gridDim.x * blockDim.x, pass_out(C, k, C.ctl->stamp0), dt, pre, true);
}

// The tail of a long cascade (few troubled cells per pass) in one workgroup:
// passes run back to back with block barriers, from tail_k0 (or kdef when the
// multi-block passes did not hand over), until a pass has no cell to re-evaluate,
// kend is reached, or the previous evaluation left more than back_thr troubled
// cells (hand back to the multi-block passes).  The counts of the running passes
// stay in LDS and are copied to the control block as each pass completes.
// Threads of the tail workgroup: 512 (two wavefronts per SIMD, at most 256
// registers a lane); 256 in the FP64 build for walls and slits, whose cell and
// face state needs more than 256 registers (one wavefront per SIMD gives it 512,
// with no spill to scratch).
template <typename real, bool WALLS>
constexpr int tail_threads()
{
    return sizeof(real) == 8 && WALLS ? 256 : 512;
}
constexpr int kTailMaxWaves = 8;

// LDS of the single-workgroup cascade.
template <typename real>
struct TailShared {
    real wl[kGtabSize];
    FaceXchg<real> xch[kTailMaxWaves];
    int cnt[2][3];  // [pass parity][faces, cells, troubled cells of the previous evaluation]
    int kfirst;
};

template <bool WALLS, bool HLL, typename real>
__device__ __forceinline__ void tail_body(const StageArgs<real> &A, const Cascade &C, int kbeg, int kdef, int kend,
                                          TailShared<real> &S)
{
    const int capf = (A.nx + 1) * A.ny + A.nx * (A.ny + 1), capc = A.nx * A.ny;
    Ctl *ctl = C.ctl;
    const unsigned stamp0 = ctl->stamp0;
    const real dtr = (real)(*A.dt * A.dtf);  // read once, not after each pass's barrier
    load_gtab<tail_threads<real, WALLS>()>(A.gtab, S.wl);
    int k0 = ctl->tail_k0 > 0 ? ctl->tail_k0 : kdef;
    if (ctl->tail_k0 <= 0 && kbeg < kdef) {
        // no hand-over: the cascade either ended inside the batch kbeg..kdef-1 (at
        // the first pass with no cell) or continues at kdef
        if (threadIdx.x == 0) S.kfirst = kdef;
        __syncthreads();
        for (int kk = kbeg + (int)threadIdx.x; kk < kdef; kk += blockDim.x)
            if (ctl->ncell[kk] <= 0) atomicMin(&S.kfirst, kk);
        __syncthreads();
        k0 = S.kfirst;
    }
    if (threadIdx.x == 0) {
        S.cnt[k0 & 1][0] = ctl->nface[k0];
        S.cnt[k0 & 1][1] = ctl->ncell[k0];
        S.cnt[k0 & 1][2] = ctl->ntroub[k0 - 1];
    }
    int k = k0;
    bool back = false;
    for (; k < kend; ++k) {
        __syncthreads();  // the previous pass's lists, counts and fluxes are complete
        // the same value in every lane: held in scalar registers, so the branches
        // below (some around block barriers) are scalar
        int nf = __builtin_amdgcn_readfirstlane(S.cnt[k & 1][0]);
        int nc = __builtin_amdgcn_readfirstlane(S.cnt[k & 1][1]);
        const int nt = __builtin_amdgcn_readfirstlane(S.cnt[k & 1][2]);
        if (threadIdx.x == 0 && k > k0) {
            ctl->nface[k] = nf;
            ctl->ncell[k] = nc;
            ctl->ntroub[k - 1] = nt;
        }
        nc = nc < capc ? nc : capc;
        nf = nf < capf ? nf : capf;
        if (nc <= 0) break;  // same values in every thread: the block leaves together
        if (nt > C.back_thr) {
            back = true;
            break;
        }
        if (threadIdx.x == 0) S.cnt[(k + 1) & 1][0] = S.cnt[(k + 1) & 1][1] = S.cnt[(k + 1) & 1][2] = 0;
        PassOut P = pass_out(C, k, stamp0);
        P.fcount = &S.cnt[(k + 1) & 1][0];
        P.ccount = &S.cnt[(k + 1) & 1][1];
        P.tcount = &S.cnt[(k + 1) & 1][2];
        const int fw = (4 * nf + 63) >> 6, cw = (nc + 63) >> 6;  // wavefronts of faces, of cells
        const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);  // uniform per wavefront
        if (fw + cw <= tail_threads<real, WALLS>() / 64) {
            // one round each, on separate wavefronts: the cell wavefronts gather
            // their inputs while the face wavefronts recompute the fluxes
            const int c0 = tail_threads<real, WALLS>() / 64 - cw;  // first cell wavefront
            const bool cellwave = wv >= c0;
            const int idx = (int)threadIdx.x - 64 * c0;
            const bool valid = cellwave && idx < nc;
            CellIn<real> X;
            X.i = X.j = 0;
            if (valid) cell_load<WALLS>(A, C.clist[k & 1][idx], X);
            if (!cellwave && wv < fw)
                faces_phase<WALLS, HLL>(A, S.wl, S.xch[wv], C.flist[k & 1], nf, threadIdx.x, 64 * fw);
            __syncthreads();
            if (cellwave) {
                bool tr = false;
                if (valid) tr = cell_finish(A, X, dtr);
                wave_count(tr, P.tcount);
                claim_after_lowering(A, P, X.i, X.j, tr);
            }
        } else {
            faces_phase<WALLS, HLL>(A, S.wl, S.xch[wv], C.flist[k & 1], nf, threadIdx.x, blockDim.x);
            __syncthreads();
            cells_phase<WALLS>(A, C.clist[k & 1], nc, threadIdx.x, blockDim.x, P, dtr);
        }
    }
    if (k >= kend) {
        __syncthreads();
        if (threadIdx.x == 0) {
            ctl->nface[k] = S.cnt[k & 1][0];
            ctl->ncell[k] = S.cnt[k & 1][1];
            ctl->ntroub[k - 1] = S.cnt[k & 1][2];
        }
    }
    if (threadIdx.x == 0) {
        ctl->tail_end = k;
        ctl->tail_back = back ? 1 : 0;
        ctl->tail_start = k0;
        if (back) ctl->tail_k0 = 0;  // the next multi-block batch starts afresh
    }
}

template <typename real, bool WALLS, bool HLL>
__global__ __launch_bounds__((tail_threads<real, WALLS>())) void k_tail(const StageArgs<real> A, const Cascade C, int kbeg, int kdef,
                                                       int kend)
{
    __shared__ TailShared<real> S;
    tail_body<WALLS, HLL>(A, C, kbeg, kdef, kend, S);
}

// -------------------------------------------------------- small kernels
__global__ void k_reset(Ctl *ctl, int nzero, unsigned stamp0)
{
    for (int k = threadIdx.x; k < nzero && k < kMaxPasses + 2; k += blockDim.x) {
        ctl->nface[k] = 0;
        ctl->ncell[k] = 0;
        ctl->ntroub[k] = 0;
    }
    if (threadIdx.x == 0) {
        ctl->tail_end = 0;
        ctl->tail_k0 = 0;
        ctl->tail_back = 0;
        ctl->stamp0 = stamp0;
        ctl->nlow = 0;
    }
}

// Histogram of the final cascade level of every cell (for statistics only).
__global__ __launch_bounds__(256) void k_level_hist(const uint8_t *order, size_t ncell, const LevIdx levidx,
                                                    unsigned long long *levcnt)
{
    __shared__ unsigned int h[4];
    if (threadIdx.x < 4) h[threadIdx.x] = 0;
    __syncthreads();
    unsigned int loc[4] = {0, 0, 0, 0};
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < ncell; k += (size_t)gridDim.x * blockDim.x) {
        const int r = order[k] & 3;
        loc[0] += r == 0;
        loc[1] += r == 1;
        loc[2] += r == 2;
        loc[3] += r == 3;
    }
    for (int r = 0; r < 4; ++r)
        if (loc[r]) atomicAdd(&h[r], loc[r]);
    __syncthreads();
    if (threadIdx.x < 4 && h[threadIdx.x]) atomicAdd(&levcnt[levidx.v[threadIdx.x]], (unsigned long long)h[threadIdx.x]);
}

__global__ void k_zero_levcnt(Ctl *ctl)
{
    if (threadIdx.x < 4) ctl->levcnt[threadIdx.x] = 0ull;
}

// Instrumentation: add this stage's final-order counts and MOOD iterations
// (1 + cascade passes that re-evaluated cells) to the accumulators.
__global__ void k_stats_accum(Ctl *ctl, int npass, int reset)
{
    __shared__ unsigned long long cnt;
    if (threadIdx.x == 0) cnt = 0ull;
    __syncthreads();
    if (reset) {
        if (threadIdx.x < 4) ctl->acc_lev[threadIdx.x] = 0ull;
        if (threadIdx.x == 0) {
            ctl->acc_iters = 0ull;
            ctl->acc_stages = 0ull;
        }
        return;
    }
    unsigned long long loc = 0;
    for (int k = 1 + threadIdx.x; k <= npass && k < kMaxPasses + 2; k += blockDim.x) loc += ctl->ncell[k] > 0;
    if (loc) atomicAdd(&cnt, loc);
    __syncthreads();
    if (threadIdx.x < 4) ctl->acc_lev[threadIdx.x] += ctl->levcnt[threadIdx.x];
    if (threadIdx.x == 0) {
        ctl->acc_iters += 1ull + cnt;
        ctl->acc_stages += 1ull;
    }
}

// max over cells of (|u_d| + c) / Delta_d in FP64, as the bit pattern of a
// non-negative double (which orders like the integer).
template <typename real>
__device__ __forceinline__ void dt_reduce_body(const real *U, size_t ncell, double gamma, double dx, double dy,
                                               unsigned long long *lam_bits, size_t first, size_t stride,
                                               double *red)
{
    double lam = 0.0;
    // four cells per round, their 16 loads issued before the arithmetic (the
    // maximum does not depend on the order)
    constexpr int kU = 4;
    for (size_t k0 = first; k0 < ncell; k0 += kU * stride) {
        double q[kU][4];
#pragma unroll
        for (int m = 0; m < kU; ++m) {
            const size_t k = k0 + (size_t)m * stride;
            const size_t kk = k < ncell ? k : first;  // in bounds; the cell is skipped below
#pragma unroll
            for (int v = 0; v < 4; ++v) q[m][v] = U[(size_t)v * ncell + kk];
        }
#pragma unroll
        for (int m = 0; m < kU; ++m) {
            if (k0 + (size_t)m * stride >= ncell) continue;
            const double r = q[m][0], mx = q[m][1], my = q[m][2], E = q[m][3];
            const double p = (gamma - 1.0) * (E - 0.5 * (mx * mx + my * my) / r);
            if (!(r > 0.0 && p > 0.0 && __builtin_isfinite(r) && __builtin_isfinite(p))) continue;
            const double cs = sqrt(gamma * p / r);
            const double lx = (fabs(mx / r) + cs) / dx;
            const double ly = (fabs(my / r) + cs) / dy;
            const double l = lx > ly ? lx : ly;
            lam = l > lam ? l : lam;
        }
    }
    red[threadIdx.x] = lam;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && red[0] > 0.0) {
        // the maximum only grows (the bit patterns of positive doubles order as
        // the values): a block whose value does not exceed the one already stored
        // skips its atomic, so the blocks do not queue on the one address
        const unsigned long long b = (unsigned long long)__double_as_longlong(red[0]);
        if (b > __hip_atomic_load(lam_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(lam_bits, b);
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_dt_reduce(const real *U, size_t ncell, double gamma, double dx,
                                                   double dy, unsigned long long *lam_bits)
{
    __shared__ double red[256];
    dt_reduce_body(U, ncell, gamma, dx, dy, lam_bits, (size_t)blockIdx.x * blockDim.x + threadIdx.x,
                   (size_t)gridDim.x * blockDim.x, red);
}

// lam0: a lower bound of the largest wave speed over cell size (an inflow slit's
// state), 0 if none.
__global__ void k_dt_finalize(Ctl *ctl, double cfl, double lam0)
{
    const double lam = __longlong_as_double((long long)ctl->lam_bits);
    ctl->dt = cfl / (lam > lam0 ? lam : lam0);
}

__global__ void k_dt_set(Ctl *ctl, double dt, int clear_lambda)
{
    if (clear_lambda) ctl->lam_bits = 0ull;
    else ctl->dt = dt;
}

// out = w0 x0 + w1 x1 + w2 x2 + w3 x3, evaluated left to right, element by element.
template <typename real>
__global__ __launch_bounds__(256) void k_lincomb4(real *out, const real *x0, const real *x1, const real *x2,
                                                  const real *x3, real w0, real w1, real w2, real w3, size_t n)
{
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (size_t)gridDim.x * blockDim.x)
        out[k] = ((w0 * x0[k] + w1 * x1[k]) + w2 * x2[k]) + w3 * x3[k];
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

__global__ void k_totals_final(const double *partial, int nblk, double area, double *out)
{
    const int v = threadIdx.x;
    if (v >= 4) return;
    double hi = 0.0, lo = 0.0;
    for (int b = 0; b < nblk; ++b) {
        dd_add(hi, lo, partial[(v * nblk + b) * 2]);
        dd_add(hi, lo, partial[(v * nblk + b) * 2 + 1]);
    }
    out[v] = (hi + lo) * area;
}

// ------------------------------------------------------------- launchers
// ------------------------------------------------------------ batched ensemble
// Many independent problems advance together: one first-pass launch over all
// their strips, one single-workgroup cascade per problem in one launch, and the
// per-problem dt in three small launches.  The per-problem arguments live in
// device tables written once; they are read through the constant address space
// (scalar loads: the tables do not change while the kernels run).
// Generic reference to entry p of a device table, loaded as constant memory.
template <typename T>
__device__ __forceinline__ const T &table_entry(const T *tab, int p)
{
    return *(const T *)(((cptr<T>)tab) + p);
}

__device__ __forceinline__ int find_problem(cptr<int> prefix, int n, int b)
{
    int lo = 0, hi = n;  // prefix[lo] <= b < prefix[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (prefix[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <typename real, int RT, int WPB, bool ISO, bool HLL, bool BND>
__global__ __launch_bounds__(64 * WPB, sizeof(real) == 4 ? 2 : 1) void k_first_pass_batch(const BatchTabs<real> B)
{
    __shared__ real ring_all[WPB][8][4][LW];
    cptr<int> blk = (cptr<int>)B.blk;
    const int p = find_problem(blk, B.nprob, blockIdx.x);
    const StageArgs<real> &A = table_entry(B.args, p);
    const Cascade &C = table_entry(B.casc, p);
    PassOut Q = table_entry(B.pout, p);
    // lowered cells are listed in clist[0]; k_claims_first_batch makes their claims
    Q.clist = C.clist[0];
    Q.ccount = &C.ctl->nlow;
    const int wv = threadIdx.x >> 6;
    first_pass_wave<real, RT, ISO, HLL, BND>(A, Q, (blockIdx.x - blk[p]) * WPB + wv, ring_all[wv]);
}

// Multi-block cascade passes of a batch.  Before each pass, k_batch_plan sizes
// every problem's share of the pass (0 when it has no work, or when its previous
// evaluation left at most tail_thr troubled cells, which then leaves the rest of
// its cascade to its tail workgroup) and lays the shares end to end: plan[p] is
// the first work block of problem p, in units of 64 faces (256 threads) and,
// at plan + nprob + 1, of 64 cells.  The pass kernels have a fixed grid whose
// blocks stride over these work blocks, so the whole batch's faces and cells of a
// pass are spread over the GPU however they fall among the problems.  Pass 0 is
// the claims of the cells the first passes lowered (64 x 4 cells per block).
constexpr int kBatchPasses = 12;
constexpr int kBatchFaceGrid = 1024, kBatchCellGrid = 2048;

template <typename real>
__global__ __launch_bounds__(1024) void k_batch_plan(const BatchTabs<real> B, int k, int *plan)
{
    __shared__ int sf[1024], sc[1024];
    __shared__ int carry[2];
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    for (int base = 0; base < B.nprob; base += blockDim.x) {
        const int p = base + (int)threadIdx.x;
        int df = 0, dc = 0;
        if (p < B.nprob) {
            const StageArgs<real> &A = table_entry(B.args, p);
            const Cascade &C = table_entry(B.casc, p);
            if (k == 0) {
                df = (C.ctl->nlow + 255) / 256;
            } else if (pass_runs(C, k)) {
                const int capf = (A.nx + 1) * A.ny + A.nx * (A.ny + 1), capc = A.nx * A.ny;
                const int nf = min(C.ctl->nface[k], capf), nc = min(C.ctl->ncell[k], capc);
                df = (nf + 63) / 64;
                dc = (nc + 63) / 64;
            } else if (C.ctl->ncell[k] > 0) {
                C.ctl->tail_k0 = k;  // the tail takes over from this pass
            }
        }
        sf[threadIdx.x] = df;
        sc[threadIdx.x] = dc;
        __syncthreads();
        // inclusive scan (Hillis-Steele) of both demands
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            const int tf = threadIdx.x >= (unsigned)off ? sf[threadIdx.x - off] : 0;
            const int tc = threadIdx.x >= (unsigned)off ? sc[threadIdx.x - off] : 0;
            __syncthreads();
            sf[threadIdx.x] += tf;
            sc[threadIdx.x] += tc;
            __syncthreads();
        }
        if (p < B.nprob) {
            plan[p] = carry[0] + sf[threadIdx.x] - df;
            plan[B.nprob + 1 + p] = carry[1] + sc[threadIdx.x] - dc;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            carry[0] += sf[blockDim.x - 1];
            carry[1] += sc[blockDim.x - 1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        plan[B.nprob] = carry[0];
        plan[2 * B.nprob + 1] = carry[1];
    }
}

// The claims of the cells each problem's first pass lowered.
template <typename real>
__global__ __launch_bounds__(256) void k_claims_first_batch(const BatchTabs<real> B, const int *plan)
{
    cptr<int> pl = (cptr<int>)plan;
    const int total = pl[B.nprob];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int p = find_problem(pl, B.nprob, w);
        const StageArgs<real> &A = table_entry(B.args, p);
        const Cascade &C = table_entry(B.casc, p);
        PassOut P = table_entry(B.pout, p);
        P.stamp = *A.stamp0;
        const int t = (w - pl[p]) * 256 + (int)threadIdx.x;
        const bool act = t < C.ctl->nlow;
        int i = 0, j = 0;
        if (act) {
            const int c = C.clist[0][t];
            j = c / A.nx;
            i = c - j * A.nx;
        }
        claim_after_lowering(A, P, i, j, act);
    }
}

template <typename real, bool WALLS, bool HLL>
__global__ __launch_bounds__(256) void k_faces_batch(const BatchTabs<real> B, int k, const int *plan)
{
    __shared__ real wl[kGtabSize];
    __shared__ FaceXchg<real> xch[4];
    cptr<int> pl = (cptr<int>)plan;
    const int total = pl[B.nprob];
    int loaded = -1;  // problem whose weights wl holds
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int p = find_problem(pl, B.nprob, w);
        const StageArgs<real> &A = table_entry(B.args, p);
        const Cascade &C = table_entry(B.casc, p);
        if (p != loaded) {
            __syncthreads();  // the previous work block's readers of wl are done
            load_gtab<256>(A.gtab, wl);
            __syncthreads();
            loaded = p;
        }
        const int capf = (A.nx + 1) * A.ny + A.nx * (A.ny + 1);
        const int n = min(C.ctl->nface[k], capf);
        faces_phase<WALLS, HLL>(A, wl, xch[threadIdx.x >> 6], C.flist[k & 1], n, (w - pl[p]) * 256 + (int)threadIdx.x,
                                4 * n);
    }
}

template <typename real, bool WALLS>
__global__ __launch_bounds__(64) void k_cells_batch(const BatchTabs<real> B, int k, const int *plan)
{
    cptr<int> pl = (cptr<int>)(plan + B.nprob + 1);
    const int total = pl[B.nprob];
    for (int w = blockIdx.x; w < total; w += gridDim.x) {
        const int p = find_problem(pl, B.nprob, w);
        const StageArgs<real> &A = table_entry(B.args, p);
        const Cascade &C = table_entry(B.casc, p);
        const int n = min(C.ctl->ncell[k], A.nx * A.ny);
        cells_phase<WALLS>(A, C.clist[k & 1], n, (w - pl[p]) * 64 + (int)threadIdx.x, n,
                           pass_out(C, k, C.ctl->stamp0), (real)(*A.dt * A.dtf));
    }
}

// Problem p = blockIdx.x runs the rest of its cascade in one workgroup, from the
// pass the multi-block passes left to it (no hand-back).
template <typename real, bool WALLS, bool HLL>
__global__ __launch_bounds__((tail_threads<real, WALLS>())) void k_tail_batch(const BatchTabs<real> B)
{
    __shared__ TailShared<real> S;
    const int p = blockIdx.x;
    const StageArgs<real> &A = table_entry(B.args, p);
    const Cascade &C = table_entry(B.casc, p);
    tail_body<WALLS, HLL>(A, C, 1, kBatchPasses + 1, kMaxPasses, S);
}

// Stage start of every problem: counts of evaluation 0 and pass 1, tail state,
// and a fresh claim stamp range (kMaxPasses + 2 stamps per stage).
__global__ void k_reset_batch(const Cascade *casc, int nprob)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    Ctl *ctl = casc[p].ctl;
    // the counts the first pass and the multi-block passes add to
    for (int k = 0; k <= kBatchPasses + 1; ++k) {
        ctl->nface[k] = 0;
        ctl->ncell[k] = 0;
        ctl->ntroub[k] = 0;
    }
    ctl->tail_end = 0;
    ctl->tail_k0 = 0;
    ctl->tail_back = 0;
    ctl->nlow = 0;
    ctl->stamp0 += (unsigned)kMaxPasses + 2;
}

// The stamp range restarts after the stamp arrays were cleared.
__global__ void k_stamp_restart_batch(const Cascade *casc, int nprob)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) casc[p].ctl->stamp0 = 0u;
}

__global__ void k_dt_begin_batch(const Cascade *casc, int nprob)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) casc[p].ctl->lam_bits = 0ull;
}

// Blocks dblk[p] .. dblk[p+1]-1 reduce problem p's U^n (the stage-0 input).
template <typename real>
__global__ __launch_bounds__(256) void k_dt_reduce_batch(const BatchTabs<real> B)
{
    __shared__ double red[256];
    cptr<int> dblk = (cptr<int>)B.dblk;
    const int p = find_problem(dblk, B.nprob, blockIdx.x);
    const StageArgs<real> &A = table_entry(B.args, p);
    const Cascade &C = table_entry(B.casc, p);
    const int lb = blockIdx.x - dblk[p], nb = dblk[p + 1] - dblk[p];
    dt_reduce_body(A.Us, (size_t)A.nx * A.ny, A.gamma64, A.dx64, A.dy64, &C.ctl->lam_bits,
                   (size_t)lb * blockDim.x + threadIdx.x, (size_t)nb * blockDim.x, red);
}

__global__ void k_dt_end_batch(const Cascade *casc, int nprob, double cfl)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) {
        Ctl *ctl = casc[p].ctl;
        ctl->dt = cfl / __longlong_as_double((long long)ctl->lam_bits);
    }
}

// Per problem: evaluations of the last stage (0 if its cascade hit the pass
// limit) and dt.
__global__ void k_batch_status(const Cascade *casc, int nprob, int *iters, double *dts)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nprob) {
        const Ctl *ctl = casc[p].ctl;
        iters[p] = ctl->tail_end >= kMaxPasses ? 0 : ctl->tail_end;
        dts[p] = ctl->dt;
    }
}

// The cascade of a batch stage after its first pass: the claims of the lowered
// cells, kBatchPasses multi-block passes, then one workgroup per problem.
template <typename real, bool WALLS, bool HLL>
static hipError_t launch_batch_cascade(const BatchTabs<real> &B, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_plan<real>, dim3(1), dim3(1024), 0, st, B, 0, B.plan);
    hipLaunchKernelGGL(k_claims_first_batch<real>, dim3(kBatchFaceGrid), dim3(256), 0, st, B, (const int *)B.plan);
    for (int k = 1; k <= kBatchPasses; ++k) {
        hipLaunchKernelGGL(k_batch_plan<real>, dim3(1), dim3(1024), 0, st, B, k, B.plan);
        hipLaunchKernelGGL((k_faces_batch<real, WALLS, HLL>), dim3(kBatchFaceGrid), dim3(256), 0, st, B, k,
                           (const int *)B.plan);
        hipLaunchKernelGGL((k_cells_batch<real, WALLS>), dim3(kBatchCellGrid), dim3(64), 0, st, B, k,
                           (const int *)B.plan);
    }
    hipLaunchKernelGGL((k_tail_batch<real, WALLS, HLL>), dim3(B.nprob), dim3(tail_threads<real, WALLS>()), 0, st, B);
    return hipGetLastError();
}

// BW: the first-pass build with the boundary handling (some problem has walls).
template <typename real, bool BW>
static hipError_t launch_batch_stage_bw(const BatchTabs<real> &B, int top, int nfp_blocks, const Cascade *casc,
                                        hipStream_t st, bool tail = true)
{
    constexpr int WPB = sizeof(real) == 8 ? 2 : 4;
    const int nb = (B.nprob + 255) / 256;
    hipLaunchKernelGGL(k_reset_batch, dim3(nb), dim3(256), 0, st, casc, B.nprob);
    const dim3 g(nfp_blocks), t(64 * WPB);
    if (B.solver == 1) {
        switch (top * 2 + (B.iso ? 1 : 0)) {
        case 7: hipLaunchKernelGGL((k_first_pass_batch<real, 3, WPB, true, true, BW>), g, t, 0, st, B); break;
        case 6: hipLaunchKernelGGL((k_first_pass_batch<real, 3, WPB, false, true, BW>), g, t, 0, st, B); break;
        case 5: hipLaunchKernelGGL((k_first_pass_batch<real, 2, WPB, true, true, BW>), g, t, 0, st, B); break;
        case 4: hipLaunchKernelGGL((k_first_pass_batch<real, 2, WPB, false, true, BW>), g, t, 0, st, B); break;
        case 3: hipLaunchKernelGGL((k_first_pass_batch<real, 1, WPB, true, true, BW>), g, t, 0, st, B); break;
        case 2: hipLaunchKernelGGL((k_first_pass_batch<real, 1, WPB, false, true, BW>), g, t, 0, st, B); break;
        default: return hipErrorInvalidValue;
        }
        if (!tail) return hipGetLastError();
        return B.walls ? launch_batch_cascade<real, true, true>(B, st) : launch_batch_cascade<real, false, true>(B, st);
    }
    switch (top * 2 + (B.iso ? 1 : 0)) {
    case 7: hipLaunchKernelGGL((k_first_pass_batch<real, 3, WPB, true, false, BW>), g, t, 0, st, B); break;
    case 6: hipLaunchKernelGGL((k_first_pass_batch<real, 3, WPB, false, false, BW>), g, t, 0, st, B); break;
    case 5: hipLaunchKernelGGL((k_first_pass_batch<real, 2, WPB, true, false, BW>), g, t, 0, st, B); break;
    case 4: hipLaunchKernelGGL((k_first_pass_batch<real, 2, WPB, false, false, BW>), g, t, 0, st, B); break;
    case 3: hipLaunchKernelGGL((k_first_pass_batch<real, 1, WPB, true, false, BW>), g, t, 0, st, B); break;
    case 2: hipLaunchKernelGGL((k_first_pass_batch<real, 1, WPB, false, false, BW>), g, t, 0, st, B); break;
    default: return hipErrorInvalidValue;
    }
    if (!tail) return hipGetLastError();
    return B.walls ? launch_batch_cascade<real, true, false>(B, st) : launch_batch_cascade<real, false, false>(B, st);
}

template <typename real>
hipError_t launch_batch_stage(const BatchTabs<real> &B, int top, int nfp_blocks, const Cascade *casc,
                              hipStream_t st)
{
    return B.walls ? launch_batch_stage_bw<real, true>(B, top, nfp_blocks, casc, st)
                   : launch_batch_stage_bw<real, false>(B, top, nfp_blocks, casc, st);
}

// The reset and the first pass of a batch stage without its cascade (timing).
template <typename real>
hipError_t launch_batch_first_pass(const BatchTabs<real> &B, int top, int nfp_blocks, const Cascade *casc,
                                   hipStream_t st)
{
    return B.walls ? launch_batch_stage_bw<real, true>(B, top, nfp_blocks, casc, st, false)
                   : launch_batch_stage_bw<real, false>(B, top, nfp_blocks, casc, st, false);
}

template <typename real>
hipError_t launch_batch_dt(const BatchTabs<real> &B, int ndt_blocks, const Cascade *casc, double cfl, hipStream_t st)
{
    const int nb = (B.nprob + 255) / 256;
    hipLaunchKernelGGL(k_dt_begin_batch, dim3(nb), dim3(256), 0, st, casc, B.nprob);
    hipLaunchKernelGGL(k_dt_reduce_batch<real>, dim3(ndt_blocks), dim3(256), 0, st, B);
    hipLaunchKernelGGL(k_dt_end_batch, dim3(nb), dim3(256), 0, st, casc, B.nprob, cfl);
    return hipGetLastError();
}

hipError_t launch_batch_status(const Cascade *casc, int nprob, int *iters, double *dts, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_status, dim3((nprob + 255) / 256), dim3(256), 0, st, casc, nprob, iters, dts);
    return hipGetLastError();
}

hipError_t launch_batch_stamp_restart(const Cascade *casc, int nprob, hipStream_t st)
{
    hipLaunchKernelGGL(k_stamp_restart_batch, dim3((nprob + 255) / 256), dim3(256), 0, st, casc, nprob);
    return hipGetLastError();
}

template <typename real, int RT>
static hipError_t launch_first_pass_rt(const StageArgs<real> &A, const PassOut &P, hipStream_t st)
{
    constexpr int WPB = sizeof(real) == 8 ? 2 : 4;
    const int nstrip = (A.nx + 61) / 62, nseg = (A.ny + A.rows - 1) / A.rows;
    const int nwave = nstrip * nseg;
    const int nblk = (nwave + WPB - 1) / WPB;
    const dim3 g(nblk), t(64 * WPB);
    const int bnd = (A.bcx == 2 || A.bcy == 2 || A.slit != 0) ? 4 : 0;
    switch (bnd + (A.solver == 1 ? 2 : 0) + (A.iso ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, false, false, false>), g, t, 0, st, A, P); break;
    case 1: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, true, false, false>), g, t, 0, st, A, P); break;
    case 2: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, false, true, false>), g, t, 0, st, A, P); break;
    case 3: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, true, true, false>), g, t, 0, st, A, P); break;
    case 4: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, false, false, true>), g, t, 0, st, A, P); break;
    case 5: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, true, false, true>), g, t, 0, st, A, P); break;
    case 6: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, false, true, true>), g, t, 0, st, A, P); break;
    default: hipLaunchKernelGGL((k_first_pass<real, RT, WPB, true, true, true>), g, t, 0, st, A, P); break;
    }
    return hipGetLastError();
}

// First pass, then the claims of the cells it lowered (listed in C.clist[0],
// which pass 1 only writes after reading its own list C.clist[1]); `mid`, if
// given, is recorded between the two.
template <typename real>
static hipError_t launch_first_pass_and_claims(const StageArgs<real> &A, const PassOut &P, const Cascade &C,
                                               hipError_t (*fp)(const StageArgs<real> &, const PassOut &, hipStream_t),
                                               hipEvent_t mid, hipStream_t st)
{
    PassOut L = P;
    L.clist = C.clist[0];
    L.ccount = &C.ctl->nlow;
    hipError_t e = fp(A, L, st);
    if (e != hipSuccess) return e;
    if (mid) {
        e = hipEventRecord(mid, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_claims_first<real>, dim3(256), dim3(256), 0, st, A, P, C.clist[0], &C.ctl->nlow);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_first_pass(const StageArgs<real> &A, const PassOut &P, const Cascade &C, hipEvent_t mid,
                             hipStream_t st)
{
    switch (A.top) {
    case 3: return launch_first_pass_and_claims<real>(A, P, C, launch_first_pass_rt<real, 3>, mid, st);
    case 2: return launch_first_pass_and_claims<real>(A, P, C, launch_first_pass_rt<real, 2>, mid, st);
    case 1: return launch_first_pass_and_claims<real>(A, P, C, launch_first_pass_rt<real, 1>, mid, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_cascade_pass(const StageArgs<real> &A, const Cascade &C, int k, int nblocks, hipStream_t st)
{
    const bool walls = A.bcx == 2 || A.bcy == 2 || A.slit != 0;
    if (walls && A.solver == 1)
        hipLaunchKernelGGL((k_faces<real, true, true>), dim3(nblocks), dim3(256), 0, st, A, C, k);
    else if (walls)
        hipLaunchKernelGGL((k_faces<real, true, false>), dim3(nblocks), dim3(256), 0, st, A, C, k);
    else if (A.solver == 1)
        hipLaunchKernelGGL((k_faces<real, false, true>), dim3(nblocks), dim3(256), 0, st, A, C, k);
    else
        hipLaunchKernelGGL((k_faces<real, false, false>), dim3(nblocks), dim3(256), 0, st, A, C, k);
    if (walls)
        hipLaunchKernelGGL((k_cells<real, true>), dim3(nblocks), dim3(64), 0, st, A, C, k);
    else
        hipLaunchKernelGGL((k_cells<real, false>), dim3(nblocks), dim3(64), 0, st, A, C, k);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_cascade_tail(const StageArgs<real> &A, const Cascade &C, int kbeg, int kdef, int kend,
                               hipStream_t st)
{
    const bool walls = A.bcx == 2 || A.bcy == 2 || A.slit != 0;
    if (walls && A.solver == 1)
        hipLaunchKernelGGL((k_tail<real, true, true>), dim3(1), dim3(tail_threads<real, true>()), 0, st, A, C, kbeg, kdef, kend);
    else if (walls)
        hipLaunchKernelGGL((k_tail<real, true, false>), dim3(1), dim3(tail_threads<real, true>()), 0, st, A, C, kbeg, kdef, kend);
    else if (A.solver == 1)
        hipLaunchKernelGGL((k_tail<real, false, true>), dim3(1), dim3(tail_threads<real, false>()), 0, st, A, C, kbeg, kdef, kend);
    else
        hipLaunchKernelGGL((k_tail<real, false, false>), dim3(1), dim3(tail_threads<real, false>()), 0, st, A, C, kbeg, kdef, kend);
    return hipGetLastError();
}

hipError_t launch_reset(Ctl *ctl, int nzero, unsigned stamp0, hipStream_t st)
{
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, st, ctl, nzero, stamp0);
    return hipGetLastError();
}

hipError_t launch_level_hist(const uint8_t *order, size_t ncell, const LevIdx &levidx, Ctl *ctl, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_levcnt, dim3(1), dim3(64), 0, st, ctl);
    size_t nblk = (ncell + 255) / 256;
    if (nblk > 1024) nblk = 1024;
    hipLaunchKernelGGL(k_level_hist, dim3((unsigned)nblk), dim3(256), 0, st, order, ncell, levidx, ctl->levcnt);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_lincomb4(real *out, const real *x0, const real *x1, const real *x2, const real *x3, double w0,
                           double w1, double w2, double w3, size_t n, hipStream_t st)
{
    size_t nb = (n + 255) / 256;
    if (nb > 8192) nb = 8192;
    hipLaunchKernelGGL(k_lincomb4<real>, dim3((unsigned)nb), dim3(256), 0, st, out, x0, x1, x2, x3, (real)w0,
                       (real)w1, (real)w2, (real)w3, n);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_dt(const real *U, size_t ncell, double gamma, double dx, double dy, double cfl, double lam0, Ctl *ctl,
                     hipStream_t st)
{
    hipLaunchKernelGGL(k_dt_set, dim3(1), dim3(1), 0, st, ctl, 0.0, 1);
    size_t nblk = (ncell + 255) / 256;
    if (nblk > 4096) nblk = 4096;
    hipLaunchKernelGGL(k_dt_reduce<real>, dim3((unsigned)nblk), dim3(256), 0, st, U, ncell, gamma, dx, dy,
                       &ctl->lam_bits);
    hipLaunchKernelGGL(k_dt_finalize, dim3(1), dim3(1), 0, st, ctl, cfl, lam0);
    return hipGetLastError();
}

hipError_t launch_stats(Ctl *ctl, int npass, int reset, hipStream_t st)
{
    hipLaunchKernelGGL(k_stats_accum, dim3(1), dim3(256), 0, st, ctl, npass, reset);
    return hipGetLastError();
}

hipError_t launch_set_dt(Ctl *ctl, double dt, hipStream_t st)
{
    hipLaunchKernelGGL(k_dt_set, dim3(1), dim3(1), 0, st, ctl, dt, 0);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_totals(const real *U, size_t ncell, double area, double *partial, int nblk, double *out,
                         hipStream_t st)
{
    hipLaunchKernelGGL(k_totals_partial<real>, dim3(nblk, 4), dim3(256), 0, st, U, ncell, partial);
    hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(64), 0, st, partial, nblk, area, out);
    return hipGetLastError();
}

template hipError_t launch_first_pass<float>(const StageArgs<float> &, const PassOut &, const Cascade &, hipEvent_t,
                                             hipStream_t);
template hipError_t launch_first_pass<double>(const StageArgs<double> &, const PassOut &, const Cascade &,
                                              hipEvent_t, hipStream_t);
template hipError_t launch_cascade_pass<float>(const StageArgs<float> &, const Cascade &, int, int, hipStream_t);
template hipError_t launch_cascade_pass<double>(const StageArgs<double> &, const Cascade &, int, int, hipStream_t);
template hipError_t launch_cascade_tail<float>(const StageArgs<float> &, const Cascade &, int, int, int, hipStream_t);
template hipError_t launch_cascade_tail<double>(const StageArgs<double> &, const Cascade &, int, int, int,
                                                hipStream_t);
template hipError_t launch_lincomb4<float>(float *, const float *, const float *, const float *, const float *,
                                           double, double, double, double, size_t, hipStream_t);
template hipError_t launch_lincomb4<double>(double *, const double *, const double *, const double *,
                                            const double *, double, double, double, double, size_t, hipStream_t);
template hipError_t launch_dt<float>(const float *, size_t, double, double, double, double, double, Ctl *, hipStream_t);
template hipError_t launch_dt<double>(const double *, size_t, double, double, double, double, double, Ctl *, hipStream_t);
template hipError_t launch_totals<float>(const float *, size_t, double, double *, int, double *, hipStream_t);
template hipError_t launch_totals<double>(const double *, size_t, double, double *, int, double *, hipStream_t);

template hipError_t launch_batch_stage<float>(const BatchTabs<float> &, int, int, const Cascade *, hipStream_t);
template hipError_t launch_batch_first_pass<float>(const BatchTabs<float> &, int, int, const Cascade *, hipStream_t);
template hipError_t launch_batch_first_pass<double>(const BatchTabs<double> &, int, int, const Cascade *, hipStream_t);
template hipError_t launch_batch_stage<double>(const BatchTabs<double> &, int, int, const Cascade *, hipStream_t);
template hipError_t launch_batch_dt<float>(const BatchTabs<float> &, int, const Cascade *, double, hipStream_t);
template hipError_t launch_batch_dt<double>(const BatchTabs<double> &, int, const Cascade *, double, hipStream_t);

}  // namespace gpm
