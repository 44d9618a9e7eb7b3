// Internal: the context of the C ABI and the helpers shared by the single-problem
// and batched entry points (not installed; see include/gpmood.h for the API).
#ifndef GPMOOD_CTX_H
#define GPMOOD_CTX_H

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "gpmood.h"
#include "gpmood_device.h"
#include "gpmood_launch.h"

using namespace gpm;

namespace {

constexpr size_t kAlign = 256;
constexpr int kTotBlocks = 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

}  // namespace

struct gpm_ctx {
    gpm_grid grid;
    int prec;
    hipStream_t stream;
    int nx, ny;
    size_t ncell;
    double dx, dy;
    bool have_scheme = false;
    gpm_scheme scheme;
    Weights<double> w64;
    Weights<float> w32;
    std::vector<double> gtab64;  // compact cascade weights (kGtabSize), both precisions
    std::vector<float> gtab32;
    int top = 0;
    int next[4] = {0, 0, 0, 0};
    int levidx[4] = {0, 0, 0, 0};
    // bound memory
    char *state = nullptr;
    char *work = nullptr;
    int cur = 0;
    uint8_t *order = nullptr;
    unsigned *cstamp = nullptr;
    unsigned *fstamp = nullptr;
    int *flist[2] = {nullptr, nullptr};
    int *clist[2] = {nullptr, nullptr};
    void *FX = nullptr;
    void *GY = nullptr;
    uint8_t *FXf = nullptr;
    uint8_t *GYf = nullptr;
    Ctl *ctl = nullptr;
    double *partial = nullptr;
    void *gtab = nullptr;
    unsigned pass = 0;
    int passes_per_check = 4;  // smallest batch of multi-block cascade passes
    int head_guess = 4;        // batch length: the previous stage's multi-block passes + 2
    int tail_threshold = 32;   // troubled cells at or below which one workgroup finishes the cascade
    int rows = 12;
    int si0 = 0, si1 = 0;  // inflow slit cells [si0, si1)
    double slit_u[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};  // bottom, top
    double slit_lam = 0.0;  // the slit state's CFL bound (0: none)
    int last_npass = 0;
    bool fresh_ctl = true;
    int *pinned = nullptr;
    // instrumentation
    int instrument = 0;           // bit 0: stage events and iteration counts, bit 1: level statistics
    long long acc_iters = 0, acc_stages = 0;
    long long cstat[3] = {0, 0, 0};  // last stage: multi-block passes, tail passes, hand-backs
    // adjoint workspace (gpm_bind_adjoint): per-face records, then the FP64
    // derivative of the compact weight table with respect to ell
    char *adj = nullptr;
    std::vector<hipEvent_t> evs;  // 3 per instrumented stage: first pass start/end, stage end
    size_t nev_used = 0;
    std::string err;
};

static inline gpm_status fail(gpm_ctx *c, gpm_status st, const std::string &msg)
{
    if (c) c->err = msg;
    return st;
}

// Adjoint workspace: the per-face records, [2][4][ny+1][nx+1][16] values of the
// state precision, then kGtabSize doubles (the ell table), then one double per
// kAdjTile x kAdjTile tile of cells (its dL/d(ell) partial); 256-byte aligned parts.
static inline size_t adj_face_bytes(const gpm_ctx *c)
{
    const size_t esz = c->prec == GPM_F64 ? 8 : 4;
    return align_up((size_t)2 * 64 * (size_t)(c->nx + 1) * (size_t)(c->ny + 1) * esz);
}
static inline size_t adj_tiles(const gpm_ctx *c)
{
    return (size_t)((c->nx + kAdjTile - 1) / kAdjTile) * (size_t)((c->ny + kAdjTile - 1) / kAdjTile);
}
static inline size_t adj_partial_offset(const gpm_ctx *c) { return adj_face_bytes(c) + align_up((size_t)kGtabSize * 8); }
static inline size_t adj_bytes(const gpm_ctx *c) { return adj_partial_offset(c) + align_up(adj_tiles(c) * 8); }

// Copy the FP64 ell-derivative of the compact weights into the adjoint workspace.
static inline gpm_status upload_adj_dl(gpm_ctx *c)
{
    if (!c->adj || !c->have_scheme) return GPM_OK;
    hipError_t e = hipMemcpyAsync(c->adj + adj_face_bytes(c), c->gtab64.data() + kGtabSize,
                                  (size_t)kGtabSize * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("adjoint table upload: ") + hipGetErrorString(e));
    return GPM_OK;
}

// Copy the compact cascade weights into the workspace (synchronous: a setup step).
static inline gpm_status upload_gtab(gpm_ctx *c)
{
    if (!c->gtab || !c->have_scheme) return GPM_OK;
    const void *src = c->prec == GPM_F64 ? (const void *)c->gtab64.data() : (const void *)c->gtab32.data();
    const size_t bytes = (size_t)2 * kGtabSize * (c->prec == GPM_F64 ? 8 : 4);
    hipError_t e = hipMemcpyAsync(c->gtab, src, bytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("weight upload: ") + hipGetErrorString(e));
    return GPM_OK;
}

#define HIPCHK(c, expr)                                                                      \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail((c), GPM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));   \
    } while (0)

static inline size_t state_slot_bytes(const gpm_ctx *c)
{
    return align_up(4 * c->ncell * (c->prec == GPM_F64 ? 8 : 4));
}

static inline size_t nfaces_x(const gpm_ctx *c) { return (size_t)(c->nx + 1) * c->ny; }
static inline size_t nfaces_y(const gpm_ctx *c) { return (size_t)c->nx * (c->ny + 1); }

// Workspace partition (each part 256-byte aligned).
enum { W_ORDER, W_CSTAMP, W_FSTAMP, W_FL0, W_FL1, W_CL0, W_CL1, W_FX, W_GY, W_FXF, W_GYF, W_CTL, W_PART, W_GTAB, W_N };

static inline size_t work_layout(const gpm_ctx *c, size_t off[W_N])
{
    const size_t nf = nfaces_x(c) + nfaces_y(c);
    const size_t esz = c->prec == GPM_F64 ? 8 : 4;
    const size_t sz[W_N] = {c->ncell, 4 * c->ncell, 4 * nf, 4 * nf, 4 * nf, 4 * c->ncell, 4 * c->ncell,
                            4 * esz * nfaces_x(c), 4 * esz * nfaces_y(c), nfaces_x(c), nfaces_y(c), sizeof(Ctl),
                            (size_t)kTotBlocks * 4 * 2 * sizeof(double), (size_t)2 * kGtabSize * esz};
    size_t o = 0;
    for (int k = 0; k < W_N; ++k) {
        off[k] = o;
        o = align_up(o + sz[k]);
    }
    return o;
}

static inline void *slot_ptr(gpm_ctx *c, int slot) { return c->state + slot * state_slot_bytes(c); }

// Are the y-face weights of radius <= top bit for bit the x-face weights of the
// transposed parity entries (equal spacing and length scale in x and y)?  The
// first pass then reads one table for both directions, with identical products.
template <typename real>
static inline int weights_isotropic(const Weights<real> &W, int top)
{
    for (int R = 1; R <= top; ++R)
        for (int p = 0; p < slots_of(R); ++p)
            for (int e = 0; e < kNQ[R]; ++e) {
                // the centre node of R = 2 does not use its odd-along-the-face entries
                if (slot_is_zero(R, p) && (kQ[e].comp == C_OE || kQ[e].comp == C_OO)) continue;
                const int t = transposed_entry(e);
                const real wy = R == 3 ? W.w3[1][p][e] : (R == 2 ? W.w2[1][p][e] : W.w1[1][p][e]);
                const real wx = R == 3 ? W.w3[0][p][t] : (R == 2 ? W.w2[0][p][t] : W.w1[0][p][t]);
                if (std::memcmp(&wx, &wy, sizeof(real)) != 0) return 0;
            }
    return 1;
}

template <typename real>
static inline void fill_args(const gpm_ctx *c, const Weights<real> &W, StageArgs<real> &A)
{
    A.nx = c->nx;
    A.ny = c->ny;
    A.bcx = c->grid.bc[0];
    A.bcy = c->grid.bc[1];
    A.rows = c->rows;
    A.top = c->top;
    A.dtf = 1.0;
    A.ca = real(0);
    A.cb = real(1);
    A.iso = weights_isotropic(W, c->top);
    A.solver = c->scheme.solver;
    A.slit = c->grid.slit;
    A.si0 = c->si0;
    A.si1 = c->si1;
    for (int v = 0; v < 4; ++v) {
        A.slitU[0][v] = (real)c->slit_u[0][v];
        A.slitU[1][v] = (real)c->slit_u[1][v];
    }
    A.flags = c->scheme.flags;
    A.dx = (real)c->dx;
    A.dy = (real)c->dy;
    A.gamma = (real)c->grid.gamma;
    A.dx64 = c->dx;
    A.dy64 = c->dy;
    A.gamma64 = c->grid.gamma;
    A.sigma_v = (real)c->scheme.sigma_v;
    A.sigma_p = (real)c->scheme.sigma_p;
    const double d3 = c->dx * c->dx * c->dx < c->dy * c->dy * c->dy ? c->dx * c->dx * c->dx : c->dy * c->dy * c->dy;
    A.plat_thr = (real)d3;
    A.delta = (real)(c->dx < c->dy ? c->dx : c->dy);
    A.W = W;
    A.dt = &c->ctl->dt;
    A.stamp0 = &c->ctl->stamp0;
    A.order = c->order;
    A.FX = (real *)c->FX;
    A.GY = (real *)c->GY;
    A.FXf = c->FXf;
    A.GYf = c->GYf;
    A.gtab = (const real *)c->gtab;
    A.gtab_dl = (const real *)c->gtab + kGtabSize;
    A.cstamp = c->cstamp;
    A.fstamp = c->fstamp;
    for (int r = 0; r < 4; ++r) A.next[r] = c->next[r];
}

// Claim stamps grow monotonically (kMaxPasses + 2 per stage); the stamp arrays
// are cleared at the start of a stage when fewer than a stage's worth is left
// before the wrap.
static inline gpm_status stamps_for_stage(gpm_ctx *c)
{
    if (c->pass >= 0xffffffffu - (unsigned)(2 * kMaxPasses + 8)) {
        HIPCHK(c, hipMemsetAsync(c->cstamp, 0, 4 * c->ncell, c->stream));
        HIPCHK(c, hipMemsetAsync(c->fstamp, 0, 4 * (nfaces_x(c) + nfaces_y(c)), c->stream));
        c->pass = 0;
    }
    return GPM_OK;
}

static inline gpm_status level_counts(gpm_ctx *c)
{
    LevIdx li;
    for (int r = 0; r < 4; ++r) li.v[r] = c->levidx[r];
    hipError_t e = launch_level_hist(c->order, c->ncell, li, c->ctl, c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("level histogram: ") + hipGetErrorString(e));
    return GPM_OK;
}

#endif
