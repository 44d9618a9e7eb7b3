// C ABI of the GP-MOOD stage engine: context, scheme setup, binding of caller
// memory, and the host control of the MOOD loop (see include/gpmood.h).
#include "gpmood.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "gp_weights.h"
#include "gpmood_device.h"
#include "gpmood_launch.h"

using namespace gpm;

#include "gpmood_ctx.h"

extern "C" {

const char *gpm_strerror(gpm_status st)
{
    switch (st) {
    case GPM_OK: return "ok";
    case GPM_EINVAL: return "invalid argument";
    case GPM_ENOMEM: return "out of host memory";
    case GPM_EHIP: return "HIP runtime error";
    case GPM_ESTATE: return "call out of order (scheme or buffers missing)";
    case GPM_ENOTCONV: return "MOOD loop exceeded its pass limit";
    case GPM_EUNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char *gpm_last_error(const gpm_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

gpm_status gpm_create(const gpm_grid *grid, int prec, void *hip_stream, gpm_ctx **out)
{
    if (!grid || !out) return GPM_EINVAL;
    *out = nullptr;
    if (grid->dim != 2) return GPM_EUNSUPPORTED;
    if (prec != GPM_F32 && prec != GPM_F64) return GPM_EINVAL;
    for (int d = 0; d < 2; ++d) {
        if (grid->n[d] < 1 || grid->n[d] > 32768) return GPM_EINVAL;
        if (!(grid->hi[d] > grid->lo[d])) return GPM_EINVAL;
        if (grid->bc[d] != GPM_BC_PERIODIC && grid->bc[d] != GPM_BC_OUTFLOW && grid->bc[d] != GPM_BC_REFLECT)
            return GPM_EINVAL;
        // the widest stencil reaches 4 cells past an edge; a periodic or reflecting
        // axis must hold its image
        if (grid->bc[d] != GPM_BC_OUTFLOW && grid->n[d] < 4) return GPM_EUNSUPPORTED;
    }
    if (!(grid->gamma > 1.0)) return GPM_EINVAL;
    int si0 = 0, si1 = 0;
    if (grid->slit != 0) {
        if (grid->slit < 0 || grid->slit > 3 || grid->bc[1] != GPM_BC_OUTFLOW || !(grid->slit_x[1] > grid->slit_x[0]) ||
            ((grid->slit & 1) && !(grid->slit_prim[0] > 0.0 && grid->slit_prim[3] > 0.0)) ||
            ((grid->slit & 2) && !(grid->slit_prim_top[0] > 0.0 && grid->slit_prim_top[3] > 0.0)))
            return GPM_EINVAL;
        const double dx = (grid->hi[0] - grid->lo[0]) / grid->n[0];
        si0 = grid->n[0];
        for (int i = 0; i < grid->n[0]; ++i) {
            const double xc = grid->lo[0] + (i + 0.5) * dx;
            if (xc >= grid->slit_x[0] && xc <= grid->slit_x[1]) {
                si0 = i < si0 ? i : si0;
                si1 = i + 1;
            }
        }
        if (si1 <= si0) return GPM_EINVAL;  // no cell centre in the slit
    }
    gpm_ctx *c = new (std::nothrow) gpm_ctx;
    if (!c) return GPM_ENOMEM;
    c->grid = *grid;
    c->prec = prec;
    c->stream = (hipStream_t)hip_stream;
    c->nx = grid->n[0];
    c->ny = grid->n[1];
    c->ncell = (size_t)c->nx * c->ny;
    // first-pass march length: 12 rows; 24 in FP64 (one wavefront per SIMD) when
    // the grid still gives at least two marches for each of the 1024 SIMDs, where
    // the shorter halo re-read pays (2048^2 FP64: 0.846 -> 0.817 ms per launch)
    const long long strips = (c->nx + 61) / 62;
    c->rows = (prec == GPM_F64 && strips * ((c->ny + 23) / 24) >= 2048) ? 24 : 12;
    c->dx = (grid->hi[0] - grid->lo[0]) / c->nx;
    c->dy = (grid->hi[1] - grid->lo[1]) / c->ny;
    c->si0 = si0;
    c->si1 = si1;
    for (int side = 0; side < 2; ++side) {
        if (!(grid->slit & (1 << side))) continue;
        const double *pr = side ? grid->slit_prim_top : grid->slit_prim;
        const double r = pr[0], u = pr[1], v = pr[2], p = pr[3];
        const double g = grid->gamma;
        double *q = c->slit_u[side];
        q[0] = r;
        q[1] = r * u;
        q[2] = r * v;
        q[3] = p / (g - 1.0) + 0.5 * r * (u * u + v * v);
        // its waves bound the CFL step, in the form of the cells' bound
        const double pp = (g - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / r);
        const double cs = std::sqrt(g * pp / r);
        const double lx = (std::fabs(q[1] / r) + cs) / c->dx, ly = (std::fabs(q[2] / r) + cs) / c->dy;
        const double lam = lx > ly ? lx : ly;
        c->slit_lam = lam > c->slit_lam ? lam : c->slit_lam;
    }
    if (hipHostMalloc((void **)&c->pinned, 64, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return GPM_EHIP;
    }
    *out = c;
    return GPM_OK;
}

void gpm_destroy(gpm_ctx *c)
{
    if (!c) return;
    if (c->pinned) (void)hipHostFree(c->pinned);
    for (hipEvent_t e : c->evs) (void)hipEventDestroy(e);
    delete c;
}

gpm_status gpm_set_scheme(gpm_ctx *c, const gpm_scheme *s)
{
    if (!c || !s) return GPM_EINVAL;
    if (s->nlev < 1 || s->nlev > 4) return fail(c, GPM_EINVAL, "nlev must be 1..4");
    for (int l = 0; l < s->nlev; ++l) {
        if (s->radius[l] < 0 || s->radius[l] > 3) return fail(c, GPM_EINVAL, "radius must be 0..3");
        if (l > 0 && !(s->radius[l] < s->radius[l - 1])) return fail(c, GPM_EINVAL, "cascade must strictly decrease");
    }
    if (s->radius[s->nlev - 1] != 0) return fail(c, GPM_EINVAL, "cascade must end at radius 0 (FOG)");
    if (s->radius[0] == 0) return fail(c, GPM_EINVAL, "top scheme must have radius >= 1");
    if (!(s->ell >= 0.0)) return fail(c, GPM_EINVAL, "ell must be >= 0");
    if (s->stencil < GPM_STENCIL_DIAMOND || s->stencil > GPM_STENCIL_POLY3)
        return fail(c, GPM_EINVAL, "unknown stencil");
    if (s->solver != GPM_SOLVER_HLLC && s->solver != GPM_SOLVER_HLL) return fail(c, GPM_EINVAL, "unknown solver");
    if (s->stencil == GPM_STENCIL_POLY3 && s->radius[0] != 1)
        return fail(c, GPM_EINVAL, "POL-MOOD3 has radius 1 (cascade {1, 0})");
    const double ell = s->ell > 0.0 ? s->ell : 12.0 * (c->dx < c->dy ? c->dx : c->dy);
    const double ax = ell / c->dx, ay = ell / c->dy;
    std::memset(&c->w64, 0, sizeof(c->w64));
    std::memset(&c->w32, 0, sizeof(c->w32));
    // the compact table, then its derivative with respect to ell (same layout)
    std::vector<double> g64(2 * kGtabSize, 0.0);
    std::vector<float> g32(2 * kGtabSize, 0.0f);
    // FOG: the cell value itself (gathered 4x at the centre), one node of weight 1
    for (int d = 0; d < 2; ++d) {
        g64[(0 * 2 + d) * kGtabPerDir + C_EE] = 0.25;
        g32[(0 * 2 + d) * kGtabPerDir + C_EE] = 0.25f;
    }
    g64[kGtabNodeOff + 0] = 1.0;
    g32[kGtabNodeOff + 0] = 1.0f;
    for (int R = 1; R <= 3; ++R) {
        bool used = false;
        for (int l = 0; l < s->nlev; ++l) used = used || s->radius[l] == R;
        if (!used) continue;
        GpwLevel L;
        const int shape = s->stencil == GPM_STENCIL_CROSS ? GPW_CROSS : (s->stencil == GPM_STENCIL_POLY3 ? GPW_POLY3 : GPW_DIAMOND);
        if (gpw_level(R, ax, ay, shape, &L) != 0) return fail(c, GPM_EINVAL, "GP covariance matrix not positive definite");
        for (int d = 0; d < 2; ++d)
            for (int p = 0; p < slots_of(R); ++p)
                for (int e = 0; e < kNQ[R]; ++e) {
                    if (R == 3) { c->w64.w3[d][p][e] = L.w64[d][p][e]; c->w32.w3[d][p][e] = L.w32[d][p][e]; }
                    if (R == 2) { c->w64.w2[d][p][e] = L.w64[d][p][e]; c->w32.w2[d][p][e] = L.w32[d][p][e]; }
                    if (R == 1) { c->w64.w1[d][0][e] = L.w64[d][0][e]; c->w32.w1[d][0][e] = L.w32[d][0][e]; }
                }
        for (int d = 0; d < 2; ++d)
            for (int p = 0; p < slots_of(R); ++p)
                for (int e = 0; e < kNQ[R]; ++e) {
                    const int a = kQ[e].a, b = kQ[e].b;
                    int pos = 0;
                    while (!((int)((kPosA >> (4 * pos)) & 15u) == a && (int)((kPosB >> (4 * pos)) & 15u) == b)) ++pos;
                    const double f = (a == 0 && b == 0) ? 0.25 : ((a == 0 || b == 0) ? 0.5 : 1.0);
                    const int k = (R * 2 + d) * kGtabPerDir + p * (kNPos * 4) + pos * 4 + kQ[e].comp;
                    g64[k] = L.w64[d][p][e] * f;
                    g32[k] = L.w32[d][p][e] * (float)f;
                    g64[kGtabSize + k] = L.dlw64[d][p][e] * f / ell;
                    g32[kGtabSize + k] = (float)(L.dlw64[d][p][e] * f / ell);
                }
        for (int p = 0; p < slots_of(R); ++p) {
            g64[kGtabNodeOff + R * 2 + p] = L.qw64[p];
            g32[kGtabNodeOff + R * 2 + p] = L.qw32[p];
        }
        for (int p = 0; p < slots_of(R); ++p) {
            if (R == 3) { c->w64.qw3[p] = L.qw64[p]; c->w32.qw3[p] = L.qw32[p]; }
            if (R == 2) { c->w64.qw2[p] = L.qw64[p]; c->w32.qw2[p] = L.qw32[p]; }
            if (R == 1) { c->w64.qw1 = L.qw64[0]; c->w32.qw1 = L.qw32[0]; }
        }
    }
    GpwCurv K;
    if (gpw_curvature(ax, ay, ell, &K) != 0) return fail(c, GPM_EINVAL, "GP-R1 covariance matrix not positive definite");
    for (int d = 0; d < 2; ++d)
        for (int k = 0; k < 3; ++k) {
            c->w64.curv[d][k] = K.w64[d][k];
            c->w32.curv[d][k] = K.w32[d][k];
        }
    c->gtab64.swap(g64);
    c->gtab32.swap(g32);
    c->scheme = *s;
    c->scheme.ell = ell;
    c->top = s->radius[0];
    for (int r = 0; r < 4; ++r) { c->next[r] = 0; c->levidx[r] = 0; }
    for (int l = 0; l < s->nlev; ++l) {
        c->levidx[s->radius[l]] = l;
        c->next[s->radius[l]] = l + 1 < s->nlev ? s->radius[l + 1] : 0;
    }
    c->have_scheme = true;
    const gpm_status st = upload_gtab(c);
    return st != GPM_OK ? st : upload_adj_dl(c);
}

gpm_status gpm_workspace_size(const gpm_ctx *c, size_t *state_bytes, size_t *work_bytes)
{
    if (!c) return GPM_EINVAL;
    size_t off[W_N];
    if (state_bytes) *state_bytes = 3 * state_slot_bytes(c);
    if (work_bytes) *work_bytes = work_layout(c, off);
    return GPM_OK;
}

gpm_status gpm_bind(gpm_ctx *c, void *state, void *work)
{
    if (!c || !state || !work) return GPM_EINVAL;
    if (((uintptr_t)state % kAlign) || ((uintptr_t)work % kAlign)) return fail(c, GPM_EINVAL, "buffers must be 256-byte aligned");
    size_t off[W_N];
    const size_t wbytes = work_layout(c, off);
    c->state = (char *)state;
    c->work = (char *)work;
    c->order = (uint8_t *)(c->work + off[W_ORDER]);
    c->cstamp = (unsigned *)(c->work + off[W_CSTAMP]);
    c->fstamp = (unsigned *)(c->work + off[W_FSTAMP]);
    c->flist[0] = (int *)(c->work + off[W_FL0]);
    c->flist[1] = (int *)(c->work + off[W_FL1]);
    c->clist[0] = (int *)(c->work + off[W_CL0]);
    c->clist[1] = (int *)(c->work + off[W_CL1]);
    c->FX = c->work + off[W_FX];
    c->GY = c->work + off[W_GY];
    c->FXf = (uint8_t *)(c->work + off[W_FXF]);
    c->GYf = (uint8_t *)(c->work + off[W_GYF]);
    c->ctl = (Ctl *)(c->work + off[W_CTL]);
    c->partial = (double *)(c->work + off[W_PART]);
    c->gtab = c->work + off[W_GTAB];
    c->cur = 0;
    c->pass = 0;
    c->fresh_ctl = true;
    HIPCHK(c, hipMemsetAsync(c->work, 0, wbytes, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return upload_gtab(c);
}

gpm_status gpm_state_ptr(const gpm_ctx *c, int slot, void **ptr, int *current_slot)
{
    if (!c || slot < 0 || slot > 2) return GPM_EINVAL;
    if (!c->state) return GPM_ESTATE;
    if (ptr) *ptr = c->state + slot * state_slot_bytes(c);
    if (current_slot) *current_slot = c->cur;
    return GPM_OK;
}


gpm_status gpm_init_state(gpm_ctx *c, const double *U)
{
    if (!c || !U) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    const size_t n = 4 * c->ncell;
    if (c->prec == GPM_F64) {
        HIPCHK(c, hipMemcpyAsync(slot_ptr(c, c->cur), U, n * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(n);
        for (size_t k = 0; k < n; ++k) tmp[k] = (float)U[k];
        HIPCHK(c, hipMemcpyAsync(slot_ptr(c, c->cur), tmp.data(), n * 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return GPM_OK;
}

gpm_status gpm_get_state(gpm_ctx *c, double *U)
{
    if (!c || !U) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    const size_t n = 4 * c->ncell;
    if (c->prec == GPM_F64) {
        HIPCHK(c, hipMemcpyAsync(U, slot_ptr(c, c->cur), n * 8, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<float> tmp(n);
        HIPCHK(c, hipMemcpyAsync(tmp.data(), slot_ptr(c, c->cur), n * 4, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (size_t k = 0; k < n; ++k) U[k] = tmp[k];
    }
    return GPM_OK;
}

static gpm_status compute_dt_from(gpm_ctx *c, const void *U, double cfl)
{
    hipError_t e = c->prec == GPM_F64
                       ? launch_dt<double>((const double *)U, c->ncell, c->grid.gamma, c->dx, c->dy, cfl, c->slit_lam,
                                           c->ctl, c->stream)
                       : launch_dt<float>((const float *)U, c->ncell, c->grid.gamma, c->dx, c->dy, cfl, c->slit_lam,
                                          c->ctl, c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("dt kernels: ") + hipGetErrorString(e));
    return GPM_OK;
}

gpm_status gpm_compute_dt(gpm_ctx *c, double cfl, double *dt_host)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    if (!(cfl > 0.0)) return fail(c, GPM_EINVAL, "cfl must be > 0");
    gpm_status st = compute_dt_from(c, slot_ptr(c, c->cur), cfl);
    if (st != GPM_OK) return st;
    if (dt_host) {
        HIPCHK(c, hipMemcpyAsync(dt_host, &c->ctl->dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return GPM_OK;
}

gpm_status gpm_compute_dt_dev(gpm_ctx *c, const void *U, double cfl, double *dt_host)
{
    if (!c || !U) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    if (!(cfl > 0.0)) return fail(c, GPM_EINVAL, "cfl must be > 0");
    gpm_status st = compute_dt_from(c, U, cfl);
    if (st != GPM_OK) return st;
    if (dt_host) {
        HIPCHK(c, hipMemcpyAsync(dt_host, &c->ctl->dt, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return GPM_OK;
}

gpm_status gpm_set_dt(gpm_ctx *c, double dt)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    hipError_t e = launch_set_dt(c->ctl, dt, c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, hipGetErrorString(e));
    return GPM_OK;
}

gpm_status gpm_set_tuning(gpm_ctx *c, int passes_per_check, int rows_per_wave, int tail_threshold)
{
    if (!c || passes_per_check < 1 || passes_per_check > 128 || rows_per_wave < 4 || rows_per_wave > 256 ||
        tail_threshold < 0 || tail_threshold > 4096)
        return GPM_EINVAL;
    c->passes_per_check = passes_per_check;
    c->head_guess = passes_per_check;
    c->rows = rows_per_wave;
    c->tail_threshold = tail_threshold;
    return GPM_OK;
}

}  // extern "C"

template <typename real>
static gpm_status run_stage(gpm_ctx *c, const Weights<real> &W, int s, const void *Un, const void *Us, void *Uout,
                           double ca = 0.0, double cb = 1.0, double dtf = 1.0)
{
    StageArgs<real> A;
    fill_args(c, W, A);
    A.s = s;
    if (s == 3) {
        A.ca = (real)ca;
        A.cb = (real)cb;
        A.dtf = dtf;
    }
    A.Un = (const real *)Un;
    A.Us = (const real *)Us;
    A.Uout = (real *)Uout;
    // evaluation 0 (first pass) claims the faces and cells of cascade pass 1;
    // pass k claims with stamp0 + k
    gpm_status st = stamps_for_stage(c);
    if (st != GPM_OK) return st;
    const unsigned stamp0 = c->pass + 1;
    c->pass += (unsigned)kMaxPasses + 2;
    const int nzero = c->fresh_ctl ? kMaxPasses + 2 : (c->last_npass + 3 < kMaxPasses + 2 ? c->last_npass + 3 : kMaxPasses + 2);
    hipError_t e = launch_reset(c->ctl, nzero, stamp0, c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("reset: ") + hipGetErrorString(e));
    c->fresh_ctl = false;
    Cascade C;
    C.flist[0] = c->flist[0];
    C.flist[1] = c->flist[1];
    C.clist[0] = c->clist[0];
    C.clist[1] = c->clist[1];
    C.ctl = c->ctl;
    C.tail_thr = c->tail_threshold;
    C.back_thr = 4 * c->tail_threshold;
    PassOut P;
    P.flist = c->flist[1];
    P.clist = c->clist[1];
    P.fcount = &c->ctl->nface[1];
    P.ccount = &c->ctl->ncell[1];
    P.tcount = &c->ctl->ntroub[0];
    P.stamp = 0;  // set on the device from ctl->stamp0
    hipEvent_t *ev = nullptr;
    if (c->instrument) {
        while (c->evs.size() < 3 * (c->nev_used + 1)) {
            hipEvent_t x;
            HIPCHK(c, hipEventCreate(&x));
            c->evs.push_back(x);
        }
        ev = &c->evs[3 * c->nev_used];
        ++c->nev_used;
        HIPCHK(c, hipEventRecord(ev[0], c->stream));
    }
    // ev[1] is recorded between the first pass and its claims
    e = launch_first_pass<real>(A, P, C, ev ? ev[1] : nullptr, c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("first pass: ") + hipGetErrorString(e));

    // Cascade: a batch of multi-block passes (each returns at once when it has no
    // work or when the tail takes over), then the single-workgroup tail, then one
    // host check.  The tail hands back when a pass grows large again; the batch
    // length follows the previous stage's number of multi-block passes.
    int nb = (int)((c->ncell + 63) / 64);
    if (nb > 512) nb = 512;
    c->cstat[0] = c->cstat[1] = c->cstat[2] = 0;
    int k = 1;  // next cascade pass
    int batch = c->head_guess;
    for (;;) {
        if (k + batch > kMaxPasses - 1) batch = kMaxPasses - 1 - k;
        if (batch < 0) {
            c->last_npass = k - 1;
            return fail(c, GPM_ENOTCONV, "MOOD loop exceeded the pass limit");
        }
        for (int b = 0; b < batch; ++b) {
            e = launch_cascade_pass<real>(A, C, k + b, nb, c->stream);
            if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("cascade pass: ") + hipGetErrorString(e));
        }
        e = launch_cascade_tail<real>(A, C, k, k + batch, kMaxPasses, c->stream);
        if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("cascade tail: ") + hipGetErrorString(e));
        HIPCHK(c, hipMemcpyAsync(c->pinned, &c->ctl->tail_end, 4 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        const int tail_end = c->pinned[0], tail_k0 = c->pinned[1], back = c->pinned[2], tail_start = c->pinned[3];
        if (tail_end >= kMaxPasses) {
            c->last_npass = kMaxPasses - 1;
            return fail(c, GPM_ENOTCONV, "MOOD loop exceeded the pass limit");
        }
        // where the passes of this batch ran: multi-block k .. tail_start-1, the
        // tail tail_start .. tail_end-1
        c->cstat[0] += tail_start - k;
        c->cstat[1] += tail_end - tail_start;
        c->cstat[2] += back ? 1 : 0;
        if (!back) {
            // multi-block passes this stage needed before the tail (or the end)
            const int head = (tail_k0 > 0 ? tail_k0 : tail_end) - 1;
            int g = head + 2;
            g = g < c->passes_per_check ? c->passes_per_check : (g > 128 ? 128 : g);
            c->head_guess = g;
            k = tail_end;
            break;
        }
        k = tail_end;
        batch = batch < 8 ? 8 : (batch > 64 ? 128 : 2 * batch);
    }
    c->last_npass = k - 1;
    if (ev) {
        c->acc_iters += c->last_npass + 1;
        c->acc_stages += 1;
        if (c->instrument & 2) {
            st = level_counts(c);
            if (st != GPM_OK) return st;
            e = launch_stats(c->ctl, c->last_npass, 0, c->stream);
            if (e != hipSuccess) return fail(c, GPM_EHIP, hipGetErrorString(e));
        }
        HIPCHK(c, hipEventRecord(ev[2], c->stream));
    }
    return GPM_OK;
}

extern "C" {

gpm_status gpm_stage_coef(gpm_ctx *c, const void *B, const void *Us, void *Uout, double a, double b, double cf)
{
    if (!c) return GPM_EINVAL;
    if (!c->have_scheme) return fail(c, GPM_ESTATE, "no scheme set");
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    if (!Us || !Uout || (a != 0.0 && !B) || !(cf > 0.0) || !std::isfinite(a) || !std::isfinite(b) ||
        !std::isfinite(cf))
        return fail(c, GPM_EINVAL, "bad stage arguments");
    if (Uout == Us) return fail(c, GPM_EINVAL, "U_out must not alias U_s");
    const void *Bp = B ? B : Us;  // not read when a == 0
    return c->prec == GPM_F64 ? run_stage<double>(c, c->w64, 3, Bp, Us, Uout, a, b, cf)
                              : run_stage<float>(c, c->w32, 3, Bp, Us, Uout, a, b, cf);
}

gpm_status gpm_lincomb4(gpm_ctx *c, void *out, const void *x0, double w0, const void *x1, double w1, const void *x2,
                        double w2, const void *x3, double w3)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    if (!out || !x0 || !x1 || !x2 || !x3) return fail(c, GPM_EINVAL, "null array");
    const size_t n = 4 * c->ncell;
    const hipError_t e = c->prec == GPM_F64
                             ? launch_lincomb4<double>((double *)out, (const double *)x0, (const double *)x1,
                                                       (const double *)x2, (const double *)x3, w0, w1, w2, w3, n,
                                                       c->stream)
                             : launch_lincomb4<float>((float *)out, (const float *)x0, (const float *)x1,
                                                      (const float *)x2, (const float *)x3, w0, w1, w2, w3, n,
                                                      c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, hipGetErrorString(e));
    return GPM_OK;
}

gpm_status gpm_stage_dev(gpm_ctx *c, int s, const void *Un, const void *Us, void *Uout)
{
    if (!c) return GPM_EINVAL;
    if (!c->have_scheme) return fail(c, GPM_ESTATE, "no scheme set");
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    if (s < 0 || s > 2 || !Us || !Uout || (s > 0 && !Un)) return fail(c, GPM_EINVAL, "bad stage arguments");
    if (Uout == Us) return fail(c, GPM_EINVAL, "U_out must not alias U_s");
    return c->prec == GPM_F64 ? run_stage<double>(c, c->w64, s, Un, Us, Uout)
                              : run_stage<float>(c, c->w32, s, Un, Us, Uout);
}

gpm_status gpm_step(gpm_ctx *c, double cfl, int nsteps)
{
    if (!c || nsteps < 0) return GPM_EINVAL;
    if (!c->have_scheme) return fail(c, GPM_ESTATE, "no scheme set");
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    for (int n = 0; n < nsteps; ++n) {
        const int u0 = c->cur, a = (c->cur + 1) % 3, b = (c->cur + 2) % 3;
        if (cfl > 0.0) {
            gpm_status st = compute_dt_from(c, slot_ptr(c, u0), cfl);
            if (st != GPM_OK) return st;
        }
        gpm_status st = gpm_stage_dev(c, 0, slot_ptr(c, u0), slot_ptr(c, u0), slot_ptr(c, a));
        if (st != GPM_OK) return st;
        st = gpm_stage_dev(c, 1, slot_ptr(c, u0), slot_ptr(c, a), slot_ptr(c, b));
        if (st != GPM_OK) return st;
        st = gpm_stage_dev(c, 2, slot_ptr(c, u0), slot_ptr(c, b), slot_ptr(c, a));
        if (st != GPM_OK) return st;
        c->cur = a;
    }
    return GPM_OK;
}

gpm_status gpm_cascade_stats(const gpm_ctx *c, long long stats[3])
{
    if (!c || !stats) return GPM_EINVAL;
    for (int q = 0; q < 3; ++q) stats[q] = c->cstat[q];
    return GPM_OK;
}

gpm_status gpm_order_ptr(const gpm_ctx *c, void **order_dev)
{
    if (!c || !order_dev) return GPM_EINVAL;
    if (!c->state) return GPM_ESTATE;
    *order_dev = c->order;
    return GPM_OK;
}

}  // extern "C"

template <typename real>
static gpm_status stage_vjp(gpm_ctx *c, const Weights<real> &W, int s, const void *Un, const void *Us,
                            const void *order, double dt, const void *lam_out, void *lam_Us, void *lam_Un,
                            double *dL_dell, double *dl_dev)
{
    AdjArgs<real> J;
    fill_args(c, W, J.A);
    J.A.s = s;
    J.A.Un = (const real *)Un;
    J.A.Us = (const real *)Us;
    J.A.Uout = nullptr;
    J.A.order = (uint8_t *)order;
    J.lam_out = (const real *)lam_out;
    J.lam_Us = (real *)lam_Us;
    J.lam_Un = (real *)lam_Un;
    // the adjoint workspace holds the per-face records, the FP64 ell table and
    // the per-tile dL/d(ell) partials
    J.gface = (real *)c->adj;
    J.dl64 = (const double *)(c->adj + adj_face_bytes(c));
    J.dl_partial = (double *)(c->adj + adj_partial_offset(c));
    hipError_t e = launch_set_dt(c->ctl, dt, c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, hipGetErrorString(e));
    J.A.dt = &c->ctl->dt;
    const size_t nft = nfaces_x(c) + nfaces_y(c);
    int nblk = (int)((nft + 127) / 128);
    if (nblk > kTotBlocks * 8) nblk = kTotBlocks * 8;
    e = launch_stage_vjp<real>(J, nblk, dl_dev ? dl_dev : &c->ctl->totals[0], dl_dev != nullptr, c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, std::string("stage adjoint: ") + hipGetErrorString(e));
    if (dL_dell) {
        double d = 0.0;
        HIPCHK(c, hipMemcpyAsync(&d, &c->ctl->totals[0], sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        *dL_dell += d;
    }
    return GPM_OK;
}

extern "C" {

static gpm_status stage_vjp_checked(gpm_ctx *c, int s, const void *Un, const void *Us, const void *order, double dt,
                                    const void *lam_out, void *lam_Us, void *lam_Un, double *dL_dell, double *dl_dev)
{
    if (!c) return GPM_EINVAL;
    if (!c->have_scheme) return fail(c, GPM_ESTATE, "no scheme set");
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    if (s < 0 || s > 2 || !Us || !order || !lam_out || !lam_Us || (s > 0 && (!Un || !lam_Un)) || !(dt > 0.0))
        return fail(c, GPM_EINVAL, "bad adjoint arguments");
    if (lam_Us == lam_out || (s > 0 && (lam_Un == lam_out || lam_Un == lam_Us)))
        return fail(c, GPM_EINVAL, "adjoint outputs must not alias");
    if (c->grid.bc[0] == GPM_BC_REFLECT || c->grid.bc[1] == GPM_BC_REFLECT)
        return fail(c, GPM_EUNSUPPORTED, "the stage adjoint has periodic and outflow boundaries only");
    if (c->scheme.solver != GPM_SOLVER_HLLC)
        return fail(c, GPM_EUNSUPPORTED, "the stage adjoint differentiates the HLLC scheme only");
    if (c->grid.slit != 0) return fail(c, GPM_EUNSUPPORTED, "the stage adjoint has no inflow slit");
    if (!c->adj) return fail(c, GPM_ESTATE, "no adjoint workspace bound (gpm_bind_adjoint)");
    return c->prec == GPM_F64
               ? stage_vjp<double>(c, c->w64, s, Un, Us, order, dt, lam_out, lam_Us, lam_Un, dL_dell, dl_dev)
               : stage_vjp<float>(c, c->w32, s, Un, Us, order, dt, lam_out, lam_Us, lam_Un, dL_dell, dl_dev);
}

gpm_status gpm_stage_vjp(gpm_ctx *c, int s, const void *Un, const void *Us, const void *order, double dt,
                         const void *lam_out, void *lam_Us, void *lam_Un, double *dL_dell)
{
    return stage_vjp_checked(c, s, Un, Us, order, dt, lam_out, lam_Us, lam_Un, dL_dell, nullptr);
}

gpm_status gpm_stage_vjp_acc(gpm_ctx *c, int s, const void *Un, const void *Us, const void *order, double dt,
                             const void *lam_out, void *lam_Us, void *lam_Un, void *dl_dev)
{
    if (!c) return GPM_EINVAL;
    if (!dl_dev || ((uintptr_t)dl_dev & 7u)) return fail(c, GPM_EINVAL, "dl_dev: NULL or not 8-byte aligned");
    return stage_vjp_checked(c, s, Un, Us, order, dt, lam_out, lam_Us, lam_Un, nullptr, (double *)dl_dev);
}

gpm_status gpm_adjoint_workspace_size(const gpm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return GPM_EINVAL;
    *bytes = adj_bytes(c);
    return GPM_OK;
}

gpm_status gpm_bind_adjoint(gpm_ctx *c, void *adj_work)
{
    if (!c || !adj_work || ((uintptr_t)adj_work & 255u)) return fail(c, GPM_EINVAL, "adjoint workspace: NULL or not 256-byte aligned");
    c->adj = (char *)adj_work;
    return upload_adj_dl(c);
}

gpm_status gpm_troubled_counts(gpm_ctx *c, long long counts[4], int *mood_iters)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    gpm_status st = level_counts(c);
    if (st != GPM_OK) return st;
    unsigned long long lc[4];
    HIPCHK(c, hipMemcpyAsync(lc, c->ctl->levcnt, sizeof(lc), hipMemcpyDeviceToHost, c->stream));
    std::vector<int> nc(c->last_npass + 2);
    HIPCHK(c, hipMemcpyAsync(nc.data(), c->ctl->ncell, sizeof(int) * nc.size(), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (counts)
        for (int l = 0; l < 4; ++l) counts[l] = (long long)lc[l];
    if (mood_iters) {
        int it = 1;
        for (size_t k = 1; k < nc.size(); ++k)
            if (nc[k] > 0) ++it;
        *mood_iters = it;
    }
    return GPM_OK;
}

gpm_status gpm_get_order_mask(gpm_ctx *c, unsigned char *out)
{
    if (!c || !out) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    HIPCHK(c, hipMemcpyAsync(out, c->order, c->ncell, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GPM_OK;
}

gpm_status gpm_totals_dev(gpm_ctx *c, const void *U, double totals[4])
{
    if (!c || !U || !totals) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    int nblk = (int)((c->ncell + 255) / 256);
    if (nblk > kTotBlocks) nblk = kTotBlocks;
    const double area = c->dx * c->dy;
    hipError_t e = c->prec == GPM_F64
                       ? launch_totals<double>((const double *)U, c->ncell, area, c->partial, nblk, c->ctl->totals,
                                               c->stream)
                       : launch_totals<float>((const float *)U, c->ncell, area, c->partial, nblk, c->ctl->totals,
                                              c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, hipGetErrorString(e));
    HIPCHK(c, hipMemcpyAsync(totals, c->ctl->totals, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GPM_OK;
}

// Scratch of gpm_totals_static, the totals entry point that allocates nothing:
// the block partials (kTotBlocks blocks x 4 variables x a double-double) and the
// four results.  Every device the library runs on holds one copy until the
// process ends.  In host code the symbol is only a stand-in: its device address
// comes from hipGetSymbolAddress, once per device (static_scratch below).
constexpr size_t kStaticPartials = (size_t)kTotBlocks * 4 * 2;
constexpr size_t kStaticDoubles = kStaticPartials + 4;
static __device__ __align__(256) double scratch[kStaticDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Device address of this device's scratch (looked up on the first call per device,
// with that device current).
static gpm_status static_scratch(gpm_ctx *c, double **out)
{
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(c, GPM_EUNSUPPORTED, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return fail(c, GPM_EHIP, e != hipSuccess ? hipGetErrorString(e) : "no scratch address");
        g_scratch_ptr[dev] = (double *)p;
    }
    *out = g_scratch_ptr[dev];
    return GPM_OK;
}

gpm_status gpm_totals_static(gpm_ctx *c, const void *U, double totals[4])
{
    if (!c || !U || !totals) return GPM_EINVAL;
    int nblk = (int)((c->ncell + 255) / 256);
    if (nblk > kTotBlocks) nblk = kTotBlocks;  // the kernels stride over any larger grid
    if ((size_t)nblk * 4 * 2 > kStaticPartials) return fail(c, GPM_EINVAL, "partials exceed the static scratch");
    double *ptr = nullptr;
    gpm_status st = static_scratch(c, &ptr);
    if (st != GPM_OK) return st;
    const double area = c->dx * c->dy;
    // every partial the final sum reads is written by this call's first kernel, so
    // nothing needs clearing
    hipError_t e = c->prec == GPM_F64
                       ? launch_totals<double>((const double *)U, c->ncell, area, ptr, nblk, ptr + kStaticPartials,
                                               c->stream)
                       : launch_totals<float>((const float *)U, c->ncell, area, ptr, nblk, ptr + kStaticPartials,
                                              c->stream);
    if (e != hipSuccess) return fail(c, GPM_EHIP, hipGetErrorString(e));
    HIPCHK(c, hipMemcpyAsync(totals, ptr + kStaticPartials, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return GPM_OK;
}

gpm_status gpm_totals(gpm_ctx *c, double totals[4])
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    return gpm_totals_dev(c, slot_ptr(c, c->cur), totals);
}

gpm_status gpm_instrument(gpm_ctx *c, int enable)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    if (enable < 0 || enable > 3) return fail(c, GPM_EINVAL, "instrument mode must be 0..3");
    if (enable) {
        hipError_t e = launch_stats(c->ctl, 0, 1, c->stream);
        if (e != hipSuccess) return fail(c, GPM_EHIP, hipGetErrorString(e));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->nev_used = 0;
        c->acc_iters = 0;
        c->acc_stages = 0;
    }
    c->instrument = enable == 2 ? 3 : enable;
    return GPM_OK;
}

gpm_status gpm_instrument_read(gpm_ctx *c, double *first_pass_ms, long long *first_pass_launches,
                               double *cascade_ms, long long *stages, long long level_cells[4],
                               long long *mood_iters)
{
    if (!c) return GPM_EINVAL;
    if (!c->state) return fail(c, GPM_ESTATE, "not bound");
    unsigned long long acc[6];
    HIPCHK(c, hipMemcpyAsync(acc, c->ctl->acc_lev, sizeof(acc), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double fp = 0.0, cm = 0.0;
    for (size_t k = 0; k < c->nev_used; ++k) {
        float a = 0.f, b = 0.f;
        HIPCHK(c, hipEventElapsedTime(&a, c->evs[3 * k], c->evs[3 * k + 1]));
        HIPCHK(c, hipEventElapsedTime(&b, c->evs[3 * k + 1], c->evs[3 * k + 2]));
        fp += a;
        cm += b;
    }
    if (first_pass_ms) *first_pass_ms = fp;
    if (first_pass_launches) *first_pass_launches = (long long)c->nev_used;
    if (cascade_ms) *cascade_ms = cm;
    if (stages) *stages = (long long)c->nev_used;
    if (level_cells)
        for (int l = 0; l < 4; ++l) level_cells[l] = (long long)acc[l];
    if (mood_iters) *mood_iters = c->acc_iters;
    return GPM_OK;
}

}  // extern "C"
