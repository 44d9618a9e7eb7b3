// C ABI of the batched ensemble: many independent 2D problems (uneven grid sizes,
// one scheme) advanced together, one launch per kernel kind and stage for the
// whole batch, optionally replayed as HIP graphs (see include/gpmood.h).
//
// Every problem keeps its own single-problem context (weights, workspace, state
// slots, control block) inside one caller buffer.  Device tables hold, for each
// of the three slot rotations of an SSP-RK3 step and each stage, every problem's
// stage arguments, so a step's launches never change their arguments and a
// captured step graph can be replayed: the claim stamps advance on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "gpmood.h"
#include "gpmood_ctx.h"
#include "gp_weights.h"

namespace {

// First-pass block count of one problem (strips of 62 columns x `rows` rows,
// WPB wavefronts per block) and dt blocks (256 threads, up to 16 cells each).
int fp_blocks(const gpm_ctx *c, int rows)
{
    const int wpb = c->prec == GPM_F64 ? 2 : 4;
    const int waves = ((c->nx + 61) / 62) * ((c->ny + rows - 1) / rows);
    return (waves + wpb - 1) / wpb;
}

int dt_blocks(const gpm_ctx *c)
{
    const size_t b = (c->ncell + 4095) / 4096;
    return (int)(b < 1 ? 1 : b);
}


}  // namespace

struct gpm_batch {
    int nprob = 0;
    int prec = GPM_F32;
    hipStream_t stream = nullptr;
    std::vector<gpm_ctx *> ctx;
    bool have_scheme = false;
    char *mem = nullptr;
    int rows = 12;
    std::vector<int> prow;      // first-pass rows per wavefront of each problem (empty: rows)
    int cur = 0;  // slot rotation of the next step (the same for every problem)
    // device tables (inside the caller buffer)
    void *args = nullptr;       // StageArgs<real>[3 rotations][3 stages][nprob]
    PassOut *pout[3] = {};      // per stage: first-pass outputs [nprob]
    Cascade *casc = nullptr;    // [nprob]
    int *blk = nullptr;         // [nprob + 1]
    int *dblk = nullptr;        // [nprob + 1]
    int *plan = nullptr;        // [2][nprob + 1] (written on the device each cascade pass)
    int *st_iters = nullptr;    // [nprob]
    double *st_dt = nullptr;    // [nprob]
    int nfp = 0, ndt = 0;
    int iso = 0;                // every problem has isotropic weights
    int walls = 0;              // some problem has a reflecting axis
    // graphs: one captured SSP-RK3 step per rotation
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t graph[3] = {nullptr, nullptr, nullptr};
    double graph_cfl = -1.0;
    unsigned long long stages_run = 0;  // since the stamps were last cleared
    std::string err;
};

static gpm_status bfail(gpm_batch *b, gpm_status st, const std::string &msg)
{
    if (b) b->err = msg;
    return st;
}

#define BHIPCHK(b, expr)                                                                     \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return bfail((b), GPM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

// Byte layout of the caller buffer: per problem its three state slots and its
// workspace, then the tables.
struct BatchLayout {
    std::vector<size_t> state_off, work_off;
    size_t args, pout, casc, blk, dblk, plan, iters, dts, total;
};

static BatchLayout batch_layout(const gpm_batch *b)
{
    BatchLayout L;
    size_t o = 0;
    for (int p = 0; p < b->nprob; ++p) {
        size_t woff[W_N];
        L.state_off.push_back(o);
        o = align_up(o + 3 * state_slot_bytes(b->ctx[p]));
        L.work_off.push_back(o);
        o = align_up(o + work_layout(b->ctx[p], woff));
    }
    const size_t asz = b->prec == GPM_F64 ? sizeof(StageArgs<double>) : sizeof(StageArgs<float>);
    L.args = o;
    o = align_up(o + 9 * (size_t)b->nprob * asz);
    L.pout = o;
    o = align_up(o + 3 * (size_t)b->nprob * sizeof(PassOut));
    L.casc = o;
    o = align_up(o + (size_t)b->nprob * sizeof(Cascade));
    L.blk = o;
    o = align_up(o + (size_t)(b->nprob + 1) * sizeof(int));
    L.dblk = o;
    o = align_up(o + (size_t)(b->nprob + 1) * sizeof(int));
    L.plan = o;
    o = align_up(o + 2 * (size_t)(b->nprob + 1) * sizeof(int));
    L.iters = o;
    o = align_up(o + (size_t)b->nprob * sizeof(int));
    L.dts = o;
    o = align_up(o + (size_t)b->nprob * sizeof(double));
    L.total = o;
    return L;
}

static void drop_graphs(gpm_batch *b)
{
    for (int r = 0; r < 3; ++r)
        if (b->graph[r]) {
            (void)hipGraphExecDestroy(b->graph[r]);
            b->graph[r] = nullptr;
        }
    b->graph_cfl = -1.0;
}

// Fill and upload the device tables (after bind and scheme, or a tuning change).
template <typename real>
static gpm_status build_tables(gpm_batch *b)
{
    const int P = b->nprob;
    std::vector<StageArgs<real>> args(9 * (size_t)P);
    std::vector<PassOut> pout(3 * (size_t)P);
    std::vector<Cascade> casc(P);
    std::vector<int> blk(P + 1), dblk(P + 1);
    blk[0] = dblk[0] = 0;
    for (int p = 0; p < P; ++p) {
        gpm_ctx *c = b->ctx[p];
        c->rows = b->prow.empty() ? b->rows : b->prow[p];
        const Weights<real> &W = *(const Weights<real> *)(sizeof(real) == 8 ? (const void *)&c->w64 : (const void *)&c->w32);
        for (int r = 0; r < 3; ++r) {
            const int u0 = r, a = (r + 1) % 3, bb = (r + 2) % 3;
            const int un[3] = {u0, u0, u0}, us[3] = {u0, a, bb}, uo[3] = {a, bb, a};
            for (int s = 0; s < 3; ++s) {
                StageArgs<real> &A = args[((size_t)r * 3 + s) * P + p];
                fill_args(c, W, A);
                A.s = s;
                A.Un = (const real *)slot_ptr(c, un[s]);
                A.Us = (const real *)slot_ptr(c, us[s]);
                A.Uout = (real *)slot_ptr(c, uo[s]);
            }
        }
        for (int s = 0; s < 3; ++s) {
            PassOut &Q = pout[(size_t)s * P + p];
            Q.flist = c->flist[1];
            Q.clist = c->clist[1];
            Q.fcount = &c->ctl->nface[1];
            Q.ccount = &c->ctl->ncell[1];
            Q.tcount = &c->ctl->ntroub[0];
            Q.stamp = 0;  // set on the device from ctl->stamp0
        }
        Cascade &C = casc[p];
        C.flist[0] = c->flist[0];
        C.flist[1] = c->flist[1];
        C.clist[0] = c->clist[0];
        C.clist[1] = c->clist[1];
        C.ctl = c->ctl;
        // multi-block passes while the previous evaluation left more than
        // tail_threshold troubled cells, then one workgroup per problem to the end
        C.tail_thr = c->tail_threshold;
        C.back_thr = 0x7fffffff;
        blk[p + 1] = blk[p] + fp_blocks(c, c->rows);
        dblk[p + 1] = dblk[p] + dt_blocks(c);
    }
    b->iso = 1;
    b->walls = 0;
    for (size_t k = 0; k < args.size(); ++k) {
        b->iso &= args[k].iso;
        b->walls |= (args[k].bcx == GPM_BC_REFLECT || args[k].bcy == GPM_BC_REFLECT) ? 1 : 0;
    }
    b->nfp = blk[P];
    b->ndt = dblk[P];
    const BatchLayout L = batch_layout(b);
    BHIPCHK(b, hipMemcpyAsync(b->mem + L.args, args.data(), args.size() * sizeof(StageArgs<real>),
                              hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipMemcpyAsync(b->mem + L.pout, pout.data(), pout.size() * sizeof(PassOut), hipMemcpyHostToDevice,
                              b->stream));
    BHIPCHK(b, hipMemcpyAsync(b->mem + L.casc, casc.data(), casc.size() * sizeof(Cascade), hipMemcpyHostToDevice,
                              b->stream));
    BHIPCHK(b, hipMemcpyAsync(b->mem + L.blk, blk.data(), blk.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipMemcpyAsync(b->mem + L.dblk, dblk.data(), dblk.size() * sizeof(int), hipMemcpyHostToDevice,
                              b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    drop_graphs(b);
    return GPM_OK;
}

static gpm_status rebuild(gpm_batch *b)
{
    if (!b->mem || !b->have_scheme) return GPM_OK;
    return b->prec == GPM_F64 ? build_tables<double>(b) : build_tables<float>(b);
}

template <typename real>
static BatchTabs<real> tabs(const gpm_batch *b, int rot, int s)
{
    BatchTabs<real> B;
    B.args = (const StageArgs<real> *)b->args + ((size_t)rot * 3 + s) * b->nprob;
    B.pout = b->pout[s];
    B.casc = b->casc;
    B.blk = b->blk;
    B.dblk = b->dblk;
    B.plan = b->plan;
    B.nprob = b->nprob;
    B.iso = b->iso;
    B.walls = b->walls;
    B.solver = b->ctx[0]->scheme.solver;
    return B;
}

// Enqueue one SSP-RK3 step with slot rotation rot on stream st.
template <typename real>
static hipError_t enqueue_step(gpm_batch *b, int rot, double cfl, hipStream_t st)
{
    const int top = b->ctx[0]->top;
    hipError_t e = launch_batch_dt<real>(tabs<real>(b, rot, 0), b->ndt, b->casc, cfl, st);
    for (int s = 0; s < 3 && e == hipSuccess; ++s)
        e = launch_batch_stage<real>(tabs<real>(b, rot, s), top, b->nfp, b->casc, st);
    return e;
}

static hipError_t enqueue_step_any(gpm_batch *b, int rot, double cfl, hipStream_t st)
{
    return b->prec == GPM_F64 ? enqueue_step<double>(b, rot, cfl, st) : enqueue_step<float>(b, rot, cfl, st);
}

// The claim stamps advance by kMaxPasses + 2 per stage on the device; clear the
// stamp arrays before they would wrap.
static gpm_status stamps_guard(gpm_batch *b, int nsteps)
{
    const unsigned long long per = (unsigned long long)kMaxPasses + 2;
    if ((b->stages_run + 3ull * nsteps + 3ull) * per < 0xffffffffull) return GPM_OK;
    for (gpm_ctx *c : b->ctx) {
        BHIPCHK(b, hipMemsetAsync(c->cstamp, 0, 4 * c->ncell, b->stream));
        BHIPCHK(b, hipMemsetAsync(c->fstamp, 0, 4 * (nfaces_x(c) + nfaces_y(c)), b->stream));
    }
    BHIPCHK(b, launch_batch_stamp_restart(b->casc, b->nprob, b->stream));
    b->stages_run = 0;
    if ((3ull * nsteps + 3ull) * per >= 0xffffffffull) return bfail(b, GPM_EINVAL, "too many steps in one call");
    return GPM_OK;
}

// Candidate march lengths of the autotuner, and the time of `reps` batch stage-0
// first passes (after one untimed launch) between two HIP events.
static const int kTuneRows[] = {4, 6, 8, 12, 16, 24, 32, 64};

template <typename real>
static gpm_status time_first_pass(gpm_batch *b, int reps, hipEvent_t e0, hipEvent_t e1, float *ms)
{
    const int top = b->ctx[0]->top;
    BHIPCHK(b, launch_batch_first_pass<real>(tabs<real>(b, b->cur, 0), top, b->nfp, b->casc, b->stream));
    BHIPCHK(b, hipEventRecord(e0, b->stream));
    for (int r = 0; r < reps; ++r)
        BHIPCHK(b, launch_batch_first_pass<real>(tabs<real>(b, b->cur, 0), top, b->nfp, b->casc, b->stream));
    BHIPCHK(b, hipEventRecord(e1, b->stream));
    BHIPCHK(b, hipEventSynchronize(e1));
    BHIPCHK(b, hipEventElapsedTime(ms, e0, e1));
    b->stages_run += (unsigned long long)reps + 1;
    return GPM_OK;
}

// Candidate cascade thresholds (troubled cells at or below which a problem's
// cascade leaves the batch-wide multi-block passes for its tail workgroup), and
// the time of `reps` whole batch stage-0 stages (first pass and cascade, after
// one untimed stage) between two HIP events.  Stage 0 reads the current slot and
// writes another, so the states are left as they were.
static const int kTuneTail[] = {8, 16, 32, 64, 128, 256};

template <typename real>
static gpm_status time_stage0(gpm_batch *b, int reps, hipEvent_t e0, hipEvent_t e1, float *ms)
{
    const int top = b->ctx[0]->top;
    BHIPCHK(b, launch_batch_stage<real>(tabs<real>(b, b->cur, 0), top, b->nfp, b->casc, b->stream));
    BHIPCHK(b, hipEventRecord(e0, b->stream));
    for (int r = 0; r < reps; ++r)
        BHIPCHK(b, launch_batch_stage<real>(tabs<real>(b, b->cur, 0), top, b->nfp, b->casc, b->stream));
    BHIPCHK(b, hipEventRecord(e1, b->stream));
    BHIPCHK(b, hipEventSynchronize(e1));
    BHIPCHK(b, hipEventElapsedTime(ms, e0, e1));
    b->stages_run += (unsigned long long)reps + 1;
    return GPM_OK;
}

static gpm_status set_tail(gpm_batch *b, int tail)
{
    for (gpm_ctx *c : b->ctx) c->tail_threshold = tail;
    return rebuild(b);
}

extern "C" {

gpm_status gpm_batch_create(int nprob, const gpm_grid *grids, int prec, void *hip_stream, gpm_batch **out)
{
    if (!out || !grids || nprob < 1 || nprob > 65536) return GPM_EINVAL;
    *out = nullptr;
    for (int p = 0; p < nprob; ++p)
        if (grids[p].slit != 0) return GPM_EUNSUPPORTED;  // single problems only (checked before allocating)
    gpm_batch *b = new (std::nothrow) gpm_batch;
    if (!b) return GPM_ENOMEM;
    b->nprob = nprob;
    b->prec = prec;
    b->stream = (hipStream_t)hip_stream;
    for (int p = 0; p < nprob; ++p) {
        gpm_ctx *c = nullptr;
        const gpm_status st = gpm_create(&grids[p], prec, hip_stream, &c);
        if (st != GPM_OK) {
            for (gpm_ctx *x : b->ctx) gpm_destroy(x);
            delete b;
            return st;
        }
        b->ctx.push_back(c);
    }
    *out = b;
    return GPM_OK;
}

void gpm_batch_destroy(gpm_batch *b)
{
    if (!b) return;
    drop_graphs(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    for (gpm_ctx *c : b->ctx) gpm_destroy(c);
    delete b;
}

const char *gpm_batch_last_error(const gpm_batch *b) { return b ? b->err.c_str() : ""; }

gpm_status gpm_batch_set_scheme(gpm_batch *b, const gpm_scheme *s)
{
    if (!b || !s) return GPM_EINVAL;
    for (int p = 0; p < b->nprob; ++p) {
        gpm_ctx *c = b->ctx[p];
        // problems with the same cell aspect share their weights (ell in cells)
        const double ell = s->ell > 0.0 ? s->ell : 12.0 * (c->dx < c->dy ? c->dx : c->dy);
        int q = -1;
        for (int r = 0; r < p && q < 0; ++r) {
            const gpm_ctx *d = b->ctx[r];
            const double elld = s->ell > 0.0 ? s->ell : 12.0 * (d->dx < d->dy ? d->dx : d->dy);
            if (ell / c->dx == elld / d->dx && ell / c->dy == elld / d->dy) q = r;
        }
        if (q < 0) {
            const gpm_status st = gpm_set_scheme(c, s);
            if (st != GPM_OK) return bfail(b, st, std::string("problem ") + std::to_string(p) + ": " + c->err);
        } else {
            const gpm_ctx *d = b->ctx[q];
            c->w64 = d->w64;
            c->w32 = d->w32;
            // the u2 curvature weights are second derivatives in physical units
            // (they scale with 1 / dx^2): this problem's own
            GpwCurv K;
            if (gpw_curvature(ell / c->dx, ell / c->dy, ell, &K) != 0)
                return bfail(b, GPM_EINVAL, std::string("problem ") + std::to_string(p) +
                                                ": GP-R1 covariance matrix not positive definite");
            for (int dd = 0; dd < 2; ++dd)
                for (int k = 0; k < 3; ++k) {
                    c->w64.curv[dd][k] = K.w64[dd][k];
                    c->w32.curv[dd][k] = K.w32[dd][k];
                }
            c->gtab64 = d->gtab64;
            c->gtab32 = d->gtab32;
            // the ell-derivative part scales with 1 / ell
            const double elld = d->scheme.ell;
            for (int k = kGtabSize; k < 2 * kGtabSize; ++k) {
                c->gtab64[k] = d->gtab64[k] * (elld / ell);
                c->gtab32[k] = (float)c->gtab64[k];
            }
            c->scheme = d->scheme;
            c->scheme.ell = ell;
            c->top = d->top;
            for (int r = 0; r < 4; ++r) {
                c->next[r] = d->next[r];
                c->levidx[r] = d->levidx[r];
            }
            c->have_scheme = true;
            const gpm_status st = upload_gtab(c);
            if (st != GPM_OK) return bfail(b, st, c->err);
        }
    }
    b->have_scheme = true;
    return rebuild(b);
}

gpm_status gpm_batch_workspace_size(const gpm_batch *b, size_t *bytes)
{
    if (!b || !bytes) return GPM_EINVAL;
    *bytes = batch_layout(b).total;
    return GPM_OK;
}

gpm_status gpm_batch_bind(gpm_batch *b, void *mem)
{
    if (!b || !mem) return GPM_EINVAL;
    if ((uintptr_t)mem % kAlign) return bfail(b, GPM_EINVAL, "buffer must be 256-byte aligned");
    const BatchLayout L = batch_layout(b);
    b->mem = (char *)mem;
    for (int p = 0; p < b->nprob; ++p) {
        const gpm_status st = gpm_bind(b->ctx[p], b->mem + L.state_off[p], b->mem + L.work_off[p]);
        if (st != GPM_OK) return bfail(b, st, b->ctx[p]->err);
    }
    b->args = b->mem + L.args;
    const size_t psz = (size_t)b->nprob * sizeof(PassOut);
    for (int s = 0; s < 3; ++s) b->pout[s] = (PassOut *)(b->mem + L.pout + s * psz);
    b->casc = (Cascade *)(b->mem + L.casc);
    b->blk = (int *)(b->mem + L.blk);
    b->dblk = (int *)(b->mem + L.dblk);
    b->plan = (int *)(b->mem + L.plan);
    b->st_iters = (int *)(b->mem + L.iters);
    b->st_dt = (double *)(b->mem + L.dts);
    b->cur = 0;
    b->stages_run = 0;
    return rebuild(b);
}

gpm_status gpm_batch_set_tuning(gpm_batch *b, int rows_per_wave)
{
    if (!b || rows_per_wave < 4 || rows_per_wave > 256) return GPM_EINVAL;
    b->rows = rows_per_wave;
    b->prow.clear();
    return rebuild(b);
}

gpm_status gpm_batch_set_tuning_per_problem(gpm_batch *b, const int *rows)
{
    if (!b || !rows) return GPM_EINVAL;
    for (int p = 0; p < b->nprob; ++p)
        if (rows[p] < 4 || rows[p] > 256) return bfail(b, GPM_EINVAL, "rows per wave must be 4..256");
    b->prow.assign(rows, rows + b->nprob);
    return rebuild(b);
}

// The autotuner: the first pass's march length (rows per wavefront) chosen per
// size class of problem (problems whose cell counts share a power of two), by
// timing the batch's stage-0 first pass on the device with HIP events.  Stage 0
// reads the current slot and writes another, so the timed launches leave the
// problems' states as they were.  One sweep of coordinate descent, the classes
// with the most cells first, each over the candidates below; ties keep the
// shorter march.  The choice changes the schedule only: every stage gives the same
// bits whatever the march length.
gpm_status gpm_batch_autotune(gpm_batch *b, double cfl, int reps, int *rows_out, double *gain)
{
    if (!b || reps < 1 || reps > 64 || !(cfl > 0.0)) return GPM_EINVAL;
    if (!b->mem || !b->have_scheme) return bfail(b, GPM_ESTATE, "not bound or no scheme");
    const int P = b->nprob;
    // size classes
    std::vector<int> cls(P);
    std::vector<long long> cells(64, 0);
    for (int p = 0; p < P; ++p) {
        int k = 0;
        while (k < 62 && (1ull << (k + 1)) <= (unsigned long long)b->ctx[p]->ncell) ++k;
        cls[p] = k;
        cells[k] += (long long)b->ctx[p]->ncell;
    }
    std::vector<int> order;
    for (int k = 0; k < 64; ++k)
        if (cells[k] > 0) order.push_back(k);
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cells[x] > cells[y]; });
    // the stages' dt (as a step would compute it) for realistic detection work
    gpm_status st = stamps_guard(b, 64 * (int)(sizeof(kTuneRows) / sizeof(int)) * (int)order.size());
    if (st != GPM_OK) return st;
    const hipError_t de = b->prec == GPM_F64
                              ? launch_batch_dt<double>(tabs<double>(b, b->cur, 0), b->ndt, b->casc, cfl, b->stream)
                              : launch_batch_dt<float>(tabs<float>(b, b->cur, 0), b->ndt, b->casc, cfl, b->stream);
    BHIPCHK(b, de);
    std::vector<int> rows(P);
    for (int p = 0; p < P; ++p) rows[p] = b->prow.empty() ? b->rows : b->prow[p];
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    for (size_t oi = 0; oi < order.size() && st == GPM_OK; ++oi) {
        const int k = order[oi];
        int best = -1;
        float tbest = 0.f;
        for (int cand : kTuneRows) {
            for (int p = 0; p < P; ++p)
                if (cls[p] == k) rows[p] = cand;
            b->prow = rows;
            st = rebuild(b);
            float ms = 0.f;
            if (st == GPM_OK)
                st = b->prec == GPM_F64 ? time_first_pass<double>(b, reps, e0, e1, &ms)
                                        : time_first_pass<float>(b, reps, e0, e1, &ms);
            if (st != GPM_OK) break;
            if (best < 0 || ms < tbest) {
                best = cand;
                tbest = ms;
            }
        }
        if (st != GPM_OK) break;
        for (int p = 0; p < P; ++p)
            if (cls[p] == k) rows[p] = best;
    }
    // the default march length and the chosen ones, timed alike
    float tdef = 0.f, ttun = 0.f;
    if (st == GPM_OK) {
        b->prow.clear();
        st = rebuild(b);
        if (st == GPM_OK)
            st = b->prec == GPM_F64 ? time_first_pass<double>(b, reps, e0, e1, &tdef)
                                    : time_first_pass<float>(b, reps, e0, e1, &tdef);
    }
    if (st == GPM_OK) {
        b->prow = rows;
        st = rebuild(b);
        if (st == GPM_OK)
            st = b->prec == GPM_F64 ? time_first_pass<double>(b, reps, e0, e1, &ttun)
                                    : time_first_pass<float>(b, reps, e0, e1, &ttun);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GPM_OK) return st;
    if (rows_out)
        for (int p = 0; p < P; ++p) rows_out[p] = rows[p];
    if (gain) *gain = ttun > 0.f ? (double)tdef / (double)ttun : 1.0;
    return st;
}

// Choose the cascade threshold of the whole batch (see kTuneTail) by timing whole
// stage-0 stages at the current states' dt; the problems' states are left as they
// were.  Like the march length, the threshold changes the schedule only.
gpm_status gpm_batch_autotune_cascade(gpm_batch *b, double cfl, int reps, int *tail_out, double *gain)
{
    if (!b || reps < 1 || reps > 64 || !(cfl > 0.0)) return GPM_EINVAL;
    if (!b->mem || !b->have_scheme) return bfail(b, GPM_ESTATE, "not bound or no scheme");
    const int ncand = (int)(sizeof(kTuneTail) / sizeof(int));
    gpm_status st = stamps_guard(b, (ncand + 2) * (reps + 1));
    if (st != GPM_OK) return st;
    const hipError_t de = b->prec == GPM_F64
                              ? launch_batch_dt<double>(tabs<double>(b, b->cur, 0), b->ndt, b->casc, cfl, b->stream)
                              : launch_batch_dt<float>(tabs<float>(b, b->cur, 0), b->ndt, b->casc, cfl, b->stream);
    BHIPCHK(b, de);
    const int tail0 = b->ctx[0]->tail_threshold;
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    int best = tail0;
    float tbest = -1.f, tdef = 0.f;
    for (int i = -1; i < ncand && st == GPM_OK; ++i) {
        const int cand = i < 0 ? tail0 : kTuneTail[i];  // the current setting first, as the reference
        st = set_tail(b, cand);
        float ms = 0.f;
        if (st == GPM_OK)
            st = b->prec == GPM_F64 ? time_stage0<double>(b, reps, e0, e1, &ms) : time_stage0<float>(b, reps, e0, e1, &ms);
        if (st != GPM_OK) break;
        if (i < 0) tdef = ms;
        if (tbest < 0.f || ms < tbest) {
            best = cand;
            tbest = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == GPM_OK) st = set_tail(b, best);
    if (st != GPM_OK) return st;
    if (tail_out) *tail_out = best;
    if (gain) *gain = tbest > 0.f ? (double)tdef / (double)tbest : 1.0;
    return GPM_OK;
}

gpm_status gpm_batch_init_state(gpm_batch *b, int p, const double *U)
{
    if (!b || p < 0 || p >= b->nprob) return GPM_EINVAL;
    gpm_ctx *c = b->ctx[p];
    c->cur = b->cur;
    const gpm_status st = gpm_init_state(c, U);
    return st == GPM_OK ? st : bfail(b, st, c->err);
}

gpm_status gpm_batch_get_state(gpm_batch *b, int p, double *U)
{
    if (!b || p < 0 || p >= b->nprob) return GPM_EINVAL;
    gpm_ctx *c = b->ctx[p];
    c->cur = b->cur;
    const gpm_status st = gpm_get_state(c, U);
    return st == GPM_OK ? st : bfail(b, st, c->err);
}

gpm_status gpm_batch_step(gpm_batch *b, double cfl, int nsteps, int use_graph)
{
    if (!b || nsteps < 0) return GPM_EINVAL;
    if (!(cfl > 0.0)) return bfail(b, GPM_EINVAL, "cfl must be > 0");
    if (!b->have_scheme) return bfail(b, GPM_ESTATE, "no scheme set");
    if (!b->mem) return bfail(b, GPM_ESTATE, "not bound");
    gpm_status st = stamps_guard(b, nsteps);
    if (st != GPM_OK) return st;
    if (use_graph) {
        if (cfl != b->graph_cfl) {
            drop_graphs(b);
            if (!b->cap_stream) BHIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
            for (int r = 0; r < 3; ++r) {
                hipGraph_t g = nullptr;
                BHIPCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
                const hipError_t e = enqueue_step_any(b, r, cfl, b->cap_stream);
                const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
                if (e != hipSuccess || e2 != hipSuccess) {
                    if (g) (void)hipGraphDestroy(g);
                    return bfail(b, GPM_EHIP, std::string("graph capture: ") +
                                                  hipGetErrorString(e != hipSuccess ? e : e2));
                }
                const hipError_t e3 = hipGraphInstantiate(&b->graph[r], g, nullptr, nullptr, 0);
                (void)hipGraphDestroy(g);
                if (e3 != hipSuccess) return bfail(b, GPM_EHIP, std::string("graph: ") + hipGetErrorString(e3));
            }
            b->graph_cfl = cfl;
        }
        for (int n = 0; n < nsteps; ++n) {
            BHIPCHK(b, hipGraphLaunch(b->graph[b->cur], b->stream));
            b->cur = (b->cur + 1) % 3;
            b->stages_run += 3;
        }
    } else {
        for (int n = 0; n < nsteps; ++n) {
            const hipError_t e = enqueue_step_any(b, b->cur, cfl, b->stream);
            if (e != hipSuccess) return bfail(b, GPM_EHIP, std::string("batch step: ") + hipGetErrorString(e));
            b->cur = (b->cur + 1) % 3;
            b->stages_run += 3;
        }
    }
    for (gpm_ctx *c : b->ctx) c->cur = b->cur;
    return GPM_OK;
}

gpm_status gpm_batch_status(gpm_batch *b, int *mood_iters, double *dt)
{
    if (!b) return GPM_EINVAL;
    if (!b->mem) return bfail(b, GPM_ESTATE, "not bound");
    const hipError_t e = launch_batch_status(b->casc, b->nprob, b->st_iters, b->st_dt, b->stream);
    if (e != hipSuccess) return bfail(b, GPM_EHIP, hipGetErrorString(e));
    std::vector<int> it(b->nprob);
    std::vector<double> d(b->nprob);
    BHIPCHK(b, hipMemcpyAsync(it.data(), b->st_iters, sizeof(int) * b->nprob, hipMemcpyDeviceToHost, b->stream));
    BHIPCHK(b, hipMemcpyAsync(d.data(), b->st_dt, sizeof(double) * b->nprob, hipMemcpyDeviceToHost, b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    bool over = false;
    for (int p = 0; p < b->nprob; ++p) {
        if (mood_iters) mood_iters[p] = it[p];
        if (dt) dt[p] = d[p];
        over = over || it[p] == 0;
        b->ctx[p]->last_npass = it[p] > 0 ? it[p] - 1 : kMaxPasses - 1;
    }
    return over ? bfail(b, GPM_ENOTCONV, "a problem's MOOD loop exceeded the pass limit") : GPM_OK;
}

gpm_status gpm_batch_troubled_counts(gpm_batch *b, int p, long long counts[4], int *mood_iters)
{
    if (!b || p < 0 || p >= b->nprob) return GPM_EINVAL;
    std::vector<int> it(b->nprob);
    const gpm_status s0 = gpm_batch_status(b, it.data(), nullptr);
    if (s0 != GPM_OK && s0 != GPM_ENOTCONV) return s0;
    gpm_ctx *c = b->ctx[p];
    const gpm_status st = gpm_troubled_counts(c, counts, nullptr);
    if (st != GPM_OK) return bfail(b, st, c->err);
    if (mood_iters) *mood_iters = it[p];
    return GPM_OK;
}

gpm_status gpm_batch_get_order_mask(gpm_batch *b, int p, unsigned char *mask)
{
    if (!b || p < 0 || p >= b->nprob) return GPM_EINVAL;
    const gpm_status st = gpm_get_order_mask(b->ctx[p], mask);
    return st == GPM_OK ? st : bfail(b, st, b->ctx[p]->err);
}

}  // extern "C"
