/*
 * gpmood.h -- C ABI of the MI355X (gfx950) GP-MOOD stage engine.
 *
 * The library advances cell averages of the 2D compressible Euler equations
 * (Bourgeois & Lee, "GP-MOOD", Sec. "Governing equations", eq. (euler_eqn);
 * ideal gas, p = (gamma-1)(E - |m|^2/(2 rho))) on a uniform Cartesian grid with
 * the GP-MOOD finite-volume method: (2R+1)th-order GP reconstruction
 * (eq. (gp_reconstructor)) at the Gauss nodes of Table tab:QR-pt-weight, HLLC
 * fluxes, the a-posteriori MOOD loop (Sec. "Stepwise implementation", Steps 3-10)
 * with EDP_1 face orders, and SSP-RK3 (eq. (rk3)).
 *
 * Conventions for every entry point:
 *  - Return a gpm_status; no C++ exception crosses the ABI.  gpm_strerror()
 *    gives a message, including the HIP error text for GPM_EHIP.
 *  - Device buffers are owned by the caller and bound with gpm_bind(); the
 *    library never allocates or frees device memory.  Host arrays are owned by
 *    the caller and only read or written during the call.
 *  - Work is queued on the HIP stream given to gpm_create() (NULL: the null
 *    stream) and is asynchronous, except for the calls documented as
 *    synchronising (they wait for the stream).
 *  - Layout of a state: structure of arrays, double or float as chosen at
 *    creation, [var][j][i] with i (x) fastest, var = rho, rho*u, rho*v, E;
 *    nx*ny interior cells, no ghost cells (boundary conditions are applied
 *    by index remapping inside the kernels).
 *  - A context is not thread-safe; separate contexts are independent.
 *  - Physically inadmissible states (negative density or pressure, NaN, Inf)
 *    are not errors: they are what the MOOD detection handles.
 */
#ifndef GPMOOD_H
#define GPMOOD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gpm_ctx gpm_ctx;

typedef enum {
    GPM_OK = 0,
    GPM_EINVAL = 1,      /* bad argument: null pointer, size, radius, cascade, ell, gamma */
    GPM_ENOMEM = 2,      /* host allocation failed */
    GPM_EHIP = 3,        /* a HIP runtime call failed (message kept) */
    GPM_ESTATE = 4,      /* call out of order (no scheme, nothing bound) */
    GPM_ENOTCONV = 5,    /* the MOOD loop exceeded its pass limit (cannot happen for a
                            terminating cascade; reported rather than looping forever) */
    GPM_EUNSUPPORTED = 6 /* configuration not built (e.g. dim != 2) */
} gpm_status;

typedef enum { GPM_F32 = 0, GPM_F64 = 1 } gpm_prec;
typedef enum { GPM_BC_PERIODIC = 0, GPM_BC_OUTFLOW = 1, GPM_BC_REFLECT = 2 } gpm_bc;

/* Grid: n[d] cells on [lo[d], hi[d]], one boundary condition per axis
   (periodic wraps, outflow copies the nearest interior cell: zero gradient,
   reflect is a slip wall: the ghost cell k past the wall is the image of the k-th
   interior cell with its momentum normal to the wall reversed: the four walls of
   Sec. "The implosion problem in 2D"; 2D stages only, not gpm3_* nor
   gpm_stage_vjp).  An inflow slit (the injection of the Mach-jet problems,
   Sec. "Numerical results") on an outflow y axis gives the ghost cells below
   (bit 0) / above (bit 1) the slit's cells the injected state; the CFL step then
   also bounds that state's waves.  2D single problems only (not gpm3_*,
   gpm_batch_* nor gpm_stage_vjp): GPM_EUNSUPPORTED there. */
typedef struct {
    int dim;        /* 2 */
    int n[3];       /* nx, ny (n[2] ignored in 2D) */
    double lo[3], hi[3];
    int bc[3];      /* gpm_bc per axis */
    double gamma;   /* ratio of specific heats, > 1 (paper: 1.4) */
    int slit;       /* inflow slit on the y boundaries: 0 none, bit 0 bottom, bit 1 top */
    double slit_x[2];     /* it covers the cells whose centres lie in [slit_x[0], slit_x[1]] */
    double slit_prim[4];  /* the injected state (rho, u, v, p), rho > 0, p > 0 (bottom side) */
    double slit_prim_top[4];  /* the same for the top side (bit 1) */
} gpm_grid;

/* Detection switches (gpm_scheme.flags); GPM_FLAGS_ALL is the paper's method. */
enum {
    GPM_CSD = 1u,      /* compressibility-shock early accept, eqs. (divV), (gradP) */
    GPM_PLATEAU = 2u,  /* plateau relaxation, eq. (plateau) */
    GPM_U2 = 4u,       /* u2 relaxation with GP-R1 curvature, eqs. (u2_a), (u2_b), App. B */
    GPM_RSCAD = 8u,    /* CAD on the cell's reconstructed Riemann states (Sec. CAD) */
    GPM_FLAGS_ALL = 15u
};

/* Scheme: the order cascade as GP radii, strictly decreasing and ending at 0
   (FOG, the safe scheme), e.g. {3,2,1,0} (7->5->3->1) or the paper's GP-MOOD7
   {3,1,0} (Sec. "The scheme cascade with GP"); radius R uses the (R+1)-point
   Gauss rule.  ell is the physical GP length scale (Sec. "Basic theory on GP
   regression": ell = 6 or 12 min(dx, dy) by default; 0 selects 12 min(dx,dy)). */
typedef struct {
    int nlev;
    int radius[4];
    double ell;
    double sigma_v, sigma_p; /* CSD thresholds (paper: 5, 5) */
    unsigned flags;          /* GPM_* detection switches */
    int stencil;             /* GPM_STENCIL_*; 2D only (the 3D engine takes DIAMOND) */
    int solver;              /* GPM_SOLVER_*; 2D stages only (3D and the stage adjoint take HLLC) */
} gpm_scheme;

/* Riemann solver (gpm_scheme.solver): HLLC, the paper's default, or HLL, the
   solver of its Mach-jet problems (Sec. "Numerical results"), with HLLC's wave
   speed bounds. */
enum { GPM_SOLVER_HLLC = 0, GPM_SOLVER_HLL = 1 };

/* Stencil of the GP levels (gpm_scheme.stencil): the blocky diamond (Sec. "The GP
   stencil"); the cross-shaped stencils of the convergence study (Sec. "Isentropic
   vortex": the diamond's cells on the axes, 5 / 9 / 13 cells); POL-MOOD3 (Sec.
   "POL-MOOD3": radius 1 with the polynomial weights of eqs. (poly3),
   (p3_coeffs); cascade {1, 0} only). */
enum { GPM_STENCIL_DIAMOND = 0, GPM_STENCIL_CROSS = 1, GPM_STENCIL_POLY3 = 2 };

/* Create a context for a grid, a precision and a HIP stream (hipStream_t, may be
   NULL).  Allocates host memory only.  Errors: GPM_EINVAL (bad grid, gamma <= 1,
   n < 1 or > 32768 per axis), GPM_EUNSUPPORTED (dim != 2 (3D: gpm3_create), or
   a periodic or reflecting axis with fewer than 4 cells: the radius-3 stencil
   reaches 4 cells past a face). */
gpm_status gpm_create(const gpm_grid *grid, int prec, void *hip_stream, gpm_ctx **out);

/* Set the cascade, ell, CSD thresholds and flags.  Builds the GP prediction
   vectors on the host in quadruple precision (eqs. (SE-pred), (SE-cov),
   (gp_reconstructor), (normalized_z) with the signed-sum normalisation; Cholesky
   of C as in Sec. "Singularity of the covariance kernel matrix") and the GP-R1
   second-derivative weights of App. B, then rounds them to the context's
   precision.  When memory is bound the call copies the cascade's weight table
   into the workspace and synchronises the stream.  Errors: GPM_EINVAL for a
   cascade that is not strictly decreasing,
   does not end at 0, has a radius outside 0..3 or more than 4 levels, ell < 0, or
   a covariance matrix that is not numerically positive definite. */
gpm_status gpm_set_scheme(gpm_ctx *ctx, const gpm_scheme *scheme);

/* Bytes the caller must provide: state_bytes for three state slots (each
   4*nx*ny elements of the context's precision), work_bytes for the workspace
   (orders, face fluxes, troubled lists, counters, reduction partials, the
   cascade's weight table).  Either pointer may be NULL. */
gpm_status gpm_workspace_size(const gpm_ctx *ctx, size_t *state_bytes, size_t *work_bytes);

/* Bind caller-owned device memory: `state` (>= state_bytes, 256-byte aligned)
   and `work` (>= work_bytes, 256-byte aligned).  Slot 0 is the current state
   after gpm_init_state(); gpm_step() rotates the slots.  Clears the workspace
   (and, with a scheme set, writes its weight table); synchronising.  Errors:
   GPM_EINVAL for a NULL or misaligned pointer. */
gpm_status gpm_bind(gpm_ctx *ctx, void *state, void *work);

/* Device address of state slot `slot` (0..2) and the slot that holds the
   current solution (for zero-copy views).  Errors: GPM_ESTATE if not bound. */
gpm_status gpm_state_ptr(const gpm_ctx *ctx, int slot, void **ptr, int *current_slot);

/* Copy interior cell averages from the host (double, SoA [4][ny][nx]) into the
   current state, converting to the context's precision.  Synchronising. */
gpm_status gpm_init_state(gpm_ctx *ctx, const double *U_host);

/* Copy the current state to the host as double (SoA).  Synchronising. */
gpm_status gpm_get_state(gpm_ctx *ctx, double *U_host);

/* CFL time step from the current state (read as U^n): dt = cfl * min over cells
   and axes of Delta_d / (|u_d| + c) in FP64 (reading of the paper's CFL
   condition, Sec. "Numerical stability"); cells without a sound speed (rho or p
   not positive and finite) are skipped.  The result stays on the device for the
   next stages; if dt_host is non-NULL the call synchronises and returns it. */
gpm_status gpm_compute_dt(gpm_ctx *ctx, double cfl, double *dt_host);

/* The same from a caller device state U (SoA [4][ny][nx], context precision). */
gpm_status gpm_compute_dt_dev(gpm_ctx *ctx, const void *U, double cfl, double *dt_host);

/* Set the device dt directly (for replays and fixed-step runs). */
gpm_status gpm_set_dt(gpm_ctx *ctx, double dt);

/* One SSP-RK3 stage s (0, 1, 2) of eq. (rk3) on caller device buffers:
   U_out = combine_s(U_n, U_s - dt F(U_s)), with the MOOD loop run to completion
   on the candidate U_s - dt F(U_s).  U_n, U_s, U_out hold 4*nx*ny elements of the
   context's precision; U_out must not alias U_s (U_n may alias U_s when s = 0).
   Synchronises once per batch of cascade passes to test for termination.
   Errors: GPM_ESTATE (no scheme or not bound), GPM_EINVAL (s, pointers),
   GPM_ENOTCONV (pass limit). */
gpm_status gpm_stage_dev(gpm_ctx *ctx, int s, const void *U_n, const void *U_s, void *U_out);

/* A general stage of an explicit SSP-RK method in Shu-Osher form (Sec. "Time
   integration": every sub-step of the five-stage SSP-RK4, eq. (rk4_substeps),
   and its last combination, eq. (rk4), take this form):
       U_out = a B + b U*,   U* = U_s - (cf dt) F(U_s),
   with the MOOD loop run to completion on U* (the same detection and cascade as
   gpm_stage_dev); dt is the context's device dt (gpm_set_dt, gpm_compute_dt*).
   B, U_s, U_out: device buffers of 4*nx*ny elements of the context's precision;
   B is not read when a = 0 and may then be NULL; U_out must not alias U_s.
   Errors: GPM_ESTATE, GPM_EINVAL (pointers, cf <= 0, non-finite a, b or cf),
   GPM_ENOTCONV. */
gpm_status gpm_stage_coef(gpm_ctx *ctx, const void *B, const void *U_s, void *U_out, double a, double b,
                          double cf);

/* out = w0 X0 + w1 X1 + w2 X2 + w3 X3 on device buffers of 4*nx*ny elements of
   the context's precision, element by element, evaluated left to right (the
   state combination W of the last SSP-RK4 stage).  out may alias an input. */
gpm_status gpm_lincomb4(gpm_ctx *ctx, void *out, const void *X0, double w0, const void *X1, double w1,
                        const void *X2, double w2, const void *X3, double w3);

/* nsteps full steps on the bound slots: dt from the current state (cfl > 0) or
   the device dt set by gpm_set_dt (cfl <= 0), then stages 0, 1, 2. */
gpm_status gpm_step(gpm_ctx *ctx, double cfl, int nsteps);

/* Statistics of the last stage: counts[l] = cells whose final scheme is
   cascade level l (the paper's per-step troubled-cell fractions), mood_iters =
   number of candidate evaluations (1 + cascade passes).  Synchronising. */
gpm_status gpm_troubled_counts(gpm_ctx *ctx, long long counts[4], int *mood_iters);

/* Final per-cell GP radius of the last stage (uint8 [ny][nx]).  Synchronising. */
gpm_status gpm_get_order_mask(gpm_ctx *ctx, unsigned char *order_host);

/* Conserved totals sum(U) * dx * dy of the current state, per variable, with a
   compensated (double-double) reduction in a fixed order.  Synchronising. */
gpm_status gpm_totals(gpm_ctx *ctx, double totals[4]);

/* Totals of an arbitrary device state (same layout as a slot).  Synchronising. */
gpm_status gpm_totals_dev(gpm_ctx *ctx, const void *U, double totals[4]);

/* gpm_totals_dev for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid allocation): the same
   kernels and the same result, bit for bit, but its partial sums live in a static
   device array of the library (64 KiB + 32 B per GPU, held until the process
   ends) instead of the bound workspace, so the context need not be bound.  The
   grid may be any size the context allows (the partials are capped at 1024
   blocks, which stride over larger grids).  It calls no hipMalloc or hipFree.
   The array is shared by every call on one GPU: calls that overlap on one GPU
   (from several threads or streams) race and must be serialised by the caller.
   The calling thread's current device must be the device of the context's
   stream and of U.  Synchronising.  Errors: GPM_EINVAL (NULL argument),
   GPM_EHIP (the array's device address could not be found), GPM_EUNSUPPORTED (a
   device index of 64 or more). */
gpm_status gpm_totals_static(gpm_ctx *ctx, const void *U, double totals[4]);

/* Tunables.  The cascade of a stage is queued as a batch of multi-block passes
   followed by a single-workgroup kernel that finishes it once a pass leaves at
   most tail_threshold troubled cells (0..4096; it hands back to a new batch if a
   pass leaves more than 4 x tail_threshold), with one host check per batch.
   passes_per_check (1..128) is the smallest batch; the batch otherwise follows
   the previous stage's number of multi-block passes.  rows_per_wave (4..256):
   rows per wavefront march in the first pass.  Defaults 4, 12 (24 in FP64 when
   the grid has at least 2048 marches of 24 rows) and 32. */
gpm_status gpm_set_tuning(gpm_ctx *ctx, int passes_per_check, int rows_per_wave, int tail_threshold);

/* Instrumentation for measurement (not part of the method).  mode bit 0: every
   first-pass launch and every stage's cascade are bracketed by HIP events on the
   context stream and MOOD iterations are counted on the host (no extra kernels);
   bit 1 (implies bit 0): the final-order counts per cascade level are also
   accumulated on the device (two small kernels per stage).  0 disables; a
   non-zero mode resets the accumulators.  Errors: GPM_EINVAL for a mode outside
   0..3. */
gpm_status gpm_instrument(gpm_ctx *ctx, int mode);

/* Read the accumulators (synchronising): first-pass time and launches, cascade
   time (from the end of the first pass to the end of the stage) and stages,
   summed final-order counts per level (mode bit 1 only, else zeros) and summed
   MOOD iterations. */
gpm_status gpm_instrument_read(gpm_ctx *ctx, double *first_pass_ms, long long *first_pass_launches,
                               double *cascade_ms, long long *stages, long long level_cells[4],
                               long long *mood_iters);

/* Where the last stage's cascade passes ran (measurement, not part of the
   method): stats[0] = passes run by multi-block kernels, stats[1] = passes run by
   the single-workgroup tail, stats[2] = hand-backs from the tail to new batches of
   multi-block passes.  stats[0] + stats[1] + 1 is the number of MOOD evaluations.
   Not synchronising (host counters, complete once a stage call has returned). */
gpm_status gpm_cascade_stats(const gpm_ctx *ctx, long long stats[3]);

/* Device address of the context's per-cell order array (uint8 [ny][nx], the GP
   radius of every cell; after a stage, its final orders).  Errors: GPM_ESTATE if
   not bound. */
gpm_status gpm_order_ptr(const gpm_ctx *ctx, void **order_dev);

/* Bytes of the device workspace the stage adjoint needs (gpm_stage_vjp), bound
   separately so that a context used only forward does not carry it: one record
   per face, the adjoints of both sides' reconstruction accumulators, 2 x 64 x
   (nx+1) x (ny+1) values of the context's precision, the FP64 derivative of the
   weight table with respect to ell, and one FP64 dL/d(ell) partial per 16 x 16
   tile of cells. */
gpm_status gpm_adjoint_workspace_size(const gpm_ctx *ctx, size_t *bytes);

/* Bind caller-owned device memory (>= gpm_adjoint_workspace_size, 256-byte
   aligned) as the adjoint workspace and write its weight table (synchronising;
   gpm_set_scheme rewrites it).  Errors: GPM_EINVAL for NULL or misalignment. */
gpm_status gpm_bind_adjoint(gpm_ctx *ctx, void *adj_work);

/* Adjoint of one stage (vector-Jacobian product) with the forward stage's final
   cell orders and its dt held fixed: the stage is then the smooth map of eq.
   (fvm_discrete) with eq. (fvm_F) and eq. (gp_reconstructor) at each face's
   EDP_1 radius and the combination of eq. (rk3); HLLC is differentiated on the
   branch the forward took.  Inputs (device, the context's precision, SoA
   [4][ny][nx]): the stage's Un and Us (Un ignored for s = 0, where Un = Us), its
   final orders `order` (uint8 [ny][nx], e.g. a copy of gpm_order_ptr's array
   taken right after the forward stage), dt, and lam_out = dL/dU_out.  Outputs:
   lam_Us = dL/dU_s (overwritten); for s > 0, lam_Un += dL/dU^n; for s = 0 a
   non-NULL lam_Un (the adjoint of U^n gathered from stages 1 and 2) is added to
   lam_Us, which then holds the total dL/dU^n of the step.  If dL_dell is
   non-NULL, the stage's contribution to dL/d(ell) (ell the physical GP length
   scale; through the ell-dependence of the reconstruction weights only, the
   detection being frozen) is added to *dL_dell (synchronising).  Deterministic:
   every face writes its record into the adjoint workspace (no atomics), and each
   cell sums the contributions of the faces whose stencils hold it in a fixed
   order, so repeated calls give the same bits.  Errors: GPM_EINVAL (bad stage, NULL or
   aliased buffers, dt <= 0), GPM_ESTATE (no adjoint workspace bound),
   GPM_EUNSUPPORTED (a reflecting axis, HLL, a slit). */
gpm_status gpm_stage_vjp(gpm_ctx *ctx, int s, const void *Un, const void *Us, const void *order, double dt,
                         const void *lam_out, void *lam_Us, void *lam_Un, double *dL_dell);

/* gpm_stage_vjp without a host round trip: the stage's dL/d(ell) contribution is
   added, in stream order, to the FP64 value at device address dl_dev (8-byte
   aligned, caller-owned, read back when the caller chooses), so that a backward
   sweep of many stages never synchronises.  Same inputs, outputs and errors as
   gpm_stage_vjp, plus GPM_EINVAL for a NULL or misaligned dl_dev. */
gpm_status gpm_stage_vjp_acc(gpm_ctx *ctx, int s, const void *Un, const void *Us, const void *order, double dt,
                             const void *lam_out, void *lam_Us, void *lam_Un, void *dl_dev);

/* ---------------------------------------------------------------------------
   Batched ensemble: many independent problems of uneven size advanced
   together.  Each problem is a 2D grid of its own size and boundary conditions;
   all share one scheme and precision.  A step advances every problem by one
   SSP-RK3 step with its own CFL time step (Sec. "Numerical stability and
   performance comparison"), using for each kernel kind one launch for the whole
   batch: the dt reduction, the first pass over all problems' strips, and one
   workgroup per problem that runs that problem's complete MOOD cascade (Sec.
   "Stepwise implementation", Steps 3-10).  Results per problem are those of a
   single-problem context.  Not thread-safe per batch. */
typedef struct gpm_batch gpm_batch;

/* Create a batch of nprob problems (grids[p] as for gpm_create; same precision
   and stream for all).  Allocates host memory only.  Errors as gpm_create, for
   the first problem that fails. */
gpm_status gpm_batch_create(int nprob, const gpm_grid *grids, int prec, void *hip_stream, gpm_batch **out);

/* One scheme for every problem (as gpm_set_scheme; ell = 0 selects 12 min(dx,dy)
   per problem).  Problems whose ell/dx and ell/dy agree share one weight build. */
gpm_status gpm_batch_set_scheme(gpm_batch *b, const gpm_scheme *scheme);

/* Bytes of the single device buffer the batch needs (all problems' state slots
   and workspaces plus the batch tables). */
gpm_status gpm_batch_workspace_size(const gpm_batch *b, size_t *bytes);

/* Bind the caller's device buffer (>= the size above, 256-byte aligned);
   clears it.  Synchronising.  Errors: GPM_EINVAL for NULL or misalignment. */
gpm_status gpm_batch_bind(gpm_batch *b, void *mem);

/* First-pass rows per wavefront for every problem (4..256, default 12). */
gpm_status gpm_batch_set_tuning(gpm_batch *b, int rows_per_wave);

/* First-pass rows per wavefront of each problem (nprob values, 4..256). */
gpm_status gpm_batch_set_tuning_per_problem(gpm_batch *b, const int *rows_per_wave);

/* Autotune the first pass's march length (rows per wavefront) per size class of
   problem (problems whose cell counts share a power of two): one sweep of
   coordinate descent over 4, 6, 8, 12, 16, 24, 32 and 64 rows, the classes with the
   most cells first, each candidate timed on the device with HIP events over reps
   (1..64) launches of the batch's stage-0 first pass, with the dt of the current
   states at this CFL.  Stage 0 reads the current state slot and writes another,
   so the problems' states are left as they were.  The choice is kept (as
   gpm_batch_set_tuning_per_problem) and returned in rows_out (nprob values,
   nullable); gain (nullable) receives the first-pass time of the default march
   length over the chosen ones.  The march length changes the schedule only:
   every result is the same bits whatever the choice.  Synchronising.  Errors:
   GPM_EINVAL, GPM_ESTATE (not bound or no scheme), GPM_EHIP. */
gpm_status gpm_batch_autotune(gpm_batch *b, double cfl, int reps, int *rows_out, double *gain);

/* The batch's cascade threshold (the troubled-cell count at or below which a
   problem's MOOD loop leaves the batch-wide multi-block passes for its own tail
   workgroup; default 32), chosen on the device among 8, 16, 32, 64, 128 and 256
   by timing whole stage-0 stages (first pass and cascade, reps timed launches
   each after one untimed) at the current states' dt; the states are left as they
   were, and the threshold changes the schedule only (every stage gives the same
   bits).  tail_out: the choice (applied to the batch); gain: time at the
   threshold in force before the call over time at the choice.  Errors as
   gpm_batch_autotune. */
gpm_status gpm_batch_autotune_cascade(gpm_batch *b, double cfl, int reps, int *tail_out, double *gain);

/* Initial state / current state of problem p (host double SoA [4][ny_p][nx_p]).
   Synchronising. */
gpm_status gpm_batch_init_state(gpm_batch *b, int p, const double *U_host);
gpm_status gpm_batch_get_state(gpm_batch *b, int p, double *U_host);

/* Advance every problem by nsteps SSP-RK3 steps at the given CFL number.  With
   use_graph != 0 each step is one replay of a captured HIP graph (captured on
   first use and again when cfl changes).  Asynchronous; pass-limit overflows are
   reported by gpm_batch_status.  Errors: GPM_EINVAL (cfl <= 0), GPM_ESTATE. */
gpm_status gpm_batch_step(gpm_batch *b, double cfl, int nsteps, int use_graph);

/* Per problem (arrays of nprob, either may be NULL): MOOD evaluations of the
   last stage and the last dt.  Synchronising.  GPM_ENOTCONV if some problem's
   cascade hit the pass limit (its entry in mood_iters is 0). */
gpm_status gpm_batch_status(gpm_batch *b, int *mood_iters, double *dt);

/* Final-order counts per cascade level and evaluations of problem p's last
   stage, and its order mask (as gpm_troubled_counts, gpm_get_order_mask). */
gpm_status gpm_batch_troubled_counts(gpm_batch *b, int p, long long counts[4], int *mood_iters);
gpm_status gpm_batch_get_order_mask(gpm_batch *b, int p, unsigned char *mask_host);

const char *gpm_batch_last_error(const gpm_batch *b);
void gpm_batch_destroy(gpm_batch *b);

/* ---------------------------------------------------------------------------
   3D stage (five variables rho, rho u, rho v, rho w, E; SoA [5][nz][ny][nx]).
   The 3D form of the method: GP stencil of radius R <= 2 on the L1 ball
   (|di|+|dj|+|dk| <= R: 7 / 25 cells), q x q tensor Gauss nodes per face (q = R+1),
   EDP_1 face orders, HLLC with two tangential momenta, detection over the six
   face neighbours (DMP eq. (DMP_RK), plateau eq. (plateau), CSD eqs. (divV),
   (gradP) with the z terms, u2 eqs. (u2_a), (u2_b) per direction with GP-R1
   second derivatives), SSP-RK3 eq. (rk3), FP64 dt = CFL min Delta_d/(|u_d|+c).
   The calls mirror the 2D ones; grid.dim must be 3, n <= 4096 per axis,
   periodic axes need >= 3 cells, reflecting walls are not built (GPM_EUNSUPPORTED),
   cascades use radii 2, 1, 0 (GP-MOOD5 = {2,1,0}).
   Not thread-safe per context. */
typedef struct gpm3_ctx gpm3_ctx;
gpm_status gpm3_create(const gpm_grid *grid, int prec, void *hip_stream, gpm3_ctx **out);
gpm_status gpm3_set_scheme(gpm3_ctx *ctx, const gpm_scheme *scheme);
gpm_status gpm3_workspace_size(const gpm3_ctx *ctx, size_t *state_bytes, size_t *work_bytes);
gpm_status gpm3_bind(gpm3_ctx *ctx, void *state, void *work);
gpm_status gpm3_init_state(gpm3_ctx *ctx, const double *U_host);
gpm_status gpm3_get_state(gpm3_ctx *ctx, double *U_host);
/* dt from the current state (synchronising if dt_host != NULL). */
gpm_status gpm3_compute_dt(gpm3_ctx *ctx, double cfl, double *dt_host);
/* nsteps SSP-RK3 steps, each with its own CFL dt (cfl > 0). */
gpm_status gpm3_step(gpm3_ctx *ctx, double cfl, int nsteps);
/* Final-order counts per cascade level and evaluations of the last stage. */
gpm_status gpm3_troubled_counts(gpm3_ctx *ctx, long long counts[3], int *mood_iters);
gpm_status gpm3_get_order_mask(gpm3_ctx *ctx, unsigned char *mask_host);
/* Compensated FP64 totals of the five variables times the cell volume. */
gpm_status gpm3_totals(gpm3_ctx *ctx, double totals[5]);
const char *gpm3_last_error(const gpm3_ctx *ctx);
void gpm3_destroy(gpm3_ctx *ctx);

const char *gpm_strerror(gpm_status st);
const char *gpm_last_error(const gpm_ctx *ctx);
void gpm_destroy(gpm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* GPMOOD_H */
