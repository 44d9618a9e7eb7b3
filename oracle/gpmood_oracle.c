/*
 * GP-MOOD oracle: a plain, slow FP64 reference of one SSP-RK3 stage in 2D.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header or table
 * with the product library; its GP weights come from oracle/weights_mp.py.
 *
 * Source: Bourgeois & Lee, "GP-MOOD: a positive-preserving high-order finite
 * volume method for hyperbolic conservation laws".
 *   - Euler equations and ideal-gas EoS: Sec. "Governing equations", eq. (euler_eqn)
 *   - FV update with q-point face quadrature: eq. (fvm_discrete), eq. (fvm_F)
 *   - GP reconstruction z^T q: eq. (gp_reconstructor) (weights are inputs here)
 *   - FOG (R = 0): Sec. "The full set of spatial reconstruction methods"
 *   - PAD eq. (PAD), CAD eq. (CAD) and CAD on Riemann states (Sec. CAD),
 *     DMP eq. (DMP_RK), plateau eq. (plateau), u2 eqs. (u2_curvature, u2_a, u2_b),
 *     CSD eqs. (divV, gradP)
 *   - EDP_1 face order: Sec. "The scheme cascade with GP"
 *   - MOOD loop: Sec. "Stepwise implementation", Steps 3-10
 *   - SSP-RK3: eq. (rk3)
 *   - HLLC: the paper only cites Toro et al. 1994; the textbook form is used
 *     (Davis wave-speed estimates, Toro's star states).
 *
 * Every loop below is the plain definition: each MOOD iteration recomputes every
 * face flux and every candidate from scratch and re-detects every cell.
 * Build with -O2 -ffp-contract=off, no fast-math (NaN/Inf are legitimate values
 * that CAD must see).  OpenMP only splits independent per-face and per-cell loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NV 4
#define GH 4 /* ghost depth: R_max + 1 = 4 for R = 3; u2 needs 2 */

enum { ORC_CSD = 1u, ORC_PLATEAU = 2u, ORC_U2 = 4u, ORC_RSCAD = 8u };

typedef struct {
    int nx, ny;
    double dx, dy;
    int bcx, bcy; /* 0 periodic, 1 outflow (zero gradient), 2 reflecting wall */
    double gamma;
    int nlev;
    int rad[4];         /* cascade radii, strictly decreasing, last one 0 (FOG) */
    int nst[4];         /* stencil size per level */
    const int *off[4];  /* per level: [nst][2] offsets (di, dj) */
    int nq[4];          /* quadrature points per face per level */
    const double *qw[4];/* per level: quadrature weights [nq] */
    const double *z[4]; /* per level: weights [4 faces: x-, x+, y-, y+][nq][nst] */
    const double *w2;   /* [2][5] u2 curvature weights on the R = 1 stencil */
    const int *off1;    /* [5][2] R = 1 stencil offsets matching w2 */
    double sigma_v, sigma_p;
    unsigned flags;
    int solver;         /* Riemann solver: 0 HLLC (the default), 1 HLL */
    int slit;           /* inflow slit on the y boundaries: bit 0 bottom, bit 1 top */
    int slit_i0, slit_i1;   /* its cells: columns slit_i0 <= i < slit_i1 */
    double slit_u[4];   /* the fixed inflow state (conservative), bottom side */
    double slit_u2[4];  /* the same, top side */
} orc_cfg;

/* ---------------------------------------------------------------- helpers */
static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

/* Source cell of index i on an axis of n cells: bc 0 periodic, 1 outflow (zero
   gradient: the edge cell), 2 reflecting (the mirror image across the wall). */
static int src_index(int i, int n, int bc)
{
    if (bc == 0) { int r = i % n; return r < 0 ? r + n : r; }
    if (bc == 2) return i < 0 ? -1 - i : (i >= n ? 2 * n - 1 - i : i);
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

typedef struct { int NX, NY; double *u; } ghosted;

static size_t gidx(const ghosted *g, int v, int i, int j)
{
    return ((size_t)v * g->NY + (size_t)(j + GH)) * g->NX + (size_t)(i + GH);
}

static void fill_ghosted(const orc_cfg *c, const double *U, ghosted *g)
{
    g->NX = c->nx + 2 * GH;
    g->NY = c->ny + 2 * GH;
    g->u = (double *)malloc(sizeof(double) * NV * g->NX * g->NY);
    for (int v = 0; v < NV; ++v)
        for (int j = -GH; j < c->ny + GH; ++j)
            for (int i = -GH; i < c->nx + GH; ++i) {
                int si = src_index(i, c->nx, c->bcx), sj = src_index(j, c->ny, c->bcy);
                /* a reflecting wall mirrors the cell and reverses its normal momentum */
                double sg = 1.0;
                if (v == 1 && c->bcx == 2 && (i < 0 || i >= c->nx)) sg = -sg;
                if (v == 2 && c->bcy == 2 && (j < 0 || j >= c->ny)) sg = -sg;
                g->u[gidx(g, v, i, j)] = sg * U[((size_t)v * c->ny + sj) * c->nx + si];
                /* an inflow slit (the Mach-jet problems of Sec. "Numerical results"):
                   the ghost cells below / above it hold the injected state */
                if (i >= c->slit_i0 && i < c->slit_i1 && (((c->slit & 1) && j < 0) || ((c->slit & 2) && j >= c->ny)))
                    g->u[gidx(g, v, i, j)] = j < 0 ? c->slit_u[v] : c->slit_u2[v];
            }
}

static double pressure(double g, const double *q) /* ideal-gas EoS on conservative variables */
{
    return (g - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}

static int level_of(const orc_cfg *c, int r)
{
    for (int l = 0; l < c->nlev; ++l)
        if (c->rad[l] == r) return l;
    return -1;
}

/* ------------------------------------------------------------------ HLLC */
/* Flux through a face with unit normal along axis `dir` (0: x, 1: y). */
static void hllc(double g, const double *UL, const double *UR, int dir, double *F)
{
    int n = 1 + dir, t = 2 - dir;
    double rl = UL[0], ul = UL[n] / rl, vl = UL[t] / rl, El = UL[3];
    double rr = UR[0], ur = UR[n] / rr, vr = UR[t] / rr, Er = UR[3];
    double pl = (g - 1.0) * (El - 0.5 * rl * (ul * ul + vl * vl));
    double pr = (g - 1.0) * (Er - 0.5 * rr * (ur * ur + vr * vr));
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    double SL = dmin(ul - cl, ur - cr);
    double SR = dmax(ul + cl, ur + cr);
    double Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) /
                (rl * (SL - ul) - rr * (SR - ur));
    double f[4];
    if (SL >= 0.0) {
        f[0] = rl * ul; f[1] = rl * ul * ul + pl; f[2] = rl * ul * vl; f[3] = ul * (El + pl);
    } else if (Ss >= 0.0) {
        double fac = rl * (SL - ul) / (SL - Ss);
        double us[4] = {fac, fac * Ss, fac * vl,
                        fac * (El / rl + (Ss - ul) * (Ss + pl / (rl * (SL - ul))))};
        double uk[4] = {rl, rl * ul, rl * vl, El};
        double fk[4] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, ul * (El + pl)};
        for (int k = 0; k < 4; ++k) f[k] = fk[k] + SL * (us[k] - uk[k]);
    } else if (SR > 0.0) {
        double fac = rr * (SR - ur) / (SR - Ss);
        double us[4] = {fac, fac * Ss, fac * vr,
                        fac * (Er / rr + (Ss - ur) * (Ss + pr / (rr * (SR - ur))))};
        double uk[4] = {rr, rr * ur, rr * vr, Er};
        double fk[4] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, ur * (Er + pr)};
        for (int k = 0; k < 4; ++k) f[k] = fk[k] + SR * (us[k] - uk[k]);
    } else {
        f[0] = rr * ur; f[1] = rr * ur * ur + pr; f[2] = rr * ur * vr; f[3] = ur * (Er + pr);
    }
    /* back from (normal, tangential) to (x, y) momentum components */
    F[0] = f[0]; F[n] = f[1]; F[t] = f[2]; F[3] = f[3];
}

void orc_hllc(double g, const double *UL, const double *UR, int dir, double *F)
{
    hllc(g, UL, UR, dir, F);
}

/* HLL flux (Sec. "Numerical results": the solver of the Mach-jet problems, after
   Harten, Lax and van Leer), with HLLC's wave speed bounds: the left or right
   physical flux outside [S_L, S_R], else the single intermediate state's flux
   (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L). */
static void hll(double g, const double *UL, const double *UR, int dir, double *F)
{
    int n = 1 + dir, t = 2 - dir;
    double rl = UL[0], ul = UL[n] / rl, vl = UL[t] / rl, El = UL[3];
    double rr = UR[0], ur = UR[n] / rr, vr = UR[t] / rr, Er = UR[3];
    double pl = (g - 1.0) * (El - 0.5 * rl * (ul * ul + vl * vl));
    double pr = (g - 1.0) * (Er - 0.5 * rr * (ur * ur + vr * vr));
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    double SL = dmin(ul - cl, ur - cr);
    double SR = dmax(ul + cl, ur + cr);
    double uk[2][4] = {{rl, rl * ul, rl * vl, El}, {rr, rr * ur, rr * vr, Er}};
    double fk[2][4] = {{rl * ul, rl * ul * ul + pl, rl * ul * vl, ul * (El + pl)},
                       {rr * ur, rr * ur * ur + pr, rr * ur * vr, ur * (Er + pr)}};
    double f[4];
    for (int k = 0; k < 4; ++k) {
        if (SL >= 0.0) f[k] = fk[0][k];
        else if (SR <= 0.0) f[k] = fk[1][k];
        else f[k] = (SR * fk[0][k] - SL * fk[1][k] + SL * SR * (uk[1][k] - uk[0][k])) / (SR - SL);
    }
    F[0] = f[0]; F[n] = f[1]; F[t] = f[2]; F[3] = f[3];
}

void orc_hll(double g, const double *UL, const double *UR, int dir, double *F)
{
    hll(g, UL, UR, dir, F);
}

static void riemann(const orc_cfg *c, const double *UL, const double *UR, int dir, double *F)
{
    if (c->solver == 1) hll(c->gamma, UL, UR, dir, F);
    else hllc(c->gamma, UL, UR, dir, F);
}

/* --------------------------------------------------- GP reconstruction */
/* State of cell (i, j) (ghosted indices allowed) at face f, point k, level l. */
static void recon(const orc_cfg *c, const ghosted *g, int l, int f, int k, int i, int j, double *q)
{
    int ns = c->nst[l];
    const double *z = c->z[l] + ((size_t)f * c->nq[l] + k) * ns;
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
        for (int m = 0; m < ns; ++m)
            s += z[m] * g->u[gidx(g, v, i + c->off[l][2 * m], j + c->off[l][2 * m + 1])];
        q[v] = s;
    }
}

/* CAD on a reconstructed Riemann state (Sec. CAD): the state is inadmissible unless
   its density and pressure are finite and positive.  A non-positive value makes the
   sound speed the square root of a negative number, an invalid operation that CAD
   exists to catch, and the solver's wave speeds then order its two states
   arbitrarily, which breaks the symmetry the Riemann-state check is there to keep.
   The flux of such a pair enters the candidates of both cells of the face, so both
   are troubled, whichever side holds the state and whichever solver runs. */
static int state_inadmissible(double gam, const double *q)
{
    double p = pressure(gam, q);
    return !(isfinite(q[0]) && isfinite(p) && q[0] > 0.0 && p > 0.0);
}

/* --------------------------------------------- per-stage relaxation data */
typedef struct { double rmin, rmax; int plat, csd, u2; } relax_t;

static double rho_at(const ghosted *g, int i, int j) { return g->u[gidx(g, 0, i, j)]; }

static void cell_relax(const orc_cfg *c, const ghosted *g, int i, int j, relax_t *r)
{
    double gam = c->gamma;
    /* DMP bounds over N(ij) U {ij}: the four face neighbours and the cell, eq. (DMP_RK) */
    const int nb[5][2] = {{0, 0}, {-1, 0}, {1, 0}, {0, -1}, {0, 1}};
    double lo = rho_at(g, i, j), hi = lo;
    for (int k = 1; k < 5; ++k) {
        double v = rho_at(g, i + nb[k][0], j + nb[k][1]);
        lo = dmin(lo, v);
        hi = dmax(hi, v);
    }
    r->rmin = lo;
    r->rmax = hi;
    /* plateau, eq. (plateau) */
    r->plat = (hi - lo) < dmin(c->dx * c->dx * c->dx, c->dy * c->dy * c->dy);
    /* CSD, eqs. (divV) and (gradP), on the stage's cell averages */
    double qE[4], qW[4], qN[4], qS[4];
    for (int v = 0; v < NV; ++v) {
        qE[v] = g->u[gidx(g, v, i + 1, j)];
        qW[v] = g->u[gidx(g, v, i - 1, j)];
        qN[v] = g->u[gidx(g, v, i, j + 1)];
        qS[v] = g->u[gidx(g, v, i, j - 1)];
    }
    double divV = (qE[1] / qE[0] - qW[1] / qW[0]) / (2.0 * c->dx) +
                  (qN[2] / qN[0] - qS[2] / qS[0]) / (2.0 * c->dy);
    double pE = pressure(gam, qE), pW = pressure(gam, qW);
    double pN = pressure(gam, qN), pS = pressure(gam, qS);
    double gradp = fabs(pE - pW) / (2.0 * c->dx * dmin(pE, pW)) +
                   fabs(pN - pS) / (2.0 * c->dy * dmin(pN, pS));
    r->csd = (divV >= -c->sigma_v) && (gradp <= c->sigma_p);
    /* u2, eqs. (u2_curvature), (u2_a), (u2_b): GP-R1 second derivatives of rho
       at the cell and its face neighbours, per direction */
    double delta = dmin(c->dx, c->dy);
    int ok = 1;
    for (int d = 0; d < 2; ++d) {
        double cmin = 0.0, cmax = 0.0;
        for (int k = 0; k < 5; ++k) {
            int mi = i + nb[k][0], mj = j + nb[k][1];
            double kap = 0.0;
            for (int m = 0; m < 5; ++m)
                kap += c->w2[d * 5 + m] * rho_at(g, mi + c->off1[2 * m], mj + c->off1[2 * m + 1]);
            if (k == 0) { cmin = kap; cmax = kap; }
            else { cmin = dmin(cmin, kap); cmax = dmax(cmax, kap); }
        }
        /* eq. (u2_b)'s ratio |Cmin|/|Cmax| >= 1/2 multiplied through by |Cmax|:
           half of |Cmax| is exact in binary arithmetic, so the comparison decides
           the paper's inequality exactly (a rounded quotient can accept a ratio
           just below 1/2); Cmax = Cmin = 0 is accepted by (a) either way */
        int a = (cmin * cmax > -delta) && (dmax(fabs(cmax), fabs(cmin)) < delta);
        int b = (cmin * cmax > -delta) && (fabs(cmin) >= 0.5 * fabs(cmax));
        ok = ok && (a || b);
    }
    r->u2 = ok;
}

/* Criteria bits of one cell: bit0 CAD(candidate), bit1 RS-CAD ok, bit2 PAD,
   bit3 CSD, bit4 plateau, bit5 DMP, bit6 u2. */
static unsigned criteria(const orc_cfg *c, const relax_t *r, const double *us, int rs_bad)
{
    double rho = us[0], p = pressure(c->gamma, us);
    unsigned b = 0;
    if (isfinite(rho) && isfinite(p)) b |= 1u;
    if (!rs_bad) b |= 2u;
    if (rho > 0.0 && p > 0.0) b |= 4u;
    if (r->csd) b |= 8u;
    if (r->plat) b |= 16u;
    if (r->rmin <= rho && rho <= r->rmax) b |= 32u;
    if (r->u2) b |= 64u;
    return b;
}

/* Steps 4-10 of the stepwise algorithm for one cell; returns 1 if troubled. */
static int detect(const orc_cfg *c, int order, unsigned b)
{
    if (order == 0) return 0;                                   /* Step 10: FOG accepted */
    if (!(b & 1u)) return 1;                                    /* Step 4: CAD */
    if ((c->flags & ORC_RSCAD) && !(b & 2u)) return 1;          /*         CAD on Riemann states */
    if (!(b & 4u)) return 1;                                    /* Step 5: PAD */
    if ((c->flags & ORC_CSD) && (b & 8u)) return 0;             /* Step 6: CSD early accept */
    if ((c->flags & ORC_PLATEAU) && (b & 16u)) return 0;        /* Step 7: plateau */
    if (b & 32u) return 0;                                      /* Step 8: DMP */
    if ((c->flags & ORC_U2) && (b & 64u)) return 0;             /* Step 9: u2 */
    return 1;
}

/* ------------------------------------------------------ candidate update */
/* One evaluation of U* = U_s - dt F_nabla(U_s) with per-cell orders (EDP_1 faces).
   rsbad[cell] receives the Riemann-state CAD flags of each cell's own states. */
static void candidate(const orc_cfg *c, const ghosted *g, const int *order, double dt,
                      double *Ustar, int *rsbad)
{
    int nx = c->nx, ny = c->ny;
    size_t ncell = (size_t)nx * ny;
    double *Fx = (double *)calloc((size_t)NV * (nx + 1) * ny, sizeof(double));
    double *Gy = (double *)calloc((size_t)NV * nx * (ny + 1), sizeof(double));
    unsigned char *rsx = (unsigned char *)calloc((size_t)(nx + 1) * ny, 1);
    unsigned char *rsy = (unsigned char *)calloc((size_t)nx * (ny + 1), 1);
    double gam = c->gamma;

    /* x faces: face i sits between cells (i-1, j) [left] and (i, j) [right] */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            int oL = order[(size_t)j * nx + src_index(i - 1, nx, c->bcx)];
            int oR = order[(size_t)j * nx + src_index(i, nx, c->bcx)];
            int l = level_of(c, oL < oR ? oL : oR); /* EDP_1: min of the two orders */
            double F[4] = {0, 0, 0, 0};
            unsigned char bad = 0;
            for (int k = 0; k < c->nq[l]; ++k) {
                double qL[4], qR[4], f[4];
                recon(c, g, l, 1, k, i - 1, j, qL); /* x+ face of the left cell */
                recon(c, g, l, 0, k, i, j, qR);     /* x- face of the right cell */
                if (state_inadmissible(gam, qL)) bad |= 1;
                if (state_inadmissible(gam, qR)) bad |= 2;
                riemann(c, qL, qR, 0, f);
                for (int v = 0; v < NV; ++v) F[v] += c->qw[l][k] * f[v];
            }
            for (int v = 0; v < NV; ++v) Fx[((size_t)v * ny + j) * (nx + 1) + i] = F[v];
            rsx[(size_t)j * (nx + 1) + i] = bad;
        }
    /* y faces: face j sits between cells (i, j-1) [bottom/left] and (i, j) [top/right] */
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            int oL = order[(size_t)src_index(j - 1, ny, c->bcy) * nx + i];
            int oR = order[(size_t)src_index(j, ny, c->bcy) * nx + i];
            int l = level_of(c, oL < oR ? oL : oR);
            double G[4] = {0, 0, 0, 0};
            unsigned char bad = 0;
            for (int k = 0; k < c->nq[l]; ++k) {
                double qL[4], qR[4], f[4];
                recon(c, g, l, 3, k, i, j - 1, qL); /* y+ face of the lower cell */
                recon(c, g, l, 2, k, i, j, qR);     /* y- face of the upper cell */
                if (state_inadmissible(gam, qL)) bad |= 1;
                if (state_inadmissible(gam, qR)) bad |= 2;
                riemann(c, qL, qR, 1, f);
                for (int v = 0; v < NV; ++v) G[v] += c->qw[l][k] * f[v];
            }
            for (int v = 0; v < NV; ++v) Gy[((size_t)v * (ny + 1) + j) * nx + i] = G[v];
            rsy[(size_t)j * nx + i] = bad;
        }
    /* candidate, eq. (fvm_discrete) with eq. (fvm_F) */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t cidx = (size_t)j * nx + i;
            for (int v = 0; v < NV; ++v) {
                double us = g->u[gidx(g, v, i, j)];
                double dF = Fx[((size_t)v * ny + j) * (nx + 1) + i + 1] - Fx[((size_t)v * ny + j) * (nx + 1) + i];
                double dG = Gy[((size_t)v * (ny + 1) + j + 1) * nx + i] - Gy[((size_t)v * (ny + 1) + j) * nx + i];
                Ustar[(size_t)v * ncell + cidx] = us - dt * (dF / c->dx + dG / c->dy);
            }
            /* an inadmissible state on either side of any of the cell's four faces */
            rsbad[cidx] = rsx[(size_t)j * (nx + 1) + i] != 0 || rsx[(size_t)j * (nx + 1) + i + 1] != 0 ||
                          rsy[(size_t)j * nx + i] != 0 || rsy[(size_t)(j + 1) * nx + i] != 0;
        }
    free(Fx); free(Gy); free(rsx); free(rsy);
}

static void combine(const orc_cfg *c, int s, const double *Un, const double *Ustar, double *Uout)
{
    size_t n = (size_t)NV * c->nx * c->ny;
    for (size_t k = 0; k < n; ++k) {
        if (s == 0) Uout[k] = Ustar[k];                                  /* U^(1) */
        else if (s == 1) Uout[k] = 0.25 * (3.0 * Un[k] + Ustar[k]);      /* hat U^(2) */
        else Uout[k] = (Un[k] + 2.0 * Ustar[k]) / 3.0;                   /* U^(n+1) */
    }
}

/* --------------------------------------------------------------- stage */
/* The MOOD loop of one stage (Sec. "Step-by-step GP-MOOD algorithm"): the
   candidate U* = Us - dt F(Us) at the top order, detection, lowering of the
   troubled cells to the next scheme of the cascade, until no cell is troubled.
   order_out: final radius per cell; counts[l]: cells ending at level l; returns
   the number of MOOD iterations (candidate evaluations). */
static int mood_loop(const orc_cfg *c, const double *Us, double dt, double *Ustar, int *order_out,
                     long long *counts)
{
    int nx = c->nx, ny = c->ny;
    size_t ncell = (size_t)nx * ny;
    ghosted g;
    fill_ghosted(c, Us, &g);
    relax_t *rx = (relax_t *)malloc(sizeof(relax_t) * ncell);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) cell_relax(c, &g, i, j, &rx[(size_t)j * nx + i]);

    int *order = (int *)malloc(sizeof(int) * ncell);
    for (size_t k = 0; k < ncell; ++k) order[k] = c->rad[0]; /* every stage starts at the top order */
    int *rsbad = (int *)malloc(sizeof(int) * ncell);
    int *trouble = (int *)malloc(sizeof(int) * ncell);
    int iters = 0;
    for (;;) {
        ++iters;
        candidate(c, &g, order, dt, Ustar, rsbad);
        long long ntr = 0;
#pragma omp parallel for schedule(static) reduction(+ : ntr)
        for (long long k = 0; k < (long long)ncell; ++k) {
            double us[4];
            for (int v = 0; v < NV; ++v) us[v] = Ustar[(size_t)v * ncell + k];
            trouble[k] = detect(c, order[k], criteria(c, &rx[k], us, rsbad[k]));
            ntr += trouble[k];
        }
        if (ntr == 0) break;
        for (size_t k = 0; k < ncell; ++k)
            if (trouble[k]) order[k] = c->rad[level_of(c, order[k]) + 1]; /* next scheme in the cascade */
    }
    if (counts)
        for (int l = 0; l < c->nlev; ++l) counts[l] = 0;
    for (size_t k = 0; k < ncell; ++k) {
        if (order_out) order_out[k] = order[k];
        if (counts) counts[level_of(c, order[k])]++;
    }
    free(order); free(rsbad); free(trouble); free(rx); free(g.u);
    return iters;
}

/* One SSP-RK3 stage (eq. (rk3)) with the full MOOD loop. */
int orc_stage(const orc_cfg *c, int s, const double *Un, const double *Us, double dt,
              double *Uout, int *order_out, long long *counts)
{
    double *Ustar = (double *)malloc(sizeof(double) * NV * c->nx * c->ny);
    int iters = mood_loop(c, Us, dt, Ustar, order_out, counts);
    combine(c, s, Un, Ustar, Uout);
    free(Ustar);
    return iters;
}

/* A stage of an explicit SSP-RK method in the form
       U_out = a B + b U*,   U* = Us - (cf dt) F(Us),
   with the full MOOD loop on U* (every sub-step of eqs. (rk4_substeps) and the
   last combination of eq. (rk4) can be written so, B being U^n or an already
   formed linear combination).  a = 0 takes U_out = b U*. */
int orc_stage_coef(const orc_cfg *c, const double *B, const double *Us, double dt, double a, double b, double cf,
                   double *Uout, int *order_out, long long *counts)
{
    size_t n = (size_t)NV * c->nx * c->ny;
    double *Ustar = (double *)malloc(sizeof(double) * n);
    int iters = mood_loop(c, Us, cf * dt, Ustar, order_out, counts);
    for (size_t k = 0; k < n; ++k) Uout[k] = (a == 0.0 ? 0.0 : a * B[k]) + b * Ustar[k];
    free(Ustar);
    return iters;
}

/* Stage with prescribed per-cell orders (no detection): "forced-mask" replay. */
void orc_stage_forced(const orc_cfg *c, int s, const double *Un, const double *Us, double dt,
                      const int *order, double *Uout)
{
    size_t ncell = (size_t)c->nx * c->ny;
    ghosted g;
    fill_ghosted(c, Us, &g);
    double *Ustar = (double *)malloc(sizeof(double) * NV * ncell);
    int *rsbad = (int *)malloc(sizeof(int) * ncell);
    candidate(c, &g, order, dt, Ustar, rsbad);
    combine(c, s, Un, Ustar, Uout);
    free(Ustar); free(rsbad); free(g.u);
}

/* Candidate only (U* and the per-cell Riemann-state CAD flags) for given orders. */
void orc_candidate(const orc_cfg *c, const double *Us, double dt, const int *order,
                   double *Ustar, int *rsbad)
{
    ghosted g;
    fill_ghosted(c, Us, &g);
    candidate(c, &g, order, dt, Ustar, rsbad);
    free(g.u);
}

/* Criteria bits (see criteria()) and the verdict for every cell, for a given
   stage input, candidate, orders and Riemann-state flags. */
void orc_criteria(const orc_cfg *c, const double *Us, const double *Ustar, const int *order,
                  const int *rsbad, unsigned *bits, int *troubled)
{
    int nx = c->nx, ny = c->ny;
    size_t ncell = (size_t)nx * ny;
    ghosted g;
    fill_ghosted(c, Us, &g);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = (size_t)j * nx + i;
            relax_t r;
            cell_relax(c, &g, i, j, &r);
            double us[4];
            for (int v = 0; v < NV; ++v) us[v] = Ustar[(size_t)v * ncell + k];
            unsigned b = criteria(c, &r, us, rsbad ? rsbad[k] : 0);
            if (bits) bits[k] = b;
            if (troubled) troubled[k] = detect(c, order[k], b);
        }
    free(g.u);
}

/* Relaxation data of every cell: rmin, rmax and (plateau, csd, u2) as 0/1 doubles. */
void orc_relax(const orc_cfg *c, const double *Us, double *out /* [ncell][5] */)
{
    int nx = c->nx, ny = c->ny;
    ghosted g;
    fill_ghosted(c, Us, &g);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            relax_t r;
            cell_relax(c, &g, i, j, &r);
            double *o = out + 5 * ((size_t)j * nx + i);
            o[0] = r.rmin; o[1] = r.rmax; o[2] = r.plat; o[3] = r.csd; o[4] = r.u2;
        }
    free(g.u);
}

/* ----------------------------------------------------------------- dt */
/* dt = CFL * min over cells and directions of Delta_d / (|u_d| + c), from U^n.
   Cells without a sound speed (rho or p not positive and finite) are skipped. */
double orc_dt(const orc_cfg *c, const double *U, double cfl)
{
    size_t ncell = (size_t)c->nx * c->ny;
    double lam = 0.0;
    for (size_t k = 0; k < ncell; ++k) {
        double q[4];
        for (int v = 0; v < NV; ++v) q[v] = U[(size_t)v * ncell + k];
        double p = pressure(c->gamma, q);
        if (!(q[0] > 0.0 && p > 0.0 && isfinite(q[0]) && isfinite(p))) continue;
        double cs = sqrt(c->gamma * p / q[0]);
        double lx = (fabs(q[1] / q[0]) + cs) / c->dx;
        double ly = (fabs(q[2] / q[0]) + cs) / c->dy;
        lam = dmax(lam, dmax(lx, ly));
    }
    for (int side = 0; side < 2; ++side) {
        if (!(c->slit & (1 << side))) continue;
        /* the injected state enters the domain: its waves bound the step too */
        const double *q = side ? c->slit_u2 : c->slit_u;
        double p = pressure(c->gamma, q);
        double cs = sqrt(c->gamma * p / q[0]);
        lam = dmax(lam, dmax((fabs(q[1] / q[0]) + cs) / c->dx, (fabs(q[2] / q[0]) + cs) / c->dy));
    }
    return cfl / lam;
}

/* --------------------------------------------------------------- step */
/* nsteps SSP-RK3 steps in place.  dts (nullable) receives each step's dt;
   counts (nullable) [nsteps*3][nlev] final-order counts; iters (nullable) [nsteps*3]. */
void orc_run(const orc_cfg *c, double *U, double cfl, double fixed_dt, int nsteps,
             double *dts, long long *counts, int *iters)
{
    size_t n = (size_t)NV * c->nx * c->ny;
    double *U1 = (double *)malloc(sizeof(double) * n);
    double *U2 = (double *)malloc(sizeof(double) * n);
    for (int st = 0; st < nsteps; ++st) {
        double dt = fixed_dt > 0.0 ? fixed_dt : orc_dt(c, U, cfl);
        if (dts) dts[st] = dt;
        long long *cn = counts ? counts + (size_t)st * 3 * c->nlev : 0;
        int a = orc_stage(c, 0, U, U, dt, U1, 0, cn);
        int b = orc_stage(c, 1, U, U1, dt, U2, 0, cn ? cn + c->nlev : 0);
        int d = orc_stage(c, 2, U, U2, dt, U1, 0, cn ? cn + 2 * c->nlev : 0);
        if (iters) { iters[3 * st] = a; iters[3 * st + 1] = b; iters[3 * st + 2] = d; }
        memcpy(U, U1, sizeof(double) * n);
    }
    free(U1); free(U2);
}

/* -------------------------------------------------------------- totals */
/* Neumaier-compensated sum of each conserved variable times the cell area. */
void orc_totals(const orc_cfg *c, const double *U, double *tot)
{
    size_t ncell = (size_t)c->nx * c->ny;
    for (int v = 0; v < NV; ++v) {
        double s = 0.0, comp = 0.0;
        for (size_t k = 0; k < ncell; ++k) {
            double x = U[(size_t)v * ncell + k];
            double t = s + x;
            if (fabs(s) >= fabs(x)) comp += (s - t) + x;
            else comp += (x - t) + s;
            s = t;
        }
        tot[v] = (s + comp) * c->dx * c->dy;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the OpenMP loops from now on (timing only; results do not depend on it). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

/* ============================================================ derivatives
   Derivatives of one stage with the per-cell orders (and dt) held fixed: the
   stage is then the smooth map of eq. (fvm_discrete) with eq. (fvm_F), the linear
   reconstruction of eq. (gp_reconstructor) at each face's EDP_1 level, and the
   combination of eq. (rk3),
       U_out = beta U^n + alpha (U_s - dt (dF/dx + dG/dy)),
   alpha, beta = (1, 0), (1/4, 3/4), (2/3, 1/3) for s = 0, 1, 2.  The Riemann
   solver is differentiated on the branch its values take, with forward-mode dual
   numbers (value, derivative).  orc_stage_jvp is the directional derivative;
   orc_stage_vjp its transpose, written as the reverse sweep of the same loops. */
typedef struct { double v, d; } dual;

static dual dc(double x) { dual r = {x, 0.0}; return r; }
static dual dadd(dual a, dual b) { dual r = {a.v + b.v, a.d + b.d}; return r; }
static dual dsub(dual a, dual b) { dual r = {a.v - b.v, a.d - b.d}; return r; }
static dual dmul(dual a, dual b) { dual r = {a.v * b.v, a.d * b.v + a.v * b.d}; return r; }
static dual ddiv(dual a, dual b)
{
    double q = a.v / b.v;
    dual r = {q, (a.d - q * b.d) / b.v};
    return r;
}
static dual dsqrt(dual a)
{
    double s = sqrt(a.v);
    dual r = {s, a.d / (2.0 * s)};
    return r;
}
static dual dmin2(dual a, dual b) { return a.v < b.v ? a : b; }
static dual dmax2(dual a, dual b) { return a.v > b.v ? a : b; }

/* HLLC of hllc() in dual numbers, the same branches taken on the values. */
static void hllc_d(double g, const dual *UL, const dual *UR, int dir, dual *F)
{
    int n = 1 + dir, t = 2 - dir;
    dual G1 = dc(g - 1.0), half = dc(0.5);
    dual rl = UL[0], ul = ddiv(UL[n], rl), vl = ddiv(UL[t], rl), El = UL[3];
    dual rr = UR[0], ur = ddiv(UR[n], rr), vr = ddiv(UR[t], rr), Er = UR[3];
    dual pl = dmul(G1, dsub(El, dmul(half, dmul(rl, dadd(dmul(ul, ul), dmul(vl, vl))))));
    dual pr = dmul(G1, dsub(Er, dmul(half, dmul(rr, dadd(dmul(ur, ur), dmul(vr, vr))))));
    dual cl = dsqrt(ddiv(dmul(dc(g), pl), rl)), cr = dsqrt(ddiv(dmul(dc(g), pr), rr));
    dual SL = dmin2(dsub(ul, cl), dsub(ur, cr));
    dual SR = dmax2(dadd(ul, cl), dadd(ur, cr));
    dual Ss = ddiv(dsub(dadd(dsub(pr, pl), dmul(dmul(rl, ul), dsub(SL, ul))), dmul(dmul(rr, ur), dsub(SR, ur))),
                   dsub(dmul(rl, dsub(SL, ul)), dmul(rr, dsub(SR, ur))));
    dual f[4];
    if (SL.v >= 0.0) {
        f[0] = dmul(rl, ul); f[1] = dadd(dmul(dmul(rl, ul), ul), pl); f[2] = dmul(dmul(rl, ul), vl);
        f[3] = dmul(ul, dadd(El, pl));
    } else if (Ss.v >= 0.0 || SR.v > 0.0) {
        int left = Ss.v >= 0.0;
        dual rk = left ? rl : rr, uk = left ? ul : ur, vk = left ? vl : vr, Ek = left ? El : Er;
        dual pk = left ? pl : pr, Sk = left ? SL : SR;
        dual fac = ddiv(dmul(rk, dsub(Sk, uk)), dsub(Sk, Ss));
        dual us[4] = {fac, dmul(fac, Ss), dmul(fac, vk),
                      dmul(fac, dadd(ddiv(Ek, rk), dmul(dsub(Ss, uk), dadd(Ss, ddiv(pk, dmul(rk, dsub(Sk, uk)))))))};
        dual uk4[4] = {rk, dmul(rk, uk), dmul(rk, vk), Ek};
        dual fk[4] = {dmul(rk, uk), dadd(dmul(dmul(rk, uk), uk), pk), dmul(dmul(rk, uk), vk), dmul(uk, dadd(Ek, pk))};
        for (int k = 0; k < 4; ++k) f[k] = dadd(fk[k], dmul(Sk, dsub(us[k], uk4[k])));
    } else {
        f[0] = dmul(rr, ur); f[1] = dadd(dmul(dmul(rr, ur), ur), pr); f[2] = dmul(dmul(rr, ur), vr);
        f[3] = dmul(ur, dadd(Er, pr));
    }
    F[0] = f[0]; F[n] = f[1]; F[t] = f[2]; F[3] = f[3];
}

/* HLL of hll() in dual numbers. */
static void hll_d(double g, const dual *UL, const dual *UR, int dir, dual *F)
{
    int n = 1 + dir, t = 2 - dir;
    dual G1 = dc(g - 1.0), half = dc(0.5);
    dual rl = UL[0], ul = ddiv(UL[n], rl), vl = ddiv(UL[t], rl), El = UL[3];
    dual rr = UR[0], ur = ddiv(UR[n], rr), vr = ddiv(UR[t], rr), Er = UR[3];
    dual pl = dmul(G1, dsub(El, dmul(half, dmul(rl, dadd(dmul(ul, ul), dmul(vl, vl))))));
    dual pr = dmul(G1, dsub(Er, dmul(half, dmul(rr, dadd(dmul(ur, ur), dmul(vr, vr))))));
    dual cl = dsqrt(ddiv(dmul(dc(g), pl), rl)), cr = dsqrt(ddiv(dmul(dc(g), pr), rr));
    dual SL = dmin2(dsub(ul, cl), dsub(ur, cr));
    dual SR = dmax2(dadd(ul, cl), dadd(ur, cr));
    dual uk[2][4] = {{rl, dmul(rl, ul), dmul(rl, vl), El}, {rr, dmul(rr, ur), dmul(rr, vr), Er}};
    dual fk[2][4] = {{dmul(rl, ul), dadd(dmul(dmul(rl, ul), ul), pl), dmul(dmul(rl, ul), vl), dmul(ul, dadd(El, pl))},
                     {dmul(rr, ur), dadd(dmul(dmul(rr, ur), ur), pr), dmul(dmul(rr, ur), vr), dmul(ur, dadd(Er, pr))}};
    dual f[4];
    for (int k = 0; k < 4; ++k) {
        if (SL.v >= 0.0) f[k] = fk[0][k];
        else if (SR.v <= 0.0) f[k] = fk[1][k];
        else f[k] = ddiv(dadd(dsub(dmul(SR, fk[0][k]), dmul(SL, fk[1][k])), dmul(dmul(SL, SR), dsub(uk[1][k], uk[0][k]))),
                         dsub(SR, SL));
    }
    F[0] = f[0]; F[n] = f[1]; F[t] = f[2]; F[3] = f[3];
}

static void riemann_d(const orc_cfg *c, const dual *UL, const dual *UR, int dir, dual *F)
{
    if (c->solver == 1) hll_d(c->gamma, UL, UR, dir, F);
    else hllc_d(c->gamma, UL, UR, dir, F);
}

static void stage_alpha_beta(int s, double *alpha, double *beta)
{
    *alpha = s == 0 ? 1.0 : (s == 1 ? 0.25 : 2.0 / 3.0);
    *beta = s == 0 ? 0.0 : (s == 1 ? 0.75 : 1.0 / 3.0);
}

/* Derivative of ghosted cell (i, j) (ghost indices allowed) with respect to the
   interior cell it copies: its source cell and the factor (-1 for the normal
   momentum mirrored by a reflecting wall, 0 for the fixed state of an inflow slit). */
static size_t ghost_source(const orc_cfg *c, int v, int i, int j, double *factor)
{
    int si = src_index(i, c->nx, c->bcx), sj = src_index(j, c->ny, c->bcy);
    double sg = 1.0;
    if (v == 1 && c->bcx == 2 && (i < 0 || i >= c->nx)) sg = -sg;
    if (v == 2 && c->bcy == 2 && (j < 0 || j >= c->ny)) sg = -sg;
    if (i >= c->slit_i0 && i < c->slit_i1 && (((c->slit & 1) && j < 0) || ((c->slit & 2) && j >= c->ny))) sg = 0.0;
    *factor = sg;
    return ((size_t)v * c->ny + sj) * c->nx + si;
}

/* The flux of one face (direction dir, between ghosted cells (iL, jL) and its
   neighbour along dir) in dual numbers: tangent dU (interior layout) along U_s. */
static void face_flux_d(const orc_cfg *c, const ghosted *g, const double *dU, int l, int dir, int iL, int jL,
                        dual *Fout)
{
    int iR = iL + (dir == 0), jR = jL + (dir == 1);
    int fL = dir == 0 ? 1 : 3, fR = dir == 0 ? 0 : 2; /* + face of the left cell, - face of the right one */
    for (int v = 0; v < NV; ++v) Fout[v] = dc(0.0);
    for (int k = 0; k < c->nq[l]; ++k) {
        dual qL[4], qR[4], f[4];
        int ns = c->nst[l];
        const double *zL = c->z[l] + ((size_t)fL * c->nq[l] + k) * ns;
        const double *zR = c->z[l] + ((size_t)fR * c->nq[l] + k) * ns;
        for (int v = 0; v < NV; ++v) {
            dual sl = dc(0.0), sr = dc(0.0);
            for (int m = 0; m < ns; ++m) {
                int oi = c->off[l][2 * m], oj = c->off[l][2 * m + 1];
                double fa, fb;
                size_t a = ghost_source(c, v, iL + oi, jL + oj, &fa);
                size_t b = ghost_source(c, v, iR + oi, jR + oj, &fb);
                dual xl = {g->u[gidx(g, v, iL + oi, jL + oj)], fa * dU[a]};
                dual xr = {g->u[gidx(g, v, iR + oi, jR + oj)], fb * dU[b]};
                sl = dadd(sl, dmul(dc(zL[m]), xl));
                sr = dadd(sr, dmul(dc(zR[m]), xr));
            }
            qL[v] = sl;
            qR[v] = sr;
        }
        riemann_d(c, qL, qR, dir, f);
        for (int v = 0; v < NV; ++v) Fout[v] = dadd(Fout[v], dmul(dc(c->qw[l][k]), f[v]));
    }
}

static int face_level(const orc_cfg *c, const int *order, int dir, int iL, int jL)
{
    int iR = iL + (dir == 0), jR = jL + (dir == 1);
    int oL = order[(size_t)src_index(jL, c->ny, c->bcy) * c->nx + src_index(iL, c->nx, c->bcx)];
    int oR = order[(size_t)src_index(jR, c->ny, c->bcy) * c->nx + src_index(iR, c->nx, c->bcx)];
    return level_of(c, oL < oR ? oL : oR); /* EDP_1 */
}

/* Directional derivative of the forced-order stage: dUout for the tangents dUs of
   U_s and dUn of U^n (s = 0 takes U^n = U_s and ignores dUn). */
void orc_stage_jvp(const orc_cfg *c, int s, const double *Us, const double *dUs, const double *dUn, double dt,
                   const int *order, double *dUout)
{
    int nx = c->nx, ny = c->ny;
    size_t ncell = (size_t)nx * ny;
    double alpha, beta;
    stage_alpha_beta(s, &alpha, &beta);
    ghosted g;
    fill_ghosted(c, Us, &g);
    double *dFx = (double *)calloc((size_t)NV * (nx + 1) * ny, sizeof(double));
    double *dGy = (double *)calloc((size_t)NV * nx * (ny + 1), sizeof(double));
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i <= nx; ++i) {
            dual F[4];
            face_flux_d(c, &g, dUs, face_level(c, order, 0, i - 1, j), 0, i - 1, j, F);
            for (int v = 0; v < NV; ++v) dFx[((size_t)v * ny + j) * (nx + 1) + i] = F[v].d;
        }
    for (int j = 0; j <= ny; ++j)
        for (int i = 0; i < nx; ++i) {
            dual F[4];
            face_flux_d(c, &g, dUs, face_level(c, order, 1, i, j - 1), 1, i, j - 1, F);
            for (int v = 0; v < NV; ++v) dGy[((size_t)v * (ny + 1) + j) * nx + i] = F[v].d;
        }
    for (int v = 0; v < NV; ++v)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t k = (size_t)v * ncell + (size_t)j * nx + i;
                double ddF = dFx[((size_t)v * ny + j) * (nx + 1) + i + 1] - dFx[((size_t)v * ny + j) * (nx + 1) + i];
                double ddG = dGy[((size_t)v * (ny + 1) + j + 1) * nx + i] - dGy[((size_t)v * (ny + 1) + j) * nx + i];
                double dstar = dUs[k] - dt * (ddF / c->dx + ddG / c->dy);
                dUout[k] = alpha * dstar + (s == 0 ? 0.0 : beta * dUn[k]);
            }
    free(dFx); free(dGy); free(g.u);
}

/* Transpose of orc_stage_jvp: for the adjoint lam_out of U_out, lam_Us = the
   adjoint of U_s and, for s > 0, lam_Un = the adjoint of U^n (for s = 0, U^n is
   U_s and lam_Un is not written).  Each face's flux adjoint is pulled back through
   the solver's Jacobian (one dual evaluation per input component) and the
   reconstruction weights onto the stencil cells. */
void orc_stage_vjp(const orc_cfg *c, int s, const double *Us, double dt, const int *order, const double *lam_out,
                   double *lam_Us, double *lam_Un)
{
    int nx = c->nx, ny = c->ny;
    size_t ncell = (size_t)nx * ny;
    double alpha, beta;
    stage_alpha_beta(s, &alpha, &beta);
    ghosted g;
    fill_ghosted(c, Us, &g);
    /* U_out = beta U^n + alpha U*: lam_U* = alpha lam_out; U* = U_s - dt div F */
    for (size_t k = 0; k < (size_t)NV * ncell; ++k) {
        lam_Us[k] = alpha * lam_out[k];
        if (s > 0 && lam_Un) lam_Un[k] = beta * lam_out[k];
    }
    for (int dir = 0; dir < 2; ++dir) {
        int nfi = dir == 0 ? nx + 1 : nx, nfj = dir == 0 ? ny : ny + 1;
        double h = dir == 0 ? c->dx : c->dy;
        for (int j = 0; j < nfj; ++j)
            for (int i = 0; i < nfi; ++i) {
                int iL = dir == 0 ? i - 1 : i, jL = dir == 0 ? j : j - 1;
                int iR = iL + (dir == 0), jR = jL + (dir == 1);
                /* the face flux enters U*(R) with +dt/h and U*(L) with -dt/h */
                double lF[4];
                int any = 0;
                for (int v = 0; v < NV; ++v) {
                    double lr = (iR < nx && jR < ny) ? lam_out[(size_t)v * ncell + (size_t)jR * nx + iR] : 0.0;
                    double ll = (iL >= 0 && jL >= 0) ? lam_out[(size_t)v * ncell + (size_t)jL * nx + iL] : 0.0;
                    lF[v] = alpha * dt / h * (lr - ll);
                    any = any || lF[v] != 0.0;
                }
                if (!any) continue;
                int l = face_level(c, order, dir, iL, jL);
                int fL = dir == 0 ? 1 : 3, fR = dir == 0 ? 0 : 2;
                int ns = c->nst[l];
                for (int k = 0; k < c->nq[l]; ++k) {
                    /* node states */
                    dual qL[4], qR[4];
                    const double *zL = c->z[l] + ((size_t)fL * c->nq[l] + k) * ns;
                    const double *zR = c->z[l] + ((size_t)fR * c->nq[l] + k) * ns;
                    for (int v = 0; v < NV; ++v) {
                        double sl = 0.0, sr = 0.0;
                        for (int m = 0; m < ns; ++m) {
                            int oi = c->off[l][2 * m], oj = c->off[l][2 * m + 1];
                            sl += zL[m] * g.u[gidx(&g, v, iL + oi, jL + oj)];
                            sr += zR[m] * g.u[gidx(&g, v, iR + oi, jR + oj)];
                        }
                        qL[v] = dc(sl);
                        qR[v] = dc(sr);
                    }
                    /* lam_q = w_k J^T lam_F, one Jacobian column per input component */
                    double gq[8];
                    for (int col = 0; col < 8; ++col) {
                        dual a[4], b[4], f[4];
                        for (int v = 0; v < NV; ++v) {
                            a[v] = qL[v];
                            b[v] = qR[v];
                        }
                        if (col < 4) a[col].d = 1.0;
                        else b[col - 4].d = 1.0;
                        riemann_d(c, a, b, dir, f);
                        double sacc = 0.0;
                        for (int v = 0; v < NV; ++v) sacc += lF[v] * f[v].d;
                        gq[col] = c->qw[l][k] * sacc;
                    }
                    /* through the reconstruction onto the stencil cells */
                    for (int v = 0; v < NV; ++v)
                        for (int m = 0; m < ns; ++m) {
                            int oi = c->off[l][2 * m], oj = c->off[l][2 * m + 1];
                            double fa, fb;
                            size_t a = ghost_source(c, v, iL + oi, jL + oj, &fa);
                            size_t b = ghost_source(c, v, iR + oi, jR + oj, &fb);
                            lam_Us[a] += fa * zL[m] * gq[v];
                            lam_Us[b] += fb * zR[m] * gq[4 + v];
                        }
                }
            }
    }
    free(g.u);
}
