/*
 * GP-MOOD oracle in 3D: a plain, slow FP64 reference of one SSP-RK3 stage.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code, header or table
 * with the product library; its GP weights come from oracle/weights3d_mp.py.
 *
 * The 2D oracle's steps (gpmood_oracle.c) written out for three space directions
 * and five conservative variables (rho, rho u, rho v, rho w, E), following
 * Bourgeois & Lee, "GP-MOOD":
 *   - Euler equations and ideal-gas EoS: Sec. "Governing equations", eq. (euler_eqn)
 *   - FV update with face quadrature: eq. (fvm_discrete), eq. (fvm_F); in 3D a face
 *     carries the tensor product of the (R+1)-point Gauss rule (reading: 3D is
 *     future work in the paper)
 *   - GP reconstruction z^T q: eq. (gp_reconstructor) (weights are inputs here)
 *   - detection: PAD eq. (PAD), CAD eq. (CAD) with the Riemann-state check, DMP
 *     eq. (DMP_RK) over the cell and its six face neighbours, plateau eq. (plateau),
 *     u2 eqs. (u2_curvature, u2_a, u2_b) per direction, CSD eqs. (divV, gradP) with
 *     the z terms added
 *   - EDP_1 face order and the MOOD loop: Sec. "The scheme cascade with GP",
 *     Sec. "Stepwise implementation", Steps 3-10; SSP-RK3: eq. (rk3)
 *   - HLLC: textbook form (Davis wave speeds, Toro's star states) with two
 *     tangential momenta.
 * Every MOOD iteration recomputes every face flux and candidate and re-detects
 * every cell.  Build with -O2 -ffp-contract=off, no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NV 5
#define GH 3 /* ghost depth: R_max + 1 = 3 for R = 2; u2 needs 2 */

enum { O3_CSD = 1u, O3_PLATEAU = 2u, O3_U2 = 4u, O3_RSCAD = 8u };

typedef struct {
    int n[3];
    double d[3];
    int bc[3];          /* 0 periodic, 1 outflow */
    double gamma;
    int nlev;
    int rad[4];         /* cascade radii, strictly decreasing, last one 0 (FOG) */
    int nst[4];         /* stencil size per level */
    const int *off[4];  /* per level: [nst][3] offsets */
    int nq[4];          /* nodes per face per level (q^2; FOG 1) */
    const double *qw[4];/* per level: node weights [nq] */
    const double *z[4]; /* per level: [6 faces][nq][nst] */
    const double *w2;   /* [3][7] u2 weights on the R = 1 stencil */
    const int *off1;    /* [7][3] R = 1 stencil offsets matching w2 */
    double sigma_v, sigma_p;
    unsigned flags;
} orc3_cfg;

static double dmin(double a, double b) { return a < b ? a : b; }
static double dmax(double a, double b) { return a > b ? a : b; }

static int src_index(int i, int n, int bc)
{
    if (bc == 0) { int r = i % n; return r < 0 ? r + n : r; }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

typedef struct { int N[3]; double *u; } ghosted3;

static size_t gidx(const ghosted3 *g, int v, int i, int j, int k)
{
    return (((size_t)v * g->N[2] + (size_t)(k + GH)) * g->N[1] + (size_t)(j + GH)) * g->N[0] + (size_t)(i + GH);
}

static size_t cidx(const orc3_cfg *c, int i, int j, int k)
{
    return ((size_t)k * c->n[1] + j) * c->n[0] + i;
}

static void fill_ghosted(const orc3_cfg *c, const double *U, ghosted3 *g)
{
    for (int d = 0; d < 3; ++d) g->N[d] = c->n[d] + 2 * GH;
    size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
    g->u = (double *)malloc(sizeof(double) * NV * g->N[0] * g->N[1] * g->N[2]);
    for (int v = 0; v < NV; ++v)
        for (int k = -GH; k < c->n[2] + GH; ++k)
            for (int j = -GH; j < c->n[1] + GH; ++j)
                for (int i = -GH; i < c->n[0] + GH; ++i) {
                    int si = src_index(i, c->n[0], c->bc[0]), sj = src_index(j, c->n[1], c->bc[1]);
                    int sk = src_index(k, c->n[2], c->bc[2]);
                    g->u[gidx(g, v, i, j, k)] = U[(size_t)v * nc + cidx(c, si, sj, sk)];
                }
}

static double pressure(double g, const double *q)
{
    return (g - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
}

static int level_of(const orc3_cfg *c, int r)
{
    for (int l = 0; l < c->nlev; ++l)
        if (c->rad[l] == r) return l;
    return -1;
}

/* HLLC through a face with normal along axis dir (0, 1, 2). */
static void hllc3(double g, const double *UL, const double *UR, int dir, double *F)
{
    int n = 1 + dir, t1 = 1 + (dir + 1) % 3, t2 = 1 + (dir + 2) % 3;
    double rl = UL[0], ul = UL[n] / rl, vl = UL[t1] / rl, wl = UL[t2] / rl, El = UL[4];
    double rr = UR[0], ur = UR[n] / rr, vr = UR[t1] / rr, wr = UR[t2] / rr, Er = UR[4];
    double pl = (g - 1.0) * (El - 0.5 * rl * (ul * ul + vl * vl + wl * wl));
    double pr = (g - 1.0) * (Er - 0.5 * rr * (ur * ur + vr * vr + wr * wr));
    double cl = sqrt(g * pl / rl), cr = sqrt(g * pr / rr);
    double SL = dmin(ul - cl, ur - cr);
    double SR = dmax(ul + cl, ur + cr);
    double Ss = (pr - pl + rl * ul * (SL - ul) - rr * ur * (SR - ur)) / (rl * (SL - ul) - rr * (SR - ur));
    double f[5];
    if (SL >= 0.0) {
        f[0] = rl * ul; f[1] = rl * ul * ul + pl; f[2] = rl * ul * vl; f[3] = rl * ul * wl; f[4] = ul * (El + pl);
    } else if (Ss >= 0.0) {
        double fac = rl * (SL - ul) / (SL - Ss);
        double us[5] = {fac, fac * Ss, fac * vl, fac * wl, fac * (El / rl + (Ss - ul) * (Ss + pl / (rl * (SL - ul))))};
        double uk[5] = {rl, rl * ul, rl * vl, rl * wl, El};
        double fk[5] = {rl * ul, rl * ul * ul + pl, rl * ul * vl, rl * ul * wl, ul * (El + pl)};
        for (int m = 0; m < 5; ++m) f[m] = fk[m] + SL * (us[m] - uk[m]);
    } else if (SR > 0.0) {
        double fac = rr * (SR - ur) / (SR - Ss);
        double us[5] = {fac, fac * Ss, fac * vr, fac * wr, fac * (Er / rr + (Ss - ur) * (Ss + pr / (rr * (SR - ur))))};
        double uk[5] = {rr, rr * ur, rr * vr, rr * wr, Er};
        double fk[5] = {rr * ur, rr * ur * ur + pr, rr * ur * vr, rr * ur * wr, ur * (Er + pr)};
        for (int m = 0; m < 5; ++m) f[m] = fk[m] + SR * (us[m] - uk[m]);
    } else {
        f[0] = rr * ur; f[1] = rr * ur * ur + pr; f[2] = rr * ur * vr; f[3] = rr * ur * wr; f[4] = ur * (Er + pr);
    }
    F[0] = f[0]; F[n] = f[1]; F[t1] = f[2]; F[t2] = f[3]; F[4] = f[4];
}

void orc3_hllc(double g, const double *UL, const double *UR, int dir, double *F) { hllc3(g, UL, UR, dir, F); }

/* State of cell (i, j, k) at face f, node q, level l. */
static void recon3(const orc3_cfg *c, const ghosted3 *g, int l, int f, int q, int i, int j, int k, double *out)
{
    int ns = c->nst[l];
    const double *z = c->z[l] + ((size_t)f * c->nq[l] + q) * ns;
    const int *o = c->off[l];
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
        for (int m = 0; m < ns; ++m) s += z[m] * g->u[gidx(g, v, i + o[3 * m], j + o[3 * m + 1], k + o[3 * m + 2])];
        out[v] = s;
    }
}

/* CAD on a reconstructed Riemann state (Sec. CAD): density and pressure finite and
   positive (a non-positive one gives an invalid sound speed); an inadmissible state
   troubles both cells of its face, as in 2D. */
static int state_inadmissible(double gam, const double *q)
{
    double p = pressure(gam, q);
    return !(isfinite(q[0]) && isfinite(p) && q[0] > 0.0 && p > 0.0);
}

typedef struct { double rmin, rmax; int plat, csd, u2; } relax3_t;

static const int NB[7][3] = {{0, 0, 0}, {-1, 0, 0}, {1, 0, 0}, {0, -1, 0}, {0, 1, 0}, {0, 0, -1}, {0, 0, 1}};

static void cell_relax3(const orc3_cfg *c, const ghosted3 *g, int i, int j, int k, relax3_t *r)
{
    double gam = c->gamma;
    double lo = g->u[gidx(g, 0, i, j, k)], hi = lo;
    for (int m = 1; m < 7; ++m) {
        double v = g->u[gidx(g, 0, i + NB[m][0], j + NB[m][1], k + NB[m][2])];
        lo = dmin(lo, v);
        hi = dmax(hi, v);
    }
    r->rmin = lo;
    r->rmax = hi;
    double d3 = dmin(dmin(c->d[0] * c->d[0] * c->d[0], c->d[1] * c->d[1] * c->d[1]), c->d[2] * c->d[2] * c->d[2]);
    r->plat = (hi - lo) < d3;
    double divV = 0.0, gradp = 0.0;
    for (int d = 0; d < 3; ++d) {
        double qp[NV], qm[NV];
        for (int v = 0; v < NV; ++v) {
            qp[v] = g->u[gidx(g, v, i + NB[2 + 2 * d][0], j + NB[2 + 2 * d][1], k + NB[2 + 2 * d][2])];
            qm[v] = g->u[gidx(g, v, i + NB[1 + 2 * d][0], j + NB[1 + 2 * d][1], k + NB[1 + 2 * d][2])];
        }
        divV += (qp[1 + d] / qp[0] - qm[1 + d] / qm[0]) / (2.0 * c->d[d]);
        double pp = pressure(gam, qp), pm = pressure(gam, qm);
        gradp += fabs(pp - pm) / (2.0 * c->d[d] * dmin(pp, pm));
    }
    r->csd = (divV >= -c->sigma_v) && (gradp <= c->sigma_p);
    double delta = dmin(dmin(c->d[0], c->d[1]), c->d[2]);
    int ok = 1;
    for (int d = 0; d < 3; ++d) {
        double cmin = 0.0, cmax = 0.0;
        for (int m = 0; m < 7; ++m) {
            int mi = i + NB[m][0], mj = j + NB[m][1], mk = k + NB[m][2];
            double kap = 0.0;
            for (int e = 0; e < 7; ++e)
                kap += c->w2[d * 7 + e] * g->u[gidx(g, 0, mi + c->off1[3 * e], mj + c->off1[3 * e + 1], mk + c->off1[3 * e + 2])];
            if (m == 0) { cmin = kap; cmax = kap; }
            else { cmin = dmin(cmin, kap); cmax = dmax(cmax, kap); }
        }
        int a = (cmin * cmax > -delta) && (dmax(fabs(cmax), fabs(cmin)) < delta);
        /* eq. (u2_b) multiplied through by |Cmax|, as in the 2D oracle */
        int b = (cmin * cmax > -delta) && (fabs(cmin) >= 0.5 * fabs(cmax));
        ok = ok && (a || b);
    }
    r->u2 = ok;
}

/* Relaxation data of every cell: rmin, rmax and (plateau, csd, u2) as 0/1 doubles. */
void orc3_relax(const orc3_cfg *c, const double *Us, double *out /* [ncell][5] */)
{
    ghosted3 g;
    fill_ghosted(c, Us, &g);
    for (int k = 0; k < c->n[2]; ++k)
        for (int j = 0; j < c->n[1]; ++j)
            for (int i = 0; i < c->n[0]; ++i) {
                relax3_t r;
                cell_relax3(c, &g, i, j, k, &r);
                double *o = out + 5 * cidx(c, i, j, k);
                o[0] = r.rmin; o[1] = r.rmax; o[2] = r.plat; o[3] = r.csd; o[4] = r.u2;
            }
    free(g.u);
}

static int detect3(const orc3_cfg *c, int order, const relax3_t *r, const double *us, int rs_bad)
{
    if (order == 0) return 0;
    double rho = us[0], p = pressure(c->gamma, us);
    if (!(isfinite(rho) && isfinite(p))) return 1;
    if ((c->flags & O3_RSCAD) && rs_bad) return 1;
    if (!(rho > 0.0 && p > 0.0)) return 1;
    if ((c->flags & O3_CSD) && r->csd) return 0;
    if ((c->flags & O3_PLATEAU) && r->plat) return 0;
    if (r->rmin <= rho && rho <= r->rmax) return 0;
    if ((c->flags & O3_U2) && r->u2) return 0;
    return 1;
}

/* Faces of axis dir: face index i_dir in [0, n_dir] between cell i_dir-1 and i_dir. */
static void candidate3(const orc3_cfg *c, const ghosted3 *g, const int *order, double dt, double *Ustar, int *rsbad)
{
    size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
    double gam = c->gamma;
    double *F[3];
    unsigned char *rs[3];
    int fn[3][3];
    for (int d = 0; d < 3; ++d) {
        for (int e = 0; e < 3; ++e) fn[d][e] = c->n[e] + (e == d);
        size_t nf = (size_t)fn[d][0] * fn[d][1] * fn[d][2];
        F[d] = (double *)calloc(NV * nf, sizeof(double));
        rs[d] = (unsigned char *)calloc(nf, 1);
    }
    for (int d = 0; d < 3; ++d) {
        size_t nf = (size_t)fn[d][0] * fn[d][1] * fn[d][2];
#pragma omp parallel for schedule(static)
        for (int k = 0; k < fn[d][2]; ++k)
            for (int j = 0; j < fn[d][1]; ++j)
                for (int i = 0; i < fn[d][0]; ++i) {
                    int L[3] = {i, j, k}, R[3] = {i, j, k};
                    L[d] -= 1;
                    int sL[3], sR[3];
                    for (int e = 0; e < 3; ++e) {
                        sL[e] = src_index(L[e], c->n[e], c->bc[e]);
                        sR[e] = src_index(R[e], c->n[e], c->bc[e]);
                    }
                    int oL = order[cidx(c, sL[0], sL[1], sL[2])], oR = order[cidx(c, sR[0], sR[1], sR[2])];
                    int l = level_of(c, oL < oR ? oL : oR);
                    double Fs[NV] = {0, 0, 0, 0, 0};
                    unsigned char bad = 0;
                    for (int q = 0; q < c->nq[l]; ++q) {
                        double qL[NV], qR[NV], f[NV];
                        recon3(c, g, l, 2 * d + 1, q, L[0], L[1], L[2], qL); /* + face of the left cell */
                        recon3(c, g, l, 2 * d, q, R[0], R[1], R[2], qR);     /* - face of the right cell */
                        if (state_inadmissible(gam, qL)) bad |= 1;
                        if (state_inadmissible(gam, qR)) bad |= 2;
                        hllc3(gam, qL, qR, d, f);
                        for (int v = 0; v < NV; ++v) Fs[v] += c->qw[l][q] * f[v];
                    }
                    size_t fi = ((size_t)k * fn[d][1] + j) * fn[d][0] + i;
                    for (int v = 0; v < NV; ++v) F[d][(size_t)v * nf + fi] = Fs[v];
                    rs[d][fi] = bad;
                }
    }
#pragma omp parallel for schedule(static)
    for (int k = 0; k < c->n[2]; ++k)
        for (int j = 0; j < c->n[1]; ++j)
            for (int i = 0; i < c->n[0]; ++i) {
                size_t ci = cidx(c, i, j, k);
                int bad = 0;
                double div[NV] = {0, 0, 0, 0, 0};
                for (int d = 0; d < 3; ++d) {
                    size_t nf = (size_t)fn[d][0] * fn[d][1] * fn[d][2];
                    int P[3] = {i, j, k};
                    size_t fm = ((size_t)P[2] * fn[d][1] + P[1]) * fn[d][0] + P[0];
                    P[d] += 1;
                    size_t fp = ((size_t)P[2] * fn[d][1] + P[1]) * fn[d][0] + P[0];
                    for (int v = 0; v < NV; ++v) div[v] += (F[d][(size_t)v * nf + fp] - F[d][(size_t)v * nf + fm]) / c->d[d];
                    bad = bad || rs[d][fm] != 0 || rs[d][fp] != 0;
                }
                for (int v = 0; v < NV; ++v) Ustar[(size_t)v * nc + ci] = g->u[gidx(g, v, i, j, k)] - dt * div[v];
                rsbad[ci] = bad;
            }
    for (int d = 0; d < 3; ++d) { free(F[d]); free(rs[d]); }
}

/* Candidate only (U* and the per-cell Riemann-state CAD flags) for given orders. */
void orc3_candidate(const orc3_cfg *c, const double *Us, double dt, const int *order, double *Ustar, int *rsbad)
{
    ghosted3 g;
    fill_ghosted(c, Us, &g);
    candidate3(c, &g, order, dt, Ustar, rsbad);
    free(g.u);
}

static void combine3(size_t n, int s, const double *Un, const double *Ustar, double *Uout)
{
    for (size_t k = 0; k < n; ++k) {
        if (s == 0) Uout[k] = Ustar[k];
        else if (s == 1) Uout[k] = 0.25 * (3.0 * Un[k] + Ustar[k]);
        else Uout[k] = (Un[k] + 2.0 * Ustar[k]) / 3.0;
    }
}

/* One stage with the full MOOD loop.  order_out[cell] = final radius; counts[l]
   = cells finishing at level l; returns the number of evaluations. */
int orc3_stage(const orc3_cfg *c, int s, const double *Un, const double *Us, double dt, double *Uout,
               int *order_out, long long *counts)
{
    size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
    ghosted3 g;
    fill_ghosted(c, Us, &g);
    relax3_t *rel = (relax3_t *)malloc(sizeof(relax3_t) * nc);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < c->n[2]; ++k)
        for (int j = 0; j < c->n[1]; ++j)
            for (int i = 0; i < c->n[0]; ++i) cell_relax3(c, &g, i, j, k, &rel[cidx(c, i, j, k)]);
    int *order = (int *)malloc(sizeof(int) * nc);
    int *rsbad = (int *)malloc(sizeof(int) * nc);
    double *Ustar = (double *)malloc(sizeof(double) * NV * nc);
    for (size_t q = 0; q < nc; ++q) order[q] = c->rad[0];
    int iters = 0;
    for (;;) {
        ++iters;
        candidate3(c, &g, order, dt, Ustar, rsbad);
        long long ntr = 0;
        int *next = (int *)malloc(sizeof(int) * nc);
        for (size_t q = 0; q < nc; ++q) {
            double us[NV];
            for (int v = 0; v < NV; ++v) us[v] = Ustar[(size_t)v * nc + q];
            int tr = detect3(c, order[q], &rel[q], us, rsbad[q]);
            next[q] = order[q];
            if (tr) {
                int l = level_of(c, order[q]);
                next[q] = c->rad[l + 1];
                ++ntr;
            }
        }
        memcpy(order, next, sizeof(int) * nc);
        free(next);
        if (ntr == 0) break;
    }
    combine3(NV * nc, s, Un, Ustar, Uout);
    for (int l = 0; l < c->nlev; ++l) counts[l] = 0;
    for (size_t q = 0; q < nc; ++q) {
        order_out[q] = order[q];
        counts[level_of(c, order[q])] += 1;
    }
    free(order); free(rsbad); free(Ustar); free(rel); free(g.u);
    return iters;
}

double orc3_dt(const orc3_cfg *c, const double *U, double cfl)
{
    size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
    double lam = 0.0;
    for (size_t q = 0; q < nc; ++q) {
        double u[NV];
        for (int v = 0; v < NV; ++v) u[v] = U[(size_t)v * nc + q];
        double p = pressure(c->gamma, u);
        if (!(u[0] > 0.0 && p > 0.0 && isfinite(u[0]) && isfinite(p))) continue;
        double cs = sqrt(c->gamma * p / u[0]);
        for (int d = 0; d < 3; ++d) lam = dmax(lam, (fabs(u[1 + d] / u[0]) + cs) / c->d[d]);
    }
    return cfl / lam;
}

/* nsteps SSP-RK3 steps in place; dts[n] and iters[n][3] receive each step's dt
   and evaluation counts (counts of the last stage's levels in counts). */
void orc3_run(const orc3_cfg *c, double *U, double cfl, int nsteps, double *dts, int *iters, long long *counts)
{
    size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
    double *U1 = (double *)malloc(sizeof(double) * NV * nc);
    double *U2 = (double *)malloc(sizeof(double) * NV * nc);
    int *ord = (int *)malloc(sizeof(int) * nc);
    for (int n = 0; n < nsteps; ++n) {
        double dt = orc3_dt(c, U, cfl);
        dts[n] = dt;
        iters[3 * n] = orc3_stage(c, 0, U, U, dt, U1, ord, counts);
        iters[3 * n + 1] = orc3_stage(c, 1, U, U1, dt, U2, ord, counts);
        iters[3 * n + 2] = orc3_stage(c, 2, U, U2, dt, U1, ord, counts);
        memcpy(U, U1, sizeof(double) * NV * nc);
    }
    free(U1); free(U2); free(ord);
}
