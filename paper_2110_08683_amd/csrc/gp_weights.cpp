// GP prediction vectors in quadruple precision (host, once per scheme).
//
// Bourgeois & Lee, "GP-MOOD":
//   eq. (SE-pred)  t*_m = prod_d sqrt(pi/2) a_d [erf((s_d+1/2)/(sqrt2 a_d)) - erf((s_d-1/2)/(sqrt2 a_d))]
//   eq. (SE-cov)   C_mn = prod_d sqrt(pi) a_d^2 { phi(u+) + phi(u-) - 2 phi(u0) },
//                  phi(u) = u erf(u) + exp(-u^2)/sqrt(pi), u = (D +- 1, D)/(sqrt2 a_d)
//   eq. (gp_reconstructor)  z = C^{-1} t*, by Cholesky of the SPD matrix C
//   eq. (normalized_z)      z <- z / (z^T 1)   (signed sum: the stated purpose is z^T 1 = 1)
//   App. B          second derivative of the t* factor along d at the cell centre
// with a_d = ell / Delta_d and all separations in cell units (eq. (delta_mnd)).
// Sec. "Singularity of the covariance kernel matrix": C is badly conditioned
// (about 4e15 for R = 3 at ell = 12 dx), so everything runs in __float128 and is
// rounded to double / float at the end, as the paper does.
#include "gp_weights.h"
#include "gpmood_tables.h"

#include <quadmath.h>

#include <cstring>
#include <vector>

namespace gpm {
namespace {

typedef __float128 qf;

const qf QPI = acosq((qf)-1);

qf t_factor(qf s, qf a)
{
    qf r2a = sqrtq((qf)2) * a;
    return sqrtq(QPI / 2) * a * (erfq((s + (qf)0.5) / r2a) - erfq((s - (qf)0.5) / r2a));
}

qf phi(qf u) { return u * erfq(u) + expq(-u * u) / sqrtq(QPI); }

qf c_factor(qf D, qf a)
{
    qf r2a = sqrtq((qf)2) * a;
    return sqrtq(QPI) * a * a * (phi((D + 1) / r2a) + phi((D - 1) / r2a) - 2 * phi(D / r2a));
}

qf d2_t_factor(qf s, qf a, qf ell)
{
    qf h = (qf)0.5;
    qf em = expq(-(s - h) * (s - h) / (2 * a * a));
    qf ep = expq(-(s + h) * (s + h) / (2 * a * a));
    return ((s - h) * em - (s + h) * ep) / (ell * ell);
}

struct Cell { int di, dj; };

std::vector<Cell> diamond(int R)
{
    std::vector<Cell> st;
    for (int dj = -R; dj <= R; ++dj)
        for (int di = -R; di <= R; ++di)
            if ((di < 0 ? -di : di) + (dj < 0 ? -dj : dj) <= R) st.push_back({di, dj});
    return st;
}

// Cholesky factor L (lower) of the n x n SPD matrix A, row-major; false if not SPD.
bool cholesky(std::vector<qf> &A, int n)
{
    for (int j = 0; j < n; ++j) {
        qf d = A[j * n + j];
        for (int k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0)) return false;
        qf l = sqrtq(d);
        A[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            qf s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = s / l;
        }
    }
    return true;
}

void chol_solve(const std::vector<qf> &L, int n, std::vector<qf> &b)
{
    for (int i = 0; i < n; ++i) {
        qf s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        qf s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

// Gauss nodes (non-negative members of the rule in Table tab:QR-pt-weight) and weights.
void gauss_slots(int R, qf g[2], qf w[2])
{
    if (R == 1) {
        g[0] = 1 / (2 * sqrtq((qf)3));
        w[0] = (qf)0.5;
    } else if (R == 2) {
        g[0] = sqrtq((qf)3 / 5) / 2;
        w[0] = (qf)5 / 18;
        g[1] = 0;
        w[1] = (qf)8 / 18;
    } else {
        qf s = sqrtq((qf)6 / 5);
        g[0] = sqrtq((qf)3 / 7 + 2 * s / 7) / 2;
        g[1] = sqrtq((qf)3 / 7 - 2 * s / 7) / 2;
        w[0] = (18 - sqrtq((qf)30)) / 72;
        w[1] = (18 + sqrtq((qf)30)) / 72;
    }
}

int index_of(const std::vector<Cell> &st, int di, int dj)
{
    for (size_t m = 0; m < st.size(); ++m)
        if (st[m].di == di && st[m].dj == dj) return (int)m;
    return -1;
}

}  // namespace

namespace {

// Quarter-basis weights of radius R at (ax, ay) = ell / (dx, dy), in quad precision,
// for the stencil shape (GPW_DIAMOND, GPW_CROSS: the cells of the diamond on the
// axes; GPW_POLY3, radius 1 only: the POL-MOOD3 polynomial weights).  Cells
// outside the stencil get weight 0.
int level_q(int R, qf ax, qf ay, qf W[2][2][25], qf qw[2], int shape)
{
    std::vector<Cell> st;
    for (const Cell &x : diamond(R))
        if (shape == GPW_DIAMOND || x.di == 0 || x.dj == 0) st.push_back(x);
    const int n = (int)st.size();
    std::vector<qf> L(n * n);
    for (int m = 0; m < n; ++m)
        for (int k = 0; k < n; ++k)
            L[m * n + k] = c_factor((qf)(st[k].di - st[m].di), ax) * c_factor((qf)(st[k].dj - st[m].dj), ay);
    if (shape != GPW_POLY3 && !cholesky(L, n)) return -1;
    if (shape == GPW_POLY3 && R != 1) return -1;
    qf g[2];
    gauss_slots(R, g, qw);
    for (int dir = 0; dir < 2; ++dir)
        for (int k = 0; k < slots_of(R); ++k) {
            // x faces: x* = (+1/2, g); y faces: x* = (g, +1/2)
            qf xs = dir == 0 ? (qf)0.5 : g[k];
            qf ys = dir == 0 ? g[k] : (qf)0.5;
            std::vector<qf> z(n);
            if (shape == GPW_POLY3) {
                // eqs. (poly3), (p3_coeffs): the quadratic matching the five cell
                // averages; normal to the face -1/6, 5/6, 1/3, along the face the
                // linear term only (the tangential node coordinate t: +-t/2)
                const qf t = dir == 0 ? ys : xs;
                for (int m = 0; m < n; ++m) {
                    const int nrm = dir == 0 ? st[m].di : st[m].dj, tan = dir == 0 ? st[m].dj : st[m].di;
                    z[m] = nrm == 0 && tan == 0 ? (qf)5 / 6
                           : (nrm == 1 ? (qf)1 / 3 : (nrm == -1 ? -(qf)1 / 6 : (qf)tan * t / 2));
                }
            } else {
                for (int m = 0; m < n; ++m) z[m] = t_factor(xs - st[m].di, ax) * t_factor(ys - st[m].dj, ay);
                chol_solve(L, n, z);
                qf sum = 0;
                for (int m = 0; m < n; ++m) sum += z[m];
                for (int m = 0; m < n; ++m) z[m] /= sum;
            }
            auto Z = [&](int di, int dj) {
                const int m = index_of(st, di, dj);
                return m < 0 ? (qf)0 : z[m];
            };
            for (int e = 0; e < kNQ[R]; ++e) {
                const int a = kQ[e].a, b = kQ[e].b, c = kQ[e].comp;
                qf w;
                if (a == 0 && b == 0) {
                    w = Z(0, 0);
                } else if (b == 0) {
                    w = c == C_EE ? (Z(a, 0) + Z(-a, 0)) / 2 : (Z(a, 0) - Z(-a, 0)) / 2;
                } else if (a == 0) {
                    w = c == C_EE ? (Z(0, b) + Z(0, -b)) / 2 : (Z(0, b) - Z(0, -b)) / 2;
                } else {
                    qf pp = Z(a, b), mp = Z(-a, b), pm = Z(a, -b), mm = Z(-a, -b);
                    if (c == C_EE) w = (pp + mp + pm + mm) / 4;
                    else if (c == C_OE) w = (pp - mp + pm - mm) / 4;
                    else if (c == C_EO) w = (pp + mp - pm - mm) / 4;
                    else w = (pp - mp - pm + mm) / 4;
                }
                W[dir][k][e] = w;
            }
        }
    return 0;
}

}  // namespace

int gpw_level(int R, double ax_d, double ay_d, int shape, GpwLevel *out)
{
    std::memset(out, 0, sizeof(*out));
    out->R = R;
    if (R <= 0) return 0;
    qf W[2][2][25] = {}, qw[2] = {0, 0};
    if (level_q(R, ax_d, ay_d, W, qw, shape) != 0) return -1;
    for (int k = 0; k < slots_of(R); ++k) {
        out->qw64[k] = (double)qw[k];
        out->qw32[k] = (float)qw[k];
    }
    for (int dir = 0; dir < 2; ++dir)
        for (int k = 0; k < slots_of(R); ++k)
            for (int e = 0; e < kNQ[R]; ++e) {
                out->w64[dir][k][e] = (double)W[dir][k][e];
                out->w32[dir][k][e] = (float)W[dir][k][e];
            }
    // d w / d log(ell): central difference in quad precision, ell scaled by 1 +- h
    // (both ax and ay scale with ell); the step keeps truncation (h^2) and the
    // rounding of the ill-conditioned solve (~1e-19 / h) below 1e-12
    const qf h = (qf)1 / 1000000;
    qf Wp[2][2][25] = {}, Wm[2][2][25] = {}, q2[2];
    if (level_q(R, (qf)ax_d * (1 + h), (qf)ay_d * (1 + h), Wp, q2, shape) != 0) return -1;
    if (level_q(R, (qf)ax_d * (1 - h), (qf)ay_d * (1 - h), Wm, q2, shape) != 0) return -1;
    for (int dir = 0; dir < 2; ++dir)
        for (int k = 0; k < slots_of(R); ++k)
            for (int e = 0; e < kNQ[R]; ++e) out->dlw64[dir][k][e] = (double)((Wp[dir][k][e] - Wm[dir][k][e]) / (2 * h));
    return 0;
}

int gpw_curvature(double ax_d, double ay_d, double ell_d, GpwCurv *out)
{
    std::memset(out, 0, sizeof(*out));
    const qf ax = ax_d, ay = ay_d, ell = ell_d;
    std::vector<Cell> st = diamond(1);
    const int n = (int)st.size();
    std::vector<qf> L(n * n);
    for (int m = 0; m < n; ++m)
        for (int k = 0; k < n; ++k)
            L[m * n + k] = c_factor((qf)(st[k].di - st[m].di), ax) * c_factor((qf)(st[k].dj - st[m].dj), ay);
    if (!cholesky(L, n)) return -1;
    for (int d = 0; d < 2; ++d) {
        std::vector<qf> w(n);
        for (int m = 0; m < n; ++m) {
            qf sx = -(qf)st[m].di, sy = -(qf)st[m].dj;  // x* = cell centre
            w[m] = d == 0 ? d2_t_factor(sx, ax, ell) * t_factor(sy, ay)
                          : t_factor(sx, ax) * d2_t_factor(sy, ay, ell);
        }
        chol_solve(L, n, w);
        qf c0 = w[index_of(st, 0, 0)];
        qf along = d == 0 ? (w[index_of(st, 1, 0)] + w[index_of(st, -1, 0)]) / 2
                          : (w[index_of(st, 0, 1)] + w[index_of(st, 0, -1)]) / 2;
        qf across = d == 0 ? (w[index_of(st, 0, 1)] + w[index_of(st, 0, -1)]) / 2
                           : (w[index_of(st, 1, 0)] + w[index_of(st, -1, 0)]) / 2;
        qf v[3] = {c0, along, across};
        for (int k = 0; k < 3; ++k) {
            out->w64[d][k] = (double)v[k];
            out->w32[d][k] = (float)v[k];
        }
    }
    return 0;
}

// ---------------------------------------------------------------- 3D
namespace {

void ball_cov(int n, const qf a[3], std::vector<qf> &L)
{
    L.assign((size_t)n * n, 0);
    for (int m = 0; m < n; ++m)
        for (int k = 0; k < n; ++k) {
            qf v = 1;
            for (int d = 0; d < 3; ++d) v *= c_factor((qf)(kBall[k][d] - kBall[m][d]), a[d]);
            L[(size_t)m * n + k] = v;
        }
}

}  // namespace

int gpw3_level(int R, double ax_d, double ay_d, double az_d, Gpw3Level *out)
{
    std::memset(out, 0, sizeof(*out));
    out->R = R;
    if (R < 1 || R > 2) return -1;
    const qf a[3] = {ax_d, ay_d, az_d};
    const int n = kNBall[R];
    std::vector<qf> L;
    ball_cov(n, a, L);
    if (!cholesky(L, n)) return -1;
    // 1D Gauss rule on [-1/2, 1/2] with q = R + 1 nodes, from the 2D slots
    qf g2[2], w2[2], g[3], w[3];
    gauss_slots(R, g2, w2);
    int q;
    if (R == 1) {
        q = 2;
        g[0] = g2[0]; g[1] = -g2[0];
        w[0] = w2[0]; w[1] = w2[0];
    } else {
        q = 3;
        g[0] = g2[0]; g[1] = 0; g[2] = -g2[0];
        w[0] = w2[0]; w[1] = w2[1]; w[2] = w2[0];
    }
    out->nq = q * q;
    std::vector<std::vector<qf>> zq(9);  // R = 2: a face's unnormalised prediction vectors
    for (int f = 0; f < 6; ++f) {
        const int ax = f / 2;
        const qf side = (f & 1) ? (qf)0.5 : (qf)-0.5;
        const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
        for (int i1 = 0; i1 < q; ++i1)
            for (int i2 = 0; i2 < q; ++i2) {
                qf x[3];
                x[ax] = side;
                x[t1] = g[i1];
                x[t2] = g[i2];
                std::vector<qf> z(n);
                for (int m = 0; m < n; ++m) {
                    qf v = 1;
                    for (int d = 0; d < 3; ++d) v *= t_factor(x[d] - kBall[m][d], a[d]);
                    z[m] = v;
                }
                chol_solve(L, n, z);
                qf sum = 0;
                for (int m = 0; m < n; ++m) sum += z[m];
                const int k = i1 * q + i2;
                for (int m = 0; m < n; ++m) {
                    out->z64[f][k][m] = (double)(z[m] / sum);
                    out->z32[f][k][m] = (float)(z[m] / sum);
                }
                out->qw64[k] = (double)(w[i1] * w[i2]);
                out->qw32[k] = (float)(w[i1] * w[i2]);
                if (R == 2) zq[k] = z;
            }
        if (R != 2) continue;
        // parity-basis weights of the four node classes, from the normalised
        // quad-precision prediction vectors
        for (int cls = 0; cls < 4; ++cls) {
            const int k = kPar3Canon[cls];
            qf zs = 0;
            for (int m = 0; m < n; ++m) zs += zq[k][m];
            for (int e = 0; e < kNPar3; ++e) {
                const Par3 &P = kPar3[e];
                const bool use = cls == 3 || P.comp == 0 || (cls == 1 && P.comp == 1) || (cls == 2 && P.comp == 2);
                qf acc = 0;
                int cnt = 0;
                for (int s1 = -1; s1 <= 1; s1 += 2)
                    for (int s2 = -1; s2 <= 1; s2 += 2) {
                        if ((P.a1 == 0 && s1 < 0) || (P.a2 == 0 && s2 < 0)) continue;
                        int d[3];
                        d[ax] = P.dn;
                        d[t1] = s1 * P.a1;
                        d[t2] = s2 * P.a2;
                        const int m = ball_index(d[0], d[1], d[2]);
                        const int chi = (P.comp == 1 || P.comp == 3 ? s1 : 1) * (P.comp == 2 || P.comp == 3 ? s2 : 1);
                        acc += (qf)chi * zq[k][m];
                        ++cnt;
                    }
                const qf v = use ? acc / zs / (qf)cnt : (qf)0;
                out->pz64[f][cls][e] = (double)v;
                out->pz32[f][cls][e] = (float)v;
            }
        }
    }
    return 0;
}

int gpw3_curvature(double ax_d, double ay_d, double az_d, double ell_d, Gpw3Curv *out)
{
    std::memset(out, 0, sizeof(*out));
    const qf a[3] = {ax_d, ay_d, az_d}, ell = ell_d;
    const int n = kNBall[1];
    std::vector<qf> L;
    ball_cov(n, a, L);
    if (!cholesky(L, n)) return -1;
    for (int d = 0; d < 3; ++d) {
        std::vector<qf> w(n);
        for (int m = 0; m < n; ++m) {
            qf v = 1;
            for (int e = 0; e < 3; ++e) {
                const qf s = -(qf)kBall[m][e];  // x* = cell centre
                v *= e == d ? d2_t_factor(s, a[e], ell) : t_factor(s, a[e]);
            }
            w[m] = v;
        }
        chol_solve(L, n, w);
        // kBall ring 1: (-x, +x, -y, +y, -z, +z) at entries 1..6
        qf v[4];
        v[0] = w[0];
        v[1] = (w[1 + 2 * d] + w[2 + 2 * d]) / 2;
        int k = 2;
        for (int e = 0; e < 3; ++e)
            if (e != d) v[k++] = (w[1 + 2 * e] + w[2 + 2 * e]) / 2;
        for (int j = 0; j < 4; ++j) {
            out->w64[d][j] = (double)v[j];
            out->w32[d][j] = (float)v[j];
        }
    }
    return 0;
}

}  // namespace gpm
