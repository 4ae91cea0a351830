/*
 * Oracle weighted state redistribution (TEST INFRASTRUCTURE ONLY; see
 * oracle.h).
 *
 * Follows Section 5.1 of the paper step by step, on each of the four
 * instances independently:
 *   small cells (V < V_target = small_vfrac * dx dy dz) are merged with
 *   neighbours - first along the EB normal, then along the next largest
 *   normal component (completing a 2x2x1 block), then a 2x2x2 block - until
 *   the neighbourhood volume reaches V_target;
 *   M, M-, W, W- and N are the explicit sets / counts;
 *   kappa (Eq. kappa), omega (Eq. omega), the neighbourhood volume V-hat
 *   (Eq. nbhd_vol) and centroid x-hat are precomputed;
 *   per field: Q-hat (Eq. qhat_omega), a least-squares gradient of Q-hat over
 *   a 3x3x3 stencil (5 wide along directions with too little centroid spread;
 *   zero if too few points), a Barth-Jespersen-style limiter, the linear
 *   reconstruction (Eq. qrecon) and the final update (Eq. final_update_omega).
 *
 * Readings where the paper is silent (also listed in the design notes):
 *   small <=> 0 < alpha < small_vfrac (1 - 1e-12); a tier is accepted when the
 *   member volume reaches V_target (1 - 1e-12);
 *   axes are ordered by |n_d| descending, ties (within 1e-12 max|n|) to the
 *   lower axis; the step along an axis follows sgn(n_d), + when |n_d| is
 *   within the tie tolerance of 0; members are fluid CVs inside the domain;
 *   kappa = min(1, (V_target - V_i) / sum_{M-} V), 0 if M- is empty;
 *   N counts the CV's own neighbourhood;
 *   gradient only for small CVs with |M| >= 2; unweighted least squares
 *   anchored at Q-hat_i with points at the neighbourhood centroids; a
 *   direction is widened when the spread of the member centroids along it is
 *   below half the mesh spacing; zero gradient with fewer than 3 points, a
 *   spread still below half the spacing after widening, or a reciprocal
 *   condition number below 1e-10 of the normal matrix in mesh units;
 *   limiter: for each component, the largest factor <= 1 that keeps the
 *   reconstruction, evaluated at the centroids of the cells it is applied to
 *   (the members of M_i), inside [min, max] of Q-hat over the fit points and
 *   the CV itself.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define TIE 1e-12

typedef struct {
    const orc_grid* g;
    double* const* geo;
    double* const* w;
    size_t NI;
    int nx, ny, nz;
} WCtx;

static int wrap(int i, int n) { return ((i % n) + n) % n; }

static size_t ID(const WCtx* c, int i, int j, int k) {
    return ((size_t)k * c->ny + wrap(j, c->ny)) * c->nx + wrap(i, c->nx);
}

static int cvplane(const WCtx* c, int inst, int k) {
    if (inst == 3) return k >= 1 && k <= c->nz - 1;
    return k >= 0 && k <= c->nz - 1;
}

static double GQ(const WCtx* c, int inst, int q, int i, int j, int k) {
    return c->geo[inst][(size_t)q * c->NI + ID(c, i, j, k)];
}

static double WQ(const WCtx* c, int inst, int q, int i, int j, int k) {
    return c->w[inst][(size_t)q * c->NI + ID(c, i, j, k)];
}

static void WSET(const WCtx* c, int inst, int q, int i, int j, int k, double v) {
    c->w[inst][(size_t)q * c->NI + ID(c, i, j, k)] = v;
}

/* fluid CV test: on a CV plane and alpha > 0 */
static int fluid(const WCtx* c, int inst, int i, int j, int k) {
    if (!cvplane(c, inst, k)) return 0;
    return GQ(c, inst, OQ_ALPHA, i, j, k) > 0.0;
}

static int bit_of(int ox, int oy, int oz) { return (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1); }

static int in_mask(double maskd, int ox, int oy, int oz) {
    const long m = (long)maskd;
    return (int)((m >> bit_of(ox, oy, oz)) & 1L);
}

/* ----------------------------------------------------------------- setup */

static void merge_one(const WCtx* c, int inst, int i, int j, int k) {
    const orc_grid* g = c->g;
    const double dv = g->dx[0] * g->dx[1] * g->dx[2];
    const double vt = g->small_vfrac * dv;
    /* EB normal (into the fluid) in physical units */
    const double n[3] = {GQ(c, inst, OQ_AX, i, j, k) * g->dx[1] * g->dx[2],
                         GQ(c, inst, OQ_AY, i, j, k) * g->dx[0] * g->dx[2],
                         GQ(c, inst, OQ_AZ, i, j, k) * g->dx[0] * g->dx[1]};
    double mx = 0.0;
    for (int d = 0; d < 3; ++d) mx = fmax(mx, fabs(n[d]));
    const double tol = TIE * mx;
    /* axis order: largest |n_d| first, ties to the lower axis */
    int order[3], used[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r) {
        double best = -1.0;
        for (int d = 0; d < 3; ++d)
            if (!used[d]) best = fmax(best, fabs(n[d]));
        for (int d = 0; d < 3; ++d) {
            if (!used[d] && fabs(n[d]) >= best - tol) {
                order[r] = d;
                used[d] = 1;
                break;
            }
        }
    }
    int sg[3];
    for (int d = 0; d < 3; ++d) sg[d] = (n[d] < -tol) ? -1 : 1;
    long mask = 1L << bit_of(0, 0, 0);
    double vsum = GQ(c, inst, OQ_ALPHA, i, j, k) * dv;
    int tier = 0;
    for (int t = 1; t <= 3; ++t) {
        tier = t;
        /* block spanned by the first t axes of the order */
        const int lim[3] = {t >= 1, t >= 2, t >= 3};
        for (int a = 0; a <= lim[0]; ++a)
            for (int b = 0; b <= lim[1]; ++b)
                for (int e = 0; e <= lim[2]; ++e) {
                    int o[3] = {0, 0, 0};
                    o[order[0]] += a * sg[order[0]];
                    o[order[1]] += b * sg[order[1]];
                    o[order[2]] += e * sg[order[2]];
                    const int bt = bit_of(o[0], o[1], o[2]);
                    if ((mask >> bt) & 1L) continue;
                    if (!fluid(c, inst, i + o[0], j + o[1], k + o[2])) continue;
                    mask |= 1L << bt;
                    vsum += GQ(c, inst, OQ_ALPHA, i + o[0], j + o[1], k + o[2]) * dv;
                }
        if (vsum >= vt * (1.0 - TIE)) break;
    }
    WSET(c, inst, OW_TIER, i, j, k, (double)tier);
    WSET(c, inst, OW_MASK, i, j, k, (double)mask);
}

int orc_wsrd_setup(const orc_grid* g, double* const geo[4], double* const w[4]) {
    WCtx c = {g, geo, w, 0, g->n[0], g->n[1], g->n[2]};
    c.NI = (size_t)(c.nz + 1) * c.ny * c.nx;
    const double dv = g->dx[0] * g->dx[1] * g->dx[2];
    const double vt = g->small_vfrac * dv;
    for (int inst = 0; inst < 4; ++inst) {
        memset(w[inst], 0, sizeof(double) * OW_N * c.NI);
        /* small flags and neighbourhoods M */
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    if (!fluid(&c, inst, i, j, k)) continue;
                    const double a = GQ(&c, inst, OQ_ALPHA, i, j, k);
                    const int small = a < g->small_vfrac * (1.0 - TIE);
                    WSET(&c, inst, OW_SMALL, i, j, k, small);
                    if (small) {
                        merge_one(&c, inst, i, j, k);
                    } else {
                        WSET(&c, inst, OW_MASK, i, j, k, (double)(1L << bit_of(0, 0, 0)));
                    }
                }
        /* N = |W| */
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    if (!fluid(&c, inst, i, j, k)) continue;
                    int cnt = 0;
                    for (int oz = -1; oz <= 1; ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                const int ri = i - ox, rj = j - oy, rk = k - oz;
                                if (!fluid(&c, inst, ri, rj, rk)) continue;
                                if (in_mask(WQ(&c, inst, OW_MASK, ri, rj, rk), ox, oy, oz)) ++cnt;
                            }
                    WSET(&c, inst, OW_NCOUNT, i, j, k, (double)cnt);
                }
        /* kappa */
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    if (!fluid(&c, inst, i, j, k)) continue;
                    const double V = GQ(&c, inst, OQ_ALPHA, i, j, k) * dv;
                    double kap = 0.0;
                    if (WQ(&c, inst, OW_SMALL, i, j, k) > 0.0 && V < vt) {
                        double s = 0.0;
                        const double m = WQ(&c, inst, OW_MASK, i, j, k);
                        for (int oz = -1; oz <= 1; ++oz)
                            for (int oy = -1; oy <= 1; ++oy)
                                for (int ox = -1; ox <= 1; ++ox) {
                                    if (ox == 0 && oy == 0 && oz == 0) continue;
                                    if (!in_mask(m, ox, oy, oz)) continue;
                                    s += GQ(&c, inst, OQ_ALPHA, i + ox, j + oy, k + oz) * dv;
                                }
                        if (s > 0.0) kap = fmin(1.0, (vt - V) / s);
                    }
                    WSET(&c, inst, OW_KAPPA, i, j, k, kap);
                }
        /* omega, V-hat, x-hat */
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    if (!fluid(&c, inst, i, j, k)) continue;
                    const double Ni = WQ(&c, inst, OW_NCOUNT, i, j, k);
                    double ks = 0.0;
                    for (int oz = -1; oz <= 1; ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                if (ox == 0 && oy == 0 && oz == 0) continue;
                                const int ri = i - ox, rj = j - oy, rk = k - oz;
                                if (!fluid(&c, inst, ri, rj, rk)) continue;
                                if (in_mask(WQ(&c, inst, OW_MASK, ri, rj, rk), ox, oy, oz))
                                    ks += WQ(&c, inst, OW_KAPPA, ri, rj, rk);
                            }
                    const double om = 1.0 - ks / Ni;
                    WSET(&c, inst, OW_OMEGA, i, j, k, om);
                }
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    if (!fluid(&c, inst, i, j, k)) continue;
                    const double V = GQ(&c, inst, OQ_ALPHA, i, j, k) * dv;
                    const double om = WQ(&c, inst, OW_OMEGA, i, j, k);
                    const double kap = WQ(&c, inst, OW_KAPPA, i, j, k);
                    const double m = WQ(&c, inst, OW_MASK, i, j, k);
                    double vh = om * V;
                    double xs[3];
                    for (int d = 0; d < 3; ++d) xs[d] = om * V * GQ(&c, inst, OQ_VCX + d, i, j, k);
                    for (int oz = -1; oz <= 1; ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                if (ox == 0 && oy == 0 && oz == 0) continue;
                                if (!in_mask(m, ox, oy, oz)) continue;
                                const double Vr = GQ(&c, inst, OQ_ALPHA, i + ox, j + oy, k + oz) * dv;
                                const double Nr = WQ(&c, inst, OW_NCOUNT, i + ox, j + oy, k + oz);
                                const int o[3] = {ox, oy, oz};
                                vh += kap * Vr / Nr;
                                for (int d = 0; d < 3; ++d)
                                    xs[d] += kap * Vr / Nr *
                                             (o[d] + GQ(&c, inst, OQ_VCX + d, i + ox, j + oy, k + oz));
                            }
                    WSET(&c, inst, OW_VHAT, i, j, k, vh / dv);
                    for (int d = 0; d < 3; ++d) WSET(&c, inst, OW_XHX + d, i, j, k, xs[d] / vh);
                }
    }
    return 0;
}

/* ----------------------------------------------------------------- apply */

/* Solve the 3x3 system A s = b by Gauss-Jordan elimination with partial
 * pivoting, also returning the 1-norm reciprocal condition number.  Returns 0
 * if singular. */
static int solve3(const double Ain[3][3], const double bin[3], double s[3], double* rcond) {
    double A[3][3], Inv[3][3], b[3];
    for (int r = 0; r < 3; ++r) {
        b[r] = bin[r];
        for (int q = 0; q < 3; ++q) {
            A[r][q] = Ain[r][q];
            Inv[r][q] = (r == q) ? 1.0 : 0.0;
        }
    }
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (!(fabs(A[piv][col]) > 0.0)) return 0;
        if (piv != col) {
            for (int q = 0; q < 3; ++q) {
                double t = A[col][q]; A[col][q] = A[piv][q]; A[piv][q] = t;
                t = Inv[col][q]; Inv[col][q] = Inv[piv][q]; Inv[piv][q] = t;
            }
            double t = b[col]; b[col] = b[piv]; b[piv] = t;
        }
        const double p = A[col][col];
        for (int q = 0; q < 3; ++q) { A[col][q] /= p; Inv[col][q] /= p; }
        b[col] /= p;
        for (int r = 0; r < 3; ++r) {
            if (r == col) continue;
            const double f = A[r][col];
            for (int q = 0; q < 3; ++q) { A[r][q] -= f * A[col][q]; Inv[r][q] -= f * Inv[col][q]; }
            b[r] -= f * b[col];
        }
    }
    double n1 = 0.0, ni = 0.0;
    for (int q = 0; q < 3; ++q) {
        double ca = 0.0, cb = 0.0;
        for (int r = 0; r < 3; ++r) { ca += fabs(Ain[r][q]); cb += fabs(Inv[r][q]); }
        n1 = fmax(n1, ca);
        ni = fmax(ni, cb);
    }
    *rcond = 1.0 / (n1 * ni);
    for (int r = 0; r < 3; ++r) s[r] = b[r];
    return 1;
}

typedef struct {
    int n;
    double d[125][3]; /* centroid offsets from x-hat_i, in mesh units */
    double q[125];
} Pts;

static void gather_pts(const WCtx* c, int inst, const double* Qh, int i, int j, int k,
                       const int wd[3], Pts* P) {
    P->n = 0;
    for (int oz = -wd[2]; oz <= wd[2]; ++oz)
        for (int oy = -wd[1]; oy <= wd[1]; ++oy)
            for (int ox = -wd[0]; ox <= wd[0]; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                if (!fluid(c, inst, i + ox, j + oy, k + oz)) continue;
                const int o[3] = {ox, oy, oz};
                for (int d = 0; d < 3; ++d)
                    P->d[P->n][d] = o[d] + WQ(c, inst, OW_XHX + d, i + ox, j + oy, k + oz) -
                                    WQ(c, inst, OW_XHX + d, i, j, k);
                P->q[P->n] = Qh[ID(c, i + ox, j + oy, k + oz)];
                P->n++;
            }
}

static double psi(double delta, double qi, double qmin, double qmax) {
    if (delta > 0.0) return fmin(1.0, (qmax - qi) / delta);
    if (delta < 0.0) return fmin(1.0, (qmin - qi) / delta);
    return 1.0;
}

/* gradient (physical units) of Q-hat for a small CV */
static void gradient(const WCtx* c, int inst, const double* Qh, int i, int j, int k, double sig[3]) {
    const double* del = c->g->dx;
    sig[0] = sig[1] = sig[2] = 0.0;
    int wd[3] = {1, 1, 1};
    Pts P;
    gather_pts(c, inst, Qh, i, j, k, wd, &P);
    double spread[3] = {0, 0, 0};
    for (int s = 0; s < P.n; ++s)
        for (int d = 0; d < 3; ++d) spread[d] = fmax(spread[d], fabs(P.d[s][d]));
    int widened = 0;
    for (int d = 0; d < 3; ++d)
        if (spread[d] < 0.5 * (1.0 - TIE)) { wd[d] = 2; widened = 1; }
    if (widened) {
        gather_pts(c, inst, Qh, i, j, k, wd, &P);
        spread[0] = spread[1] = spread[2] = 0.0;
        for (int s = 0; s < P.n; ++s)
            for (int d = 0; d < 3; ++d) spread[d] = fmax(spread[d], fabs(P.d[s][d]));
    }
    if (P.n < 3) return;
    for (int d = 0; d < 3; ++d)
        if (spread[d] < 0.5 * (1.0 - TIE)) return;
    const double qi = Qh[ID(c, i, j, k)];
    double A[3][3] = {{0}}, b[3] = {0};
    for (int s = 0; s < P.n; ++s)
        for (int r = 0; r < 3; ++r) {
            b[r] += P.d[s][r] * (P.q[s] - qi);
            for (int q = 0; q < 3; ++q) A[r][q] += P.d[s][r] * P.d[s][q];
        }
    double sol[3], rc;
    if (!solve3(A, b, sol, &rc)) return;
    if (!(rc >= 1e-10)) return;
    double qmin = qi, qmax = qi;
    for (int s = 0; s < P.n; ++s) { qmin = fmin(qmin, P.q[s]); qmax = fmax(qmax, P.q[s]); }
    /* evaluation points: centroids of the members of M_i, relative to x-hat_i */
    const double m = WQ(c, inst, OW_MASK, i, j, k);
    double ev[8][3];
    int ne = 0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (!in_mask(m, ox, oy, oz)) continue;
                const int o[3] = {ox, oy, oz};
                for (int d = 0; d < 3; ++d)
                    ev[ne][d] = o[d] + GQ(c, inst, OQ_VCX + d, i + ox, j + oy, k + oz) -
                                WQ(c, inst, OW_XHX + d, i, j, k);
                ++ne;
            }
    const int lim = c->g->limiter;
    if (lim == 0) {
        for (int d = 0; d < 3; ++d) {
            double l = 1.0;
            for (int e = 0; e < ne; ++e) l = fmin(l, psi(sol[d] * ev[e][d], qi, qmin, qmax));
            sol[d] *= l;
        }
    } else if (lim == 1) {
        double l = 1.0;
        for (int e = 0; e < ne; ++e)
            l = fmin(l, psi(sol[0] * ev[e][0] + sol[1] * ev[e][1] + sol[2] * ev[e][2], qi, qmin,
                            qmax));
        for (int d = 0; d < 3; ++d) sol[d] *= l;
    }
    for (int d = 0; d < 3; ++d) sig[d] = sol[d] / del[d];
}

static int redistribute_impl(const orc_grid* g, double* const geo[4], double* const w[4],
                             const double* const Uhat[5], double* const Uout[5],
                             double* const sig_out[5], double* const qhat_out[5]) {
    static const int FI[5] = {0, 0, 1, 2, 3};
    WCtx c = {g, geo, w, 0, g->n[0], g->n[1], g->n[2]};
    c.NI = (size_t)(c.nz + 1) * c.ny * c.nx;
    const double dv = g->dx[0] * g->dx[1] * g->dx[2];
    const double* del = g->dx;
    double* Qh = (double*)calloc(c.NI, sizeof(double));
    double* sg = (double*)calloc(3 * c.NI, sizeof(double));
    for (int f = 0; f < 5; ++f) {
        const int inst = FI[f];
        const double* U = Uhat[f];
        /* Q-hat */
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    const size_t id = ID(&c, i, j, k);
                    Qh[id] = 0.0;
                    if (!fluid(&c, inst, i, j, k)) continue;
                    const double kap = WQ(&c, inst, OW_KAPPA, i, j, k);
                    if (!(kap > 0.0)) {
                        Qh[id] = U[id]; /* single-cell neighbourhood: Q-hat = U-hat */
                        continue;
                    }
                    const double V = GQ(&c, inst, OQ_ALPHA, i, j, k) * dv;
                    const double om = WQ(&c, inst, OW_OMEGA, i, j, k);
                    const double m = WQ(&c, inst, OW_MASK, i, j, k);
                    double s = om * V * U[id];
                    for (int oz = -1; oz <= 1; ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                if (ox == 0 && oy == 0 && oz == 0) continue;
                                if (!in_mask(m, ox, oy, oz)) continue;
                                const double Vr =
                                    GQ(&c, inst, OQ_ALPHA, i + ox, j + oy, k + oz) * dv;
                                const double Nr = WQ(&c, inst, OW_NCOUNT, i + ox, j + oy, k + oz);
                                s += kap * Vr / Nr * U[ID(&c, i + ox, j + oy, k + oz)];
                            }
                    Qh[id] = s / (WQ(&c, inst, OW_VHAT, i, j, k) * dv);
                }
        /* gradients of small CVs with |M| >= 2 */
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    const size_t id = ID(&c, i, j, k);
                    sg[3 * id] = sg[3 * id + 1] = sg[3 * id + 2] = 0.0;
                    if (!fluid(&c, inst, i, j, k)) continue;
                    if (!(WQ(&c, inst, OW_SMALL, i, j, k) > 0.0)) continue;
                    const long m = (long)WQ(&c, inst, OW_MASK, i, j, k);
                    if (m == (1L << bit_of(0, 0, 0))) continue;
                    gradient(&c, inst, Qh, i, j, k, &sg[3 * id]);
                }
        /* final update */
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    const size_t id = ID(&c, i, j, k);
                    if (!fluid(&c, inst, i, j, k)) {
                        Uout[f][id] = 0.0;
                        continue;
                    }
                    const double om = WQ(&c, inst, OW_OMEGA, i, j, k);
                    const double Ni = WQ(&c, inst, OW_NCOUNT, i, j, k);
                    /* q-hat_i at x_i */
                    double qi = Qh[id];
                    for (int d = 0; d < 3; ++d)
                        qi += sg[3 * id + d] *
                              (GQ(&c, inst, OQ_VCX + d, i, j, k) - WQ(&c, inst, OW_XHX + d, i, j, k)) *
                              del[d];
                    double s = 0.0;
                    for (int oz = -1; oz <= 1; ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                if (ox == 0 && oy == 0 && oz == 0) continue;
                                const int ri = i - ox, rj = j - oy, rk = k - oz;
                                if (!fluid(&c, inst, ri, rj, rk)) continue;
                                if (!in_mask(WQ(&c, inst, OW_MASK, ri, rj, rk), ox, oy, oz)) continue;
                                const size_t rid = ID(&c, ri, rj, rk);
                                const int o[3] = {ox, oy, oz};
                                double qr = Qh[rid];
                                for (int d = 0; d < 3; ++d)
                                    qr += sg[3 * rid + d] *
                                          (o[d] + GQ(&c, inst, OQ_VCX + d, i, j, k) -
                                           WQ(&c, inst, OW_XHX + d, ri, rj, rk)) *
                                          del[d];
                                s += WQ(&c, inst, OW_KAPPA, ri, rj, rk) * qr;
                            }
                    Uout[f][id] = om * qi + s / Ni;
                }
        if (sig_out && sig_out[f]) memcpy(sig_out[f], sg, sizeof(double) * 3 * c.NI);
        if (qhat_out && qhat_out[f]) memcpy(qhat_out[f], Qh, sizeof(double) * c.NI);
    }
    free(Qh);
    free(sg);
    return 0;
}

int orc_redistribute(const orc_grid* g, double* const geo[4], double* const w[4],
                     const double* const Uhat[5], double* const Uout[5]) {
    return redistribute_impl(g, geo, w, Uhat, Uout, NULL, NULL);
}

int orc_redistribute_sig(const orc_grid* g, double* const geo[4], double* const w[4],
                         const double* const Uhat[5], double* const Uout[5],
                         double* const sig[5]) {
    return redistribute_impl(g, geo, w, Uhat, Uout, sig, NULL);
}

int orc_redistribute_diag(const orc_grid* g, double* const geo[4], double* const w[4],
                          const double* const Uhat[5], double* const Uout[5], double* const sig[5],
                          double* const qhat[5]) {
    return redistribute_impl(g, geo, w, Uhat, Uout, sig, qhat);
}
