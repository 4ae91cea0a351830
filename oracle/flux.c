/*
 * Oracle flux divergence and explicit stage update (TEST INFRASTRUCTURE ONLY;
 * see oracle.h).
 *
 * Follows Section 3.1 (Eqs. update-cc and update-fc: the update of a cell- or
 * face-centred quantity is minus the area-fraction weighted flux difference
 * divided by the volume fraction, plus the EB flux term) and Section 4.1 (the
 * advective flux rho u (x) phi, third-order upwind written as fourth-order
 * centred plus a hyperviscous term, reduced to second-order centred when the
 * upstream cell is covered, and moved to the cut-face centroid by bilinear
 * interpolation of provisional fluxes; zero normal convective flux at walls).
 * The source term is zero (Section 3.1).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - the mass flux that advects a momentum on a staggered face is the mean
 *    of the two stored face momenta next to it over those whose control
 *    volume holds fluid (one such: its value);
 *  - face velocities are the face momentum divided by the mean density of the
 *    fluid cells on either side; theta = (rho theta) / rho;
 *  - the "upstream cell" is the far end of the upwind three-point stencil; it
 *    counts as covered when its volume fraction is zero or it lies outside a
 *    wall (periodic directions wrap);
 *  - the interpolation neighbours are chosen by the signs of the face-centroid
 *    offsets; the weights are the absolute offsets; if a needed neighbour face
 *    has no fluid or lies outside a wall the provisional flux is used as is;
 *  - the momentum flux of the z-face instance through the mid planes of the
 *    bottom and top cell layers is zero (those planes border the wall faces,
 *    which hold the Dirichlet value 0 and are not control volumes);
 *  - the EB flux is zero (no-flux wall).  A test-only closure mode sets it to
 *    minus (area vector) . (mean provisional flux of the CV), under which any
 *    uniform flow must be steady.
 */
#include "oracle.h"

#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const orc_grid* g;
    double* const* geo;
    size_t NI;
    int nx, ny, nz;
} FCtx;

static int wrapi(int i, int n) { return ((i % n) + n) % n; }

static size_t IDX(const FCtx* c, int i, int j, int k) {
    return ((size_t)k * c->ny + wrapi(j, c->ny)) * c->nx + wrapi(i, c->nx);
}

/* is plane k a control-volume plane of instance inst */
static int is_cv(const FCtx* c, int inst, int k) {
    if (inst == 3) return k >= 1 && k <= c->nz - 1;
    return k >= 0 && k <= c->nz - 1;
}

/* is plane k a plane on which the instance stores lower-face data */
static int has_face_plane(const FCtx* c, int inst, int k) {
    if (inst == 3) return k >= 1 && k <= c->nz;
    return k >= 0 && k <= c->nz;
}

static double G(const FCtx* c, int inst, int q, int i, int j, int k) {
    if (k < 0 || k > c->nz) return 0.0;
    return c->geo[inst][(size_t)q * c->NI + IDX(c, i, j, k)];
}

static double alpha(const FCtx* c, int inst, int i, int j, int k) {
    if (!is_cv(c, inst, k)) return 0.0;
    return G(c, inst, OQ_ALPHA, i, j, k);
}

/* state value with non-fluid entries read as zero */
static double sval(const FCtx* c, const double* f, int inst, int i, int j, int k) {
    if (alpha(c, inst, i, j, k) > 0.0) return f[IDX(c, i, j, k)];
    return 0.0;
}

static const int FIELD_INST[5] = {0, 0, 1, 2, 3};

/* Diagnostics: theta on cells, velocities on faces (zero where not fluid). */
static void diagnostics(const FCtx* c, const double* const U[5], double* th, double* vel[3]) {
    const int nx = c->nx, ny = c->ny, nz = c->nz;
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t id = IDX(c, i, j, k);
                th[id] = 0.0;
                if (alpha(c, 0, i, j, k) > 0.0) th[id] = U[1][id] / U[0][id];
                for (int d = 0; d < 3; ++d) {
                    vel[d][id] = 0.0;
                    if (!(alpha(c, d + 1, i, j, k) > 0.0)) continue;
                    /* the two cells sharing this face */
                    int i0 = i, j0 = j, k0 = k;
                    if (d == 0) i0 = i - 1;
                    if (d == 1) j0 = j - 1;
                    if (d == 2) k0 = k - 1;
                    double s = 0.0;
                    int cnt = 0;
                    if (alpha(c, 0, i0, j0, k0) > 0.0) { s += U[0][IDX(c, i0, j0, k0)]; ++cnt; }
                    if (alpha(c, 0, i, j, k) > 0.0) { s += U[0][id]; ++cnt; }
                    if (cnt > 0) vel[d][id] = U[2 + d][id] / (s / cnt);
                }
            }
}

typedef struct {
    const FCtx* c;
    const double* const* U;
    const double* th;
    double* const* vel;
} Diag;

/* advected quantity phi of `field` at CV (i,j,k) of its instance */
static double phi(const Diag* D, int field, int i, int j, int k) {
    const FCtx* c = D->c;
    const int inst = FIELD_INST[field];
    if (!is_cv(c, inst, k)) return 0.0;
    if (!(alpha(c, inst, i, j, k) > 0.0)) return 0.0;
    const size_t id = IDX(c, i, j, k);
    switch (field) {
        case 0: return 1.0;
        case 1: return D->th[id];
        default: return D->vel[field - 2][id];
    }
}

/* mass flux through the lower d-face of CV (i,j,k) of instance inst */
static double mass_flux(const Diag* D, int inst, int d, int i, int j, int k) {
    const FCtx* c = D->c;
    const double* mom = D->U[2 + d];
    const int minst = d + 1; /* instance on which the d-momentum lives */
    if (inst == 0) return sval(c, mom, minst, i, j, k);
    /* staggered instances: the face is made of two halves, one in each of the
     * two face momenta adjacent to it (offset by one cell in the instance's
     * own direction); the mass flux is the mean of those momenta over the
     * ones whose CV holds fluid (the half of a covered one is closed, and the
     * area fraction already accounts for it) */
    const int s = inst - 1;
    int i0 = i, j0 = j, k0 = k;
    if (s == 0) i0 = i - 1;
    if (s == 1) j0 = j - 1;
    if (s == 2) k0 = k - 1;
    const int fa = alpha(c, minst, i0, j0, k0) > 0.0, fb = alpha(c, minst, i, j, k) > 0.0;
    const double sum = sval(c, mom, minst, i0, j0, k0) + sval(c, mom, minst, i, j, k);
    if (fa && fb) return 0.5 * sum;
    return sum; /* one fluid CV: its momentum; none: 0 */
}

/* provisional flux on the lower d-face of CV p=(i,j,k) of the field's instance */
static double fhat(const Diag* D, int field, int d, int i, int j, int k) {
    const FCtx* c = D->c;
    const int inst = FIELD_INST[field];
    /* walls: no convective flux through the domain bottom/top, nor (z-face
     * instance) through the mid planes of the bottom and top cell layers */
    if (d == 2) {
        if (inst != 3 && (k == 0 || k == c->nz)) return 0.0;
        if (inst == 3 && (k == 1 || k == c->nz)) return 0.0;
    }
    const double m = mass_flux(D, inst, d, i, j, k);
    if (field == 0) return m;
    int o[3] = {0, 0, 0};
    o[d] = 1;
    const double pLL = phi(D, field, i - 2 * o[0], j - 2 * o[1], k - 2 * o[2]);
    const double pL = phi(D, field, i - o[0], j - o[1], k - o[2]);
    const double pR = phi(D, field, i, j, k);
    const double pRR = phi(D, field, i + o[0], j + o[1], k + o[2]);
    /* upstream end of the upwind stencil */
    const int up = (m >= 0.0) ? -2 : 1;
    const double aE = alpha(c, inst, i + up * o[0], j + up * o[1], k + up * o[2]);
    double pf;
    if (!(aE > 0.0)) {
        pf = 0.5 * (pL + pR); /* second-order centred */
    } else {
        const double sg = (m >= 0.0) ? 1.0 : -1.0;
        /* fourth-order centred plus hyperviscosity = third-order upwind */
        pf = (7.0 * (pL + pR) - (pLL + pRR)) / 12.0 + sg * ((pRR - pLL) - 3.0 * (pR - pL)) / 12.0;
    }
    return m * pf;
}

/* side of a face-centroid offset (mesh units); offsets within 1e-12 of zero
 * count as none: a face cut by a vertical wall has its centroid at
 * mid-height, which rounding puts a few 1e-17 to either side */
static int sgn0(double x) { return x > 1e-12 ? 1 : (x < -1e-12 ? -1 : 0); }

/* flux used in the divergence on the lower d-face of CV (i,j,k) */
static double face_flux(const Diag* D, int field, int d, int i, int j, int k) {
    const FCtx* c = D->c;
    const int inst = FIELD_INST[field];
    const int qb = OQ_BX + d, qf = OQ_FX1 + 2 * d;
    const double beta = G(c, inst, qb, i, j, k);
    if (!(beta > 0.0)) return 0.0;
    const double F0 = fhat(D, field, d, i, j, k);
    if (!(beta < 1.0)) return F0;
    /* cut face: bilinear interpolation toward the face-centroid offset */
    const int tang[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    const double g1 = G(c, inst, qf, i, j, k), g2 = G(c, inst, qf + 1, i, j, k);
    const int s1 = sgn0(g1), s2 = sgn0(g2);
    if (s1 == 0 && s2 == 0) return F0;
    int e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
    e1[tang[d][0]] = s1;
    e2[tang[d][1]] = s2;
    /* neighbour faces that carry weight */
    int nb[3][3];
    int use[3] = {s1 != 0, s2 != 0, s1 != 0 && s2 != 0};
    for (int a = 0; a < 3; ++a) {
        nb[0][a] = (a == 0 ? i : a == 1 ? j : k) + e1[a];
        nb[1][a] = (a == 0 ? i : a == 1 ? j : k) + e2[a];
        nb[2][a] = (a == 0 ? i : a == 1 ? j : k) + e1[a] + e2[a];
    }
    for (int q = 0; q < 3; ++q) {
        if (!use[q]) continue;
        /* a neighbour shifted in z must lie on a CV plane of the instance;
         * shifts within the same plane stay inside (periodic x, y) */
        if (nb[q][2] != k && !is_cv(c, inst, nb[q][2])) return F0;
        if (!(G(c, inst, qb, nb[q][0], nb[q][1], nb[q][2]) > 0.0)) return F0;
    }
    const double w1 = s1 ? fabs(g1) : 0.0, w2 = s2 ? fabs(g2) : 0.0;
    double F = (1.0 - w1) * (1.0 - w2) * F0;
    if (use[0]) F += w1 * (1.0 - w2) * fhat(D, field, d, nb[0][0], nb[0][1], nb[0][2]);
    if (use[1]) F += (1.0 - w1) * w2 * fhat(D, field, d, nb[1][0], nb[1][1], nb[1][2]);
    if (use[2]) F += w1 * w2 * fhat(D, field, d, nb[2][0], nb[2][1], nb[2][2]);
    return F;
}

static void setup(FCtx* c, const orc_grid* g, double* const geo[4]) {
    c->g = g;
    c->geo = geo;
    c->nx = g->n[0];
    c->ny = g->n[1];
    c->nz = g->n[2];
    c->NI = (size_t)(c->nz + 1) * c->ny * c->nx;
}

int orc_advance(const orc_grid* g, double* const geo[4], const double* const Un[5],
                const double* const Ucur[5], double* const Uhat[5], double cdt) {
    FCtx c;
    setup(&c, g, geo);
    const size_t NI = c.NI;
    double* th = (double*)calloc(NI, sizeof(double));
    double* vel[3];
    for (int d = 0; d < 3; ++d) vel[d] = (double*)calloc(NI, sizeof(double));
    diagnostics(&c, Ucur, th, vel);
    Diag D = {&c, Ucur, th, vel};
    const double del[3] = {g->dx[0], g->dx[1], g->dx[2]};
    for (int field = 0; field < 5; ++field) {
        const int inst = FIELD_INST[field];
#pragma omp parallel for schedule(dynamic, 1)
        for (int k = 0; k <= c.nz; ++k)
            for (int j = 0; j < c.ny; ++j)
                for (int i = 0; i < c.nx; ++i) {
                    const size_t id = IDX(&c, i, j, k);
                    const double a = alpha(&c, inst, i, j, k);
                    if (!(a > 0.0)) {
                        Uhat[field][id] = 0.0;
                        continue;
                    }
                    double bracket = 0.0;
                    double fbar[3];
                    for (int d = 0; d < 3; ++d) {
                        const int ip = i + (d == 0), jp = j + (d == 1), kp = k + (d == 2);
                        const double blo = G(&c, inst, OQ_BX + d, i, j, k);
                        const double bhi = G(&c, inst, OQ_BX + d, ip, jp, kp);
                        const double Flo = face_flux(&D, field, d, i, j, k);
                        const double Fhi = face_flux(&D, field, d, ip, jp, kp);
                        bracket += (bhi * Fhi - blo * Flo) / del[d];
                        /* mean provisional flux over the CV's fluid d-faces */
                        double s = 0.0;
                        int cnt = 0;
                        if (blo > 0.0) { s += fhat(&D, field, d, i, j, k); ++cnt; }
                        if (bhi > 0.0) { s += fhat(&D, field, d, ip, jp, kp); ++cnt; }
                        fbar[d] = cnt ? s / cnt : 0.0;
                    }
                    if (g->eb_flux == 1) {
                        /* A^EB F^EB / V_cell with F^EB the outward normal flux
                         * -n . Fbar; the stored area vector is normalised per
                         * face area, so a_d / (dx dy dz) = ahat_d / dx_d */
                        for (int d = 0; d < 3; ++d)
                            bracket -= G(&c, inst, OQ_AX + d, i, j, k) * fbar[d] / del[d];
                    }
                    const double dU = -bracket / a;
                    Uhat[field][id] = sval(&c, Un[field], inst, i, j, k) + cdt * dU;
                }
    }
    free(th);
    for (int d = 0; d < 3; ++d) free(vel[d]);
    return 0;
}

int orc_face_fluxes(const orc_grid* g, double* const geo[4], const double* const U[5], int field,
                    double* const F[3], double* const Fhat[3]) {
    FCtx c;
    setup(&c, g, geo);
    const size_t NI = c.NI;
    double* th = (double*)calloc(NI, sizeof(double));
    double* vel[3];
    for (int d = 0; d < 3; ++d) vel[d] = (double*)calloc(NI, sizeof(double));
    diagnostics(&c, U, th, vel);
    Diag D = {&c, U, th, vel};
    const int inst = FIELD_INST[field];
    for (int k = 0; k <= c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                const size_t id = IDX(&c, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    const int ok = (d == 2) ? has_face_plane(&c, inst, k) : is_cv(&c, inst, k);
                    F[d][id] = ok ? face_flux(&D, field, d, i, j, k) : 0.0;
                    Fhat[d][id] = ok ? fhat(&D, field, d, i, j, k) : 0.0;
                }
            }
    free(th);
    for (int d = 0; d < 3; ++d) free(vel[d]);
    return 0;
}

/* Threads of the parallel plane loops (n > 0 sets them); returns the number
 * in use.  Every loop writes only the entries of its own plane, so results
 * do not depend on the count. */
int orc_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}
