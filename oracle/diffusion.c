/*
 * Oracle thermal diffusion of rho theta with least-squares gradients at cut
 * faces and EB facets (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Follows Section 4.2 of the paper: the diffusive flux of rho theta is
 * rho alpha_theta grad(theta) (Eq. theta-comp); on cut faces and at the EB
 * the gradient comes from a least-squares fit of a second-order polynomial
 * to the state over a local neighbourhood of cells, 3 wide when the gradient
 * is taken on the variable's own grid (the EB facet centroid of a cell) and
 * 4 wide along the direction in which the evaluation point sits between two
 * cells (a face centroid), to keep the stencil symmetric.
 *
 * Readings where the paper is silent (also listed in the design notes):
 *  - full faces use the centred difference of theta between the two cells;
 *    cut faces take the normal component of the fitted gradient at the face
 *    centroid; a face counts as full when beta >= 1 - 1e-12, so that the
 *    last-bit rounding of two geometry builders (a face that the terrain only
 *    touches) cannot switch the gradient method;
 *  - the fit is unweighted; the points are the fluid cells of the stencil at
 *    their volume centroids with theta = (rho theta) / rho; the polynomial is
 *    quadratic (1, dx, dy, dz, the three squares, the three products, in
 *    mesh units about the evaluation point); with fewer than 10 points or a
 *    reciprocal condition number of the normal matrix below 1e-7 the fit
 *    falls back to linear, and with fewer than 4 points or the linear normal
 *    matrix as poorly conditioned the gradient is zero (a nearly degenerate
 *    point set would amplify the rounding of theta by the inverse of that
 *    number);
 *  - the EB is adiabatic (zero diffusive flux) or isothermal at theta_wall:
 *    then the fit at the facet centroid is constrained to take the value
 *    theta_wall there (no constant term), 3 x 3 x 3 cells around the cut cell
 *    including itself, 9 quadratic terms, linear fallback with 3;
 *  - the density on a face is the mean over the fluid cells on either side,
 *    on the EB the cut cell's own;
 *  - the domain bottom and top are adiabatic walls; x and y are periodic;
 *  - the result is intensive: D = (1 / V) times the sum over the CV's faces
 *    and facet of rho alpha grad(theta) . n_out times the open area.
 */
#include "oracle.h"
#include "lsq.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    const orc_grid* g;
    double* const* geo;
    const double* const* U;
    size_t NI;
    int nx, ny, nz;
} DCtx;

static int wrapd(int i, int n) { return ((i % n) + n) % n; }

static size_t DID(const DCtx* c, int i, int j, int k) {
    return ((size_t)k * c->ny + wrapd(j, c->ny)) * c->nx + wrapd(i, c->nx);
}

static double DG(const DCtx* c, int q, int i, int j, int k) {
    if (k < 0 || k > c->nz) return 0.0;
    return c->geo[0][(size_t)q * c->NI + DID(c, i, j, k)];
}

static int dfluid(const DCtx* c, int i, int j, int k) {
    if (k < 0 || k > c->nz - 1) return 0;
    return DG(c, OQ_ALPHA, i, j, k) > 0.0;
}

static double dtheta(const DCtx* c, int i, int j, int k) {
    const size_t id = DID(c, i, j, k);
    return c->U[1][id] / c->U[0][id];
}

static double drho(const DCtx* c, int i, int j, int k) { return c->U[0][DID(c, i, j, k)]; }

/* physical centroid of cell (i,j,k) (unwrapped indices: positions follow
 * the stencil across the periodic seams) */
static void centroid(const DCtx* c, int i, int j, int k, double p[3]) {
    const int idx[3] = {i, j, k};
    for (int d = 0; d < 3; ++d)
        p[d] = c->g->lo[d] + (idx[d] + 0.5 + DG(c, OQ_VCX + d, i, j, k)) * c->g->dx[d];
}

/* diffusive flux density rho alpha d(theta)/dx_d on the lower d-face of cell
 * (i,j,k) (both adjacent cells fluid, beta > 0) */
static double face_flux(const DCtx* c, const orc_diff* p, int d, int i, int j, int k) {
    const int o[3] = {d == 0, d == 1, d == 2};
    const int il = i - o[0], jl = j - o[1], kl = k - o[2];
    const double beta = DG(c, OQ_BX + d, i, j, k);
    const double rf = 0.5 * (drho(c, il, jl, kl) + drho(c, i, j, k));
    double g;
    if (beta >= 1.0 - 1e-12) { /* full face (tie tolerance: see the header) */
        g = (dtheta(c, i, j, k) - dtheta(c, il, jl, kl)) / c->g->dx[d];
    } else {
        /* face centroid (physical) */
        double x[3];
        const int idx[3] = {i, j, k};
        const int tang[3][2] = {{1, 2}, {0, 2}, {0, 1}};
        for (int a = 0; a < 3; ++a) x[a] = c->g->lo[a] + (idx[a] + 0.5) * c->g->dx[a];
        x[d] -= 0.5 * c->g->dx[d];
        x[tang[d][0]] += DG(c, OQ_FX1 + 2 * d, i, j, k) * c->g->dx[tang[d][0]];
        x[tang[d][1]] += DG(c, OQ_FX1 + 2 * d + 1, i, j, k) * c->g->dx[tang[d][1]];
        /* stencil: 4 cells along d (two on each side of the face), 3 across */
        double e[36][3], q[36];
        int np = 0;
        int lo[3] = {-1, -1, -1}, hi[3] = {1, 1, 1};
        lo[d] = -2;
        hi[d] = 1;
        for (int oz = lo[2]; oz <= hi[2]; ++oz)
            for (int oy = lo[1]; oy <= hi[1]; ++oy)
                for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                    if (!dfluid(c, i + ox, j + oy, k + oz)) continue;
                    double ps[3];
                    centroid(c, i + ox, j + oy, k + oz, ps);
                    for (int a = 0; a < 3; ++a) e[np][a] = (ps[a] - x[a]) / c->g->dx[a];
                    q[np] = dtheta(c, i + ox, j + oy, k + oz);
                    ++np;
                }
        double gr[3];
        lsq_gradient(c->g->dx, np, e, q, 1, gr);
        g = gr[d];
    }
    return rf * p->alpha_theta * g;
}

int orc_diffusion(const orc_grid* g, double* const geo[4], const double* const U[5], const orc_diff* p,
                  double* D, double* const Fd[3], double* Feb) {
    DCtx c = {g, geo, U, 0, g->n[0], g->n[1], g->n[2]};
    c.NI = (size_t)(c.nz + 1) * c.ny * c.nx;
    const double dv = g->dx[0] * g->dx[1] * g->dx[2];
    /* flux densities on the lower faces of every cell (0 at walls and closed faces) */
    double* F[3];
    for (int d = 0; d < 3; ++d) F[d] = (double*)calloc(c.NI, sizeof(double));
    double* E = (double*)calloc(c.NI, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k <= c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                const size_t id = DID(&c, i, j, k);
                for (int d = 0; d < 3; ++d) {
                    if (d == 2 && (k == 0 || k == c.nz)) continue; /* adiabatic walls */
                    if (d != 2 && k == c.nz) continue;
                    if (!(DG(&c, OQ_BX + d, i, j, k) > 0.0)) continue;
                    F[d][id] = face_flux(&c, p, d, i, j, k);
                }
                /* EB facet of a cut cell (isothermal wall only) */
                if (p->eb_mode == 1 && k < c.nz && dfluid(&c, i, j, k) && DG(&c, OQ_AREA, i, j, k) > 0.0) {
                    double x[3];
                    const int idx[3] = {i, j, k};
                    for (int a = 0; a < 3; ++a)
                        x[a] = g->lo[a] + (idx[a] + 0.5 + DG(&c, OQ_EBX + a, i, j, k)) * g->dx[a];
                    double e[27][3], q[27];
                    int np = 0;
                    for (int oz = -1; oz <= 1; ++oz)
                        for (int oy = -1; oy <= 1; ++oy)
                            for (int ox = -1; ox <= 1; ++ox) {
                                if (!dfluid(&c, i + ox, j + oy, k + oz)) continue;
                                double ps[3];
                                centroid(&c, i + ox, j + oy, k + oz, ps);
                                for (int a = 0; a < 3; ++a) e[np][a] = (ps[a] - x[a]) / g->dx[a];
                                q[np] = dtheta(&c, i + ox, j + oy, k + oz) - p->theta_wall;
                                ++np;
                            }
                    double gr[3];
                    lsq_gradient(g->dx, np, e, q, 0, gr);
                    /* area vector into the fluid (physical); the outward normal of
                     * the fluid CV is its opposite */
                    const double av[3] = {DG(&c, OQ_AX, i, j, k) * g->dx[1] * g->dx[2],
                                          DG(&c, OQ_AY, i, j, k) * g->dx[0] * g->dx[2],
                                          DG(&c, OQ_AZ, i, j, k) * g->dx[0] * g->dx[1]};
                    /* rho alpha grad(theta) . n_out A = -rho alpha grad . a */
                    E[id] = -drho(&c, i, j, k) * p->alpha_theta * (gr[0] * av[0] + gr[1] * av[1] + gr[2] * av[2]);
                }
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                const size_t id = DID(&c, i, j, k);
                D[id] = 0.0;
                if (!dfluid(&c, i, j, k)) continue;
                double s = 0.0;
                for (int d = 0; d < 3; ++d) {
                    const int ip = i + (d == 0), jp = j + (d == 1), kp = k + (d == 2);
                    const double fa = g->dx[0] * g->dx[1] * g->dx[2] / g->dx[d];
                    const double bl = DG(&c, OQ_BX + d, i, j, k), bh = DG(&c, OQ_BX + d, ip, jp, kp);
                    const double fh = F[d][DID(&c, ip, jp, kp)], fl = F[d][id];
                    s += (bh * fh - bl * fl) * fa;
                }
                s += E[id];
                D[id] = s / (DG(&c, OQ_ALPHA, i, j, k) * dv);
            }
    for (int d = 0; d < 3; ++d) {
        if (Fd && Fd[d]) memcpy(Fd[d], F[d], sizeof(double) * c.NI);
        free(F[d]);
    }
    if (Feb) memcpy(Feb, E, sizeof(double) * c.NI);
    free(E);
    return 0;
}
