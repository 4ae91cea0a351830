/*
 * Oracle momentum diffusion: the viscous stress on the staggered control
 * volumes (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Follows Sections 2.1 and 4.2 of the paper: the diffusive flux of momentum
 * is the viscous stress tau = lambda (div u) I + mu (grad u + grad u^T);
 * velocities live on the faces of the cells (u on x-faces, v on y-faces, w on
 * z-faces) and the stress components on the faces of the staggered control
 * volumes, tau_xx at cell centres and tau_xy, tau_xz, tau_yz at cell edges.
 * On cut faces and at the EB the gradients come from a least-squares fit of
 * a second-order polynomial over a local neighbourhood, 3 wide along an axis
 * where the evaluation point lines up with the variable's own grid and 4
 * wide where it sits between two of its points (a variable of another grid
 * type), so that the stencil stays symmetric.
 *
 * Readings where the paper is silent or garbled (also in the design notes):
 *  - lambda = -(2/3) mu (the paper prints 2/3 mu; with the minus sign the
 *    stress is the trace-free one of Stokes' hypothesis); mu constant;
 *  - velocity of a staggered CV: its momentum over the mean density of the
 *    fluid cells on either side of its face (reading F2); 0 where not fluid;
 *  - full faces (beta >= 1 - 1e-12): the centred differences of the
 *    staggered grid (tau_cc = 2 mu du_c/dx_c + lambda div u at the cell
 *    centre from the six face velocities of that cell; tau_cd = mu (du_c/dx_d
 *    + du_d/dx_c) at an edge from the two c-velocities across it in d and
 *    the two d-velocities across it in c);
 *  - cut faces (0 < beta < 1 - 1e-12): the same components from fitted
 *    gradients at the face centroid, each velocity component fitted over its
 *    own grid's fluid CVs (at their volume centroids); the stencil of a
 *    component runs 3 CVs along an axis on which the face centre lines up
 *    with that component's CV centres and 4 (two on each side) otherwise;
 *  - the fit is that of the thermal diffusion: quadratic with a linear
 *    fallback, reciprocal condition number at least 1e-7;
 *  - EB: stress-free (eb_mode 0) or no-slip (eb_mode 1): every velocity
 *    component vanishes at the facet centroid; the fits there have no
 *    constant term and the stencil rule above with the CV centre as nominal
 *    point (3 x 3 x 3 for the own component, 4 x 4 x 3 for the others); the
 *    stress acts on the facet area vector;
 *  - the domain bottom and top walls are stress-free (no diffusive momentum
 *    flux through them); x and y are periodic;
 *  - the result is intensive: D_c = (1 / V) times the sum over the CV's faces
 *    and facet of tau_c . n_out times the open area.
 */
#include "lsq.h"
#include "oracle.h"

#include <stdlib.h>
#include <string.h>

typedef struct {
    const orc_grid* g;
    double* const* geo;
    const double* const* U;
    size_t NI;
    int nx, ny, nz;
    double mu, lam;
} VCtx;

static int wrapv(int i, int n) { return ((i % n) + n) % n; }

static size_t VID(const VCtx* c, int i, int j, int k) {
    return ((size_t)k * c->ny + wrapv(j, c->ny)) * c->nx + wrapv(i, c->nx);
}

static double VG(const VCtx* c, int inst, int q, int i, int j, int k) {
    if (k < 0 || k > c->nz) return 0.0;
    return c->geo[inst][(size_t)q * c->NI + VID(c, i, j, k)];
}

/* is (i,j,k) a fluid CV of instance inst */
static int vfluid(const VCtx* c, int inst, int i, int j, int k) {
    if (inst == 3) {
        if (k < 1 || k > c->nz - 1) return 0;
    } else if (k < 0 || k > c->nz - 1) {
        return 0;
    }
    return VG(c, inst, OQ_ALPHA, i, j, k) > 0.0;
}

/* velocity component e (0 u, 1 v, 2 w) of the CV (i,j,k) of instance e + 1 */
static double vel(const VCtx* c, int e, int i, int j, int k) {
    if (!vfluid(c, e + 1, i, j, k)) return 0.0;
    const int o[3] = {e == 0, e == 1, e == 2};
    double s = 0.0;
    int n = 0;
    if (k < c->nz && VG(c, 0, OQ_ALPHA, i, j, k) > 0.0) { s += c->U[0][VID(c, i, j, k)]; ++n; }
    const int il = i - o[0], jl = j - o[1], kl = k - o[2];
    if (kl >= 0 && VG(c, 0, OQ_ALPHA, il, jl, kl) > 0.0) { s += c->U[0][VID(c, il, jl, kl)]; ++n; }
    if (!n) return 0.0;
    return c->U[2 + e][VID(c, i, j, k)] / (s / n);
}

/* physical volume centroid of CV (i,j,k) of instance inst (unwrapped
 * indices: positions follow the stencil across the periodic seams) */
static void cv_centroid(const VCtx* c, int inst, int i, int j, int k, double p[3]) {
    const int idx[3] = {i, j, k};
    for (int d = 0; d < 3; ++d) {
        const double ctr = idx[d] + 0.5 - ((inst == d + 1) ? 0.5 : 0.0);
        p[d] = c->g->lo[d] + (ctr + VG(c, inst, OQ_VCX + d, i, j, k)) * c->g->dx[d];
    }
}

/* Fitted gradient of velocity component e at physical point x, over the
 * fluid CVs of instance e + 1 in the stencil around the nominal point xn (in
 * cell units: cell (i,j,k) spans [i, i + 1)); prescribed = 1: the component
 * vanishes at x (no constant term). */
static void fit_gradient(const VCtx* c, int e, const double x[3], const double xn[3], int prescribed,
                         double grad[3]) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        /* CV centres of the component's grid along a: m + off */
        const double off = (a == e) ? 0.0 : 0.5;
        const double t = xn[a] - off;
        const double m = floor(t + 0.5);
        if (fabs(t - m) < 0.25) { /* lines up with a CV centre: 3 points */
            lo[a] = (int)m - 1;
            hi[a] = (int)m + 1;
        } else { /* between two: 2 on each side */
            const int f = (int)floor(t);
            lo[a] = f - 1;
            hi[a] = f + 2;
        }
    }
    double ev[64][3], q[64];
    int np = 0;
    for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
            for (int i = lo[0]; i <= hi[0]; ++i) {
                if (!vfluid(c, e + 1, i, j, k)) continue;
                double p[3];
                cv_centroid(c, e + 1, i, j, k, p);
                for (int a = 0; a < 3; ++a) ev[np][a] = (p[a] - x[a]) / c->g->dx[a];
                q[np] = vel(c, e, i, j, k);
                ++np;
            }
    lsq_gradient(c->g->dx, np, ev, q, !prescribed, grad);
}

/* stress tau_{cd} from a full velocity gradient G[e][a] = du_e/dx_a */
static double tau_of(const VCtx* c, double G[3][3], int cc, int d) {
    double t = c->mu * (G[cc][d] + G[d][cc]);
    if (cc == d) t += c->lam * (G[0][0] + G[1][1] + G[2][2]);
    return t;
}

/* flux density tau_{cd} on the lower d-face of the CV (i,j,k) of instance
 * cc + 1 (the face has fluid: beta > 0) */
static double face_stress(const VCtx* c, int cc, int d, int i, int j, int k) {
    const int s = cc + 1;
    const double* dx = c->g->dx;
    const double beta = VG(c, s, OQ_BX + d, i, j, k);
    const int od[3] = {d == 0, d == 1, d == 2}, oc[3] = {cc == 0, cc == 1, cc == 2};
    if (beta >= 1.0 - 1e-12) {
        if (d == cc) {
            /* cell centre of cell Q = P - e_c: the six face velocities of Q */
            const int qi = i - oc[0], qj = j - oc[1], qk = k - oc[2];
            double div = 0.0;
            for (int e = 0; e < 3; ++e) {
                const int oe[3] = {e == 0, e == 1, e == 2};
                div += (vel(c, e, qi + oe[0], qj + oe[1], qk + oe[2]) - vel(c, e, qi, qj, qk)) / dx[e];
            }
            const double dudx = (vel(c, cc, i, j, k) - vel(c, cc, qi, qj, qk)) / dx[cc];
            return 2.0 * c->mu * dudx + c->lam * div;
        }
        /* edge: c-velocities across it in d, d-velocities across it in c */
        const double a1 = (vel(c, cc, i, j, k) - vel(c, cc, i - od[0], j - od[1], k - od[2])) / dx[d];
        const double a2 = (vel(c, d, i, j, k) - vel(c, d, i - oc[0], j - oc[1], k - oc[2])) / dx[cc];
        return c->mu * (a1 + a2);
    }
    /* cut face: fitted gradients at the face centroid */
    const int idx[3] = {i, j, k};
    const int tang[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    double xn[3], x[3];
    for (int a = 0; a < 3; ++a) xn[a] = idx[a] + 0.5 - 0.5 * oc[a] - 0.5 * od[a];
    for (int a = 0; a < 3; ++a) x[a] = c->g->lo[a] + xn[a] * dx[a];
    x[tang[d][0]] += VG(c, s, OQ_FX1 + 2 * d, i, j, k) * dx[tang[d][0]];
    x[tang[d][1]] += VG(c, s, OQ_FX1 + 2 * d + 1, i, j, k) * dx[tang[d][1]];
    double G[3][3] = {{0}};
    for (int e = 0; e < 3; ++e) {
        if (d == cc || e == cc || e == d) fit_gradient(c, e, x, xn, 0, G[e]);
    }
    return tau_of(c, G, cc, d);
}

int orc_viscous(const orc_grid* g, double* const geo[4], const double* const U[5], const orc_visc* p,
                double* const D[3], double* const F[9], double* const E[3]) {
    VCtx c = {g, geo, U, 0, g->n[0], g->n[1], g->n[2], p->mu, -2.0 / 3.0 * p->mu};
    c.NI = (size_t)(c.nz + 1) * c.ny * c.nx;
    const double dv = g->dx[0] * g->dx[1] * g->dx[2];
    double* Fl[9];
    double* El[3];
    for (int q = 0; q < 9; ++q) Fl[q] = (double*)calloc(c.NI, sizeof(double));
    for (int q = 0; q < 3; ++q) El[q] = (double*)calloc(c.NI, sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k <= c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                const size_t id = VID(&c, i, j, k);
                for (int cc = 0; cc < 3; ++cc) {
                    const int s = cc + 1;
                    for (int d = 0; d < 3; ++d) {
                        /* z-faces on the bottom and top walls of the u and v
                         * CVs are stress-free; the w CVs' z-faces are cell
                         * centres (k = 1 .. nz, the last one the upper face
                         * of CV nz - 1) */
                        if (d == 2 && cc != 2 && (k == 0 || k == c.nz)) continue;
                        if (d == 2 && cc == 2 && k == 0) continue;
                        if (d != 2 && k == c.nz) continue;
                        if (cc == 2 && d != 2 && k == 0) continue; /* no w CV at k = 0 */
                        if (!(VG(&c, s, OQ_BX + d, i, j, k) > 0.0)) continue;
                        Fl[3 * cc + d][id] = face_stress(&c, cc, d, i, j, k);
                    }
                    /* EB facet of the CV (no-slip walls only) */
                    if (p->eb_mode == 1 && vfluid(&c, s, i, j, k) && VG(&c, s, OQ_AREA, i, j, k) > 0.0) {
                        const int idx[3] = {i, j, k};
                        double xn[3], x[3];
                        for (int a = 0; a < 3; ++a) {
                            xn[a] = idx[a] + 0.5 - (a == cc ? 0.5 : 0.0);
                            x[a] = g->lo[a] + (xn[a] + VG(&c, s, OQ_EBX + a, i, j, k)) * g->dx[a];
                        }
                        double G[3][3];
                        for (int e = 0; e < 3; ++e) fit_gradient(&c, e, x, xn, 1, G[e]);
                        const double av[3] = {VG(&c, s, OQ_AX, i, j, k) * g->dx[1] * g->dx[2],
                                              VG(&c, s, OQ_AY, i, j, k) * g->dx[0] * g->dx[2],
                                              VG(&c, s, OQ_AZ, i, j, k) * g->dx[0] * g->dx[1]};
                        /* tau_c . n_out A with n_out = -(area vector into the fluid) / A */
                        double t = 0.0;
                        for (int d = 0; d < 3; ++d) t -= tau_of(&c, G, cc, d) * av[d];
                        El[cc][id] = t;
                    }
                }
            }
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= c.nz; ++k)
        for (int j = 0; j < c.ny; ++j)
            for (int i = 0; i < c.nx; ++i) {
                const size_t id = VID(&c, i, j, k);
                for (int cc = 0; cc < 3; ++cc) {
                    const int s = cc + 1;
                    D[cc][id] = 0.0;
                    if (!vfluid(&c, s, i, j, k)) continue;
                    double sum = 0.0;
                    for (int d = 0; d < 3; ++d) {
                        const int ip = i + (d == 0), jp = j + (d == 1), kp = k + (d == 2);
                        const double fa = dv / g->dx[d];
                        const double bl = VG(&c, s, OQ_BX + d, i, j, k), bh = VG(&c, s, OQ_BX + d, ip, jp, kp);
                        const double fh = kp <= c.nz ? Fl[3 * cc + d][VID(&c, ip, jp, kp)] : 0.0;
                        sum += (bh * fh - bl * Fl[3 * cc + d][id]) * fa;
                    }
                    sum += El[cc][id];
                    D[cc][id] = sum / (VG(&c, s, OQ_ALPHA, i, j, k) * dv);
                }
            }
    for (int q = 0; q < 9; ++q) {
        if (F && F[q]) memcpy(F[q], Fl[q], sizeof(double) * c.NI);
        free(Fl[q]);
    }
    for (int q = 0; q < 3; ++q) {
        if (E && E[q]) memcpy(E[q], El[q], sizeof(double) * c.NI);
        free(El[q]);
    }
    return 0;
}
