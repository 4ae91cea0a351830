/*
 * Oracle momentum sources of the compressible model (TEST INFRASTRUCTURE ONLY;
 * see oracle.h): the perturbation pressure gradient and the buoyancy of
 * Section 2.1 (Eq. mom-comp, B = -rho' g acting along -z, with p' and rho'
 * the departures from a hydrostatic reference state that depends on z only),
 * with the pressure from the equation of state of Section 2.1.  The paper
 * adds the pressure gradient to the right-hand side as a source term
 * (Section 4.1) and states no discretisation for it; the readings here (also
 * listed in the design notes) are:
 *  - the reference state is given per level (cell-centre height of level k)
 *    as rho theta0(k) and rho0(k); it satisfies the equation of state, so
 *    p0(k) = P00 (R rho theta0(k) / P00)^gamma;
 *  - p' and rho' live on fluid cells: p' = p - p0(k), rho' = rho - rho0(k).
 *    p' is evaluated as p0 ((rho theta / rho theta0)^gamma - 1) =
 *    p0 expm1(gamma log1p((rho theta - rho theta0) / rho theta0)), which is
 *    p - p0 in exact arithmetic; the plain difference of two values near
 *    1e5 Pa would lose about three of FP64's digits to cancellation;
 *  - the source of the momentum CV around the lower d-face of cell c is
 *    intensive: -(p'(c) - p'(c - e_d)) / dx_d when both cells are fluid,
 *    zero otherwise;
 *  - the z-face CVs add the buoyancy -g rho', rho' being the mean over the
 *    fluid cells among the two;
 *  - the stage update adds c dt times the source to the provisional momentum
 *    of every fluid CV, before redistribution.
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>

static int wrapi(int i, int n) { return ((i % n) + n) % n; }

/* perturbation pressure of a cell of level k with the given rho theta */
static double pprime(const orc_src* s, const double* rt0, int k, double rt) {
    const double p0 = s->P00 * pow(s->R * rt0[k] / s->P00, s->gamma);
    return p0 * expm1(s->gamma * log1p((rt - rt0[k]) / rt0[k]));
}

int orc_sources(const orc_grid* g, double* const geo[4], const double* const U[5], const orc_src* s,
                const double* rt0, const double* rho0, double* const S[3]) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const size_t NI = (size_t)(nz + 1) * ny * nx;
#define ID(i, j, k) (((size_t)(k) * ny + wrapi((j), ny)) * nx + wrapi((i), nx))
    /* cell-centred CVs are the planes 0 .. nz-1 of instance 0 */
#define FLUID(i, j, k) ((k) >= 0 && (k) < nz && geo[0][ID(i, j, k)] > 0.0)
    for (int d = 0; d < 3; ++d) {
        const int inst = d + 1;
        for (int k = 0; k <= nz; ++k)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const size_t id = ID(i, j, k);
                    S[d][id] = 0.0;
                    const int is_cv = inst == 3 ? (k >= 1 && k <= nz - 1) : (k <= nz - 1);
                    if (!is_cv || !(geo[inst][id] > 0.0)) continue;
                    const int il = i - (d == 0), jl = j - (d == 1), kl = k - (d == 2);
                    const int fa = FLUID(i, j, k), fb = FLUID(il, jl, kl);
                    double src = 0.0;
                    if (fa && fb) {
                        const double pa = pprime(s, rt0, k, U[1][ID(i, j, k)]);
                        const double pb = pprime(s, rt0, kl, U[1][ID(il, jl, kl)]);
                        src = -(pa - pb) / g->dx[d];
                    }
                    if (d == 2) {
                        double r = 0.0;
                        int cnt = 0;
                        if (fa) { r += U[0][ID(i, j, k)] - rho0[k]; ++cnt; }
                        if (fb) { r += U[0][ID(il, jl, kl)] - rho0[kl]; ++cnt; }
                        if (cnt) src -= s->g * r / cnt;
                    }
                    S[d][id] = src;
                }
    }
#undef FLUID
#undef ID
    (void)NI;
    return 0;
}
