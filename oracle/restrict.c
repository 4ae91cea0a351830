/*
 * Oracle restriction (averaging down) between two levels of a static
 * block-structured hierarchy with refinement ratio 2 (TEST INFRASTRUCTURE
 * ONLY; see oracle.h).  Follows Section 4.3: the geometry of the coarse level
 * is built from the fine one by merging subcells, so that volume and area
 * fractions are preserved; cell-centred variables are averaged with volume
 * weights (volume fractions), face-centred ones with area weights (area
 * fractions), so that the mass in every coarse cell and the mass flux through
 * every coarse face equal those of the fine cells and faces they cover.
 *
 * Readings (also listed in the design notes):
 *  - the coarse grid covers the fine grid's domain; coarse cell (I,J,K) holds
 *    the fine cells (2I+a, 2J+b, 2K+c), a, b, c in {0, 1};
 *  - merged geometry: alpha_C = mean of the eight children's alpha; the area
 *    fraction of a coarse cell's lower d-face = mean of the four fine lower
 *    d-faces on it;
 *  - rho and rho theta: sum of alpha_f U_f over the children / sum of alpha_f
 *    (zero when the coarse cell is covered);
 *  - a momentum on a coarse d-face: sum of beta_f U_f over the four fine
 *    d-faces on it / sum of beta_f; when that face has no open area (a
 *    staggered CV can hold fluid behind a covered face, Section 3.2), the
 *    weights are the volume fractions of the four fine staggered CVs instead;
 *    zero when both sums vanish; the wall faces of the z momentum are zero;
 *  - only weights > 0 contribute.
 */
#include "oracle.h"

#include <stddef.h>

static size_t fid(int nx, int ny, int i, int j, int k) { return ((size_t)k * ny + j) * nx + i; }

int orc_coarsen_geometry(const orc_grid* g, double* const geo[4], double* alpha, double* const beta[3]) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    if ((nx | ny | nz) & 1) return 1;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const size_t NI = (size_t)(nz + 1) * ny * nx;
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                const size_t o = fid(cx, cy, I, J, K);
                double a = 0.0;
                for (int c = 0; c < 2; ++c)
                    for (int b = 0; b < 2; ++b)
                        for (int q = 0; q < 2; ++q)
                            a += geo[0][OQ_ALPHA * NI + fid(nx, ny, 2 * I + q, 2 * J + b, 2 * K + c)];
                alpha[o] = a / 8.0;
                for (int d = 0; d < 3; ++d) {
                    double s = 0.0;
                    for (int u = 0; u < 2; ++u)
                        for (int v = 0; v < 2; ++v) {
                            /* the four fine lower d-faces on the coarse lower d-face */
                            const int i = 2 * I + (d == 0 ? 0 : u), j = 2 * J + (d == 1 ? 0 : (d == 0 ? u : v));
                            const int k = 2 * K + (d == 2 ? 0 : v);
                            s += geo[0][(OQ_BX + d) * NI + fid(nx, ny, i, j, k)];
                        }
                    beta[d][o] = s / 4.0;
                }
            }
    return 0;
}

/* Ufine: dense instance storage of the fine grid; Ucoarse: dense instance
 * storage of the coarse grid (nz/2 + 1 planes). */
int orc_restrict(const orc_grid* g, double* const geo[4], const double* const Uf[5], double* const Uc[5]) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    if ((nx | ny | nz) & 1) return 1;
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const size_t NI = (size_t)(nz + 1) * ny * nx;
    const size_t NC = (size_t)(cz + 1) * cy * cx;
    for (int f = 0; f < 5; ++f)
        for (size_t q = 0; q < NC; ++q) Uc[f][q] = 0.0;
    for (int K = 0; K < cz; ++K)
        for (int J = 0; J < cy; ++J)
            for (int I = 0; I < cx; ++I) {
                const size_t o = fid(cx, cy, I, J, K);
                /* cell-centred fields */
                for (int f = 0; f < 2; ++f) {
                    double sw = 0.0, su = 0.0;
                    for (int c = 0; c < 2; ++c)
                        for (int b = 0; b < 2; ++b)
                            for (int a = 0; a < 2; ++a) {
                                const size_t id = fid(nx, ny, 2 * I + a, 2 * J + b, 2 * K + c);
                                const double w = geo[0][OQ_ALPHA * NI + id];
                                if (w > 0.0) { sw += w; su += w * Uf[f][id]; }
                            }
                    Uc[f][o] = sw > 0.0 ? su / sw : 0.0;
                }
                /* momenta on the coarse lower faces */
                for (int d = 0; d < 3; ++d) {
                    if (d == 2 && K == 0) continue; /* bottom wall */
                    double sb = 0.0, sub = 0.0, sa = 0.0, sua = 0.0;
                    for (int u = 0; u < 2; ++u)
                        for (int v = 0; v < 2; ++v) {
                            const int i = 2 * I + (d == 0 ? 0 : u), j = 2 * J + (d == 1 ? 0 : (d == 0 ? u : v));
                            const int k = 2 * K + (d == 2 ? 0 : v);
                            const size_t id = fid(nx, ny, i, j, k);
                            const double b = geo[0][(OQ_BX + d) * NI + id];
                            const double al = geo[d + 1][OQ_ALPHA * NI + id];
                            if (b > 0.0) { sb += b; sub += b * Uf[2 + d][id]; }
                            if (al > 0.0) { sa += al; sua += al * Uf[2 + d][id]; }
                        }
                    Uc[2 + d][o] = sb > 0.0 ? sub / sb : (sa > 0.0 ? sua / sa : 0.0);
                }
            }
    return 0;
}
