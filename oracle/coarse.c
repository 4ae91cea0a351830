/*
 * Oracle geometry of the coarse level of a two-level hierarchy (TEST
 * INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Section 4.3: the coarse level's geometry is built from the fine one by
 * merging subcells, so that volumes and areas (and hence mass and mass
 * fluxes) agree between the levels.  With refinement ratio 2 every coarse
 * control volume of every instance is a union of eight fine cells: the
 * coarse cell (I, J, K) holds the fine cells (2I + a, 2J + b, 2K + c), a
 * coarse half cell the four fine cells on its side, and the x-face control
 * volume around coarse face I (between the coarse cell centres, which are
 * fine nodes) the fine cells 2I - 1 and 2I in x.  So a coarse box piece is
 * the union of fine cells, its moments are the sums of theirs (shifted to
 * the coarse node), its faces the fine faces on its boundary, and it is
 * covered (regular) when all of its fine cells are.
 */
#include "geom_piece.h"

#include <string.h>

typedef struct {
    const PieceSrc* fine;
} Merged;

/* shift all moments of a box by (sx, sy, sz) (origin moved by -s) */
static void shift_box(BoxOut* o, double sx, double sy, double sz) {
    const double s[3] = {sx, sy, sz};
    for (int d = 0; d < 3; ++d) {
        o->mv[d] += s[d] * o->vol;
        o->em[d] += s[d] * o->area;
        for (int f = 0; f < 6; ++f) o->fm[f][d] += s[d] * o->fa[f];
    }
}

/* union of two boxes adjacent along d (A lower, B upper) */
static void join(const BoxOut* A, const BoxOut* B, int d, BoxOut* o) {
    BoxOut r;
    memset(&r, 0, sizeof(r));
    r.vol = A->vol + B->vol;
    r.area = A->area + B->area;
    for (int e = 0; e < 3; ++e) {
        r.mv[e] = A->mv[e] + B->mv[e];
        r.av[e] = A->av[e] + B->av[e];
        r.em[e] = A->em[e] + B->em[e];
    }
    for (int f = 0; f < 6; ++f) {
        const BoxOut* S = (f / 2 == d) ? ((f % 2) ? B : A) : NULL;
        if (S) {
            r.fa[f] = S->fa[f];
            for (int e = 0; e < 3; ++e) r.fm[f][e] = S->fm[f][e];
        } else {
            r.fa[f] = A->fa[f] + B->fa[f];
            for (int e = 0; e < 3; ++e) r.fm[f][e] = A->fm[f][e] + B->fm[f][e];
        }
    }
    *o = r;
}

/* fine offsets of box piece `part` along axis d: {0, 1}, {0} or {1} */
static int piece_range(int part, int d, int* lo) {
    if (part == 2 * d + 1) { *lo = 0; return 1; }
    if (part == 2 * d + 2) { *lo = 1; return 1; }
    *lo = 0;
    return 2;
}

static void merged_piece(const PieceSrc* S, int I, int J, int K, int part, BoxOut* o) {
    const PieceSrc* F = ((const Merged*)S->data)->fine;
    const double* dxf = F->g->dx;
    int lo[3], n[3];
    for (int d = 0; d < 3; ++d) n[d] = piece_range(part, d, &lo[d]);
    BoxOut layer[2];
    for (int c = 0; c < n[2]; ++c) {
        BoxOut row[2];
        for (int b = 0; b < n[1]; ++b) {
            BoxOut cell[2];
            for (int a = 0; a < n[0]; ++a) {
                const int oa = lo[0] + a, ob = lo[1] + b, oc = lo[2] + c;
                F->piece(F, 2 * I + oa, 2 * J + ob, 2 * K + oc, 0, &cell[a]);
                shift_box(&cell[a], oa * dxf[0], ob * dxf[1], oc * dxf[2]);
            }
            if (n[0] == 2) join(&cell[0], &cell[1], 0, &row[b]);
            else row[b] = cell[0];
        }
        if (n[1] == 2) join(&row[0], &row[1], 1, &layer[c]);
        else layer[c] = row[0];
    }
    if (n[2] == 2) join(&layer[0], &layer[1], 2, o);
    else *o = layer[0];
}

static int merged_type(const PieceSrc* S, int I, int J, int K, int part) {
    const PieceSrc* F = ((const Merged*)S->data)->fine;
    int lo[3], n[3];
    for (int d = 0; d < 3; ++d) n[d] = piece_range(part, d, &lo[d]);
    int all_cov = 1, all_reg = 1;
    for (int c = 0; c < n[2]; ++c)
        for (int b = 0; b < n[1]; ++b)
            for (int a = 0; a < n[0]; ++a) {
                const int t = F->type(F, 2 * I + lo[0] + a, 2 * J + lo[1] + b, 2 * K + lo[2] + c, 0);
                all_cov = all_cov && t == 0;
                all_reg = all_reg && t == 1;
            }
    return all_cov ? 0 : (all_reg ? 1 : 2);
}

int orc_geometry_merged(const orc_grid* gc, const double* fine_nodes, int kind, double* const geo[4],
                        int8_t* const ctype[4]) {
    orc_grid gf = *gc;
    for (int d = 0; d < 3; ++d) {
        gf.n[d] = 2 * gc->n[d];
        gf.dx[d] = 0.5 * gc->dx[d];
    }
    const NodeData nd = {&gf, fine_nodes};
    PieceSrc fine;
    if (kind == 0) {
        orc_terrain_src(&nd, &fine);
    } else {
        const int nx = gf.n[0], ny = gf.n[1], nz = gf.n[2];
        const size_t plane = (size_t)(nx + 1) * (ny + 1);
        for (int k = 0; k < nz; ++k)
            for (size_t q = 0; q < plane; ++q)
                if (!(fine_nodes[(size_t)(k + 1) * plane + q] >= fine_nodes[(size_t)k * plane + q])) return 1;
        orc_levelset_src(&nd, &fine);
    }
    const Merged m = {&fine};
    PieceSrc S = {gc, &m, merged_piece, merged_type};
    return orc_assemble(&S, geo, ctype);
}
