/*
 * Oracle geometry for a general level set (TEST INFRASTRUCTURE ONLY; see
 * oracle.h).
 *
 * Section 3.2 of the paper: the embedded boundary is the zero set of an
 * implicit function (a signed distance or a height function) sampled at the
 * grid nodes and reconstructed as planar facets inside each cell.  Reading
 * (the paper defers to the AMReX EB module): inside every cell the level set
 * is the piecewise linear interpolant over the six Kuhn tetrahedra
 *   T_s = { 1 >= u[s0] >= u[s1] >= u[s2] >= 0 }
 * (u the unit coordinates of the cell, s a permutation of the axes), whose
 * vertices are the nodes 0, e[s0], e[s0] + e[s1] and (1, 1, 1).  Fluid is
 * {phi > 0}.  For phi = z - h(x, y) the interpolant is z minus the terrain
 * interpolant on the two triangles of the (i,j)-(i+1,j+1) diagonal, so this
 * builder and the terrain builder describe the same geometry.
 *
 * Ties, generalising the terrain rules: a face carries fluid where phi > 0
 * (phi >= 0 on the domain bottom); the EB facets of a control volume are the
 * parts of the zero set that bound its fluid region (a facet lying on a face
 * belongs to the control volume on its fluid side), except on the domain
 * bottom, where the wall takes precedence.  A zero set lying exactly on the
 * mid-plane of a cell is not resolved by a rule (inputs avoid it).
 *
 * Requirement: phi nondecreasing along z at every node column.  Then the
 * interpolant is nondecreasing in z inside every tetrahedron (its z slope is
 * a difference of two nodal values one above the other), so every column is
 * covered below, cut, then regular; this holds for a terrain, a hemisphere or
 * a wall-mounted cylinder standing on the bottom.
 *
 * Algorithm (generic and plain, not fast): the fluid part of tetrahedron T
 * inside a box piece is the convex polyhedron cut out by T's four half-spaces,
 * the piece's mid-plane half-space and {phi_T >= 0}.  Each face polygon of it
 * is obtained on its own, by Sutherland-Hodgman clipping of a polygon in the
 * face's plane (the triangle of a tetrahedron face, the cell's cross-section
 * at the mid-plane, the cross-section of T with phi_T = 0) against the other
 * half-spaces.  The volume and its first moments follow from the divergence
 * theorem over these polygons, each integrated exactly by fan triangulation
 * with the edge-midpoint rule.
 */
#include "geom_piece.h"

#include <math.h>
#include <string.h>

typedef struct {
    double u[3]; /* unit cell coordinates                   */
    double f;    /* the tetrahedron's linear level set there */
} LV;

typedef struct {
    int n;
    LV v[24];
} LPoly;

/* Keep the part of a convex polygon where c0 + c . u + cf f <= 0. */
static void lclip(const LPoly* in, double c0, const double c[3], double cf, LPoly* out) {
    out->n = 0;
    for (int a = 0; a < in->n; ++a) {
        const LV* p = &in->v[a];
        const LV* q = &in->v[(a + 1) % in->n];
        const double sp = c0 + c[0] * p->u[0] + c[1] * p->u[1] + c[2] * p->u[2] + cf * p->f;
        const double sq = c0 + c[0] * q->u[0] + c[1] * q->u[1] + c[2] * q->u[2] + cf * q->f;
        const int ip = sp <= 0.0, iq = sq <= 0.0;
        if (ip) out->v[out->n++] = *p;
        if (ip != iq) {
            const double t = sp / (sp - sq);
            LV r;
            for (int d = 0; d < 3; ++d) r.u[d] = (1.0 - t) * p->u[d] + t * q->u[d];
            r.f = (1.0 - t) * p->f + t * q->f;
            out->v[out->n++] = r;
        }
    }
}

/* A half-space c0 + c . u + cf f <= 0. */
typedef struct {
    double c0, c[3], cf;
} Half;

/* Integrals over a planar convex polygon (physical coordinates relative to
 * the cell node): area vector (orientation made to agree with `nout`),
 * area, first moments and the integrals of x_d^2. */
typedef struct {
    double a[3], A, m[3], q[3];
} PolyInt;

static void poly_int(const LPoly* P, const double del[3], const double nout[3], PolyInt* r) {
    memset(r, 0, sizeof(*r));
    if (P->n < 3) return;
    double x[24][3];
    for (int v = 0; v < P->n; ++v)
        for (int d = 0; d < 3; ++d) x[v][d] = P->v[v].u[d] * del[d];
    for (int t = 1; t + 1 < P->n; ++t) {
        const double* A = x[0];
        const double* B = x[t];
        const double* C = x[t + 1];
        const double e1[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
        const double e2[3] = {C[0] - A[0], C[1] - A[1], C[2] - A[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        for (int d = 0; d < 3; ++d) r->a[d] += 0.5 * cr[d];
        const double S = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        r->A += S;
        for (int d = 0; d < 3; ++d) {
            r->m[d] += S * (A[d] + B[d] + C[d]) / 3.0;
            const double m1 = 0.5 * (A[d] + B[d]), m2 = 0.5 * (B[d] + C[d]), m3 = 0.5 * (C[d] + A[d]);
            r->q[d] += S / 3.0 * (m1 * m1 + m2 * m2 + m3 * m3);
        }
    }
    if (r->a[0] * nout[0] + r->a[1] * nout[1] + r->a[2] * nout[2] < 0.0)
        for (int d = 0; d < 3; ++d) r->a[d] = -r->a[d];
}

/* Add one bounding polygon of a fluid polyhedron to its volume moments
 * (divergence theorem: V = 1/3 sum a . x_c, M_d = 1/2 sum n_d int x_d^2). */
static void add_to_volume(const PolyInt* r, double* vol, double mv[3]) {
    if (!(r->A > 0.0)) return;
    *vol += (r->a[0] * r->m[0] + r->a[1] * r->m[1] + r->a[2] * r->m[2]) / (3.0 * r->A);
    for (int d = 0; d < 3; ++d) mv[d] += 0.5 * (r->a[d] / r->A) * r->q[d];
}

typedef struct {
    const orc_grid* g;
    const double* phi; /* (nz+1) x (ny+1) x (nx+1) nodes, x fastest */
} LsCtx;

/* nodal phi of cell (i, j, k), index bit 0 = x, bit 1 = y, bit 2 = z */
static void cell_phi(const LsCtx* L, int i, int j, int k, double ph[8]) {
    const int nx = L->g->n[0], ny = L->g->n[1];
    i = ((i % nx) + nx) % nx;
    j = ((j % ny) + ny) % ny;
    for (int c = 0; c < 8; ++c) {
        const int ii = i + (c & 1), jj = j + ((c >> 1) & 1), kk = k + ((c >> 2) & 1);
        ph[c] = L->phi[((size_t)kk * (ny + 1) + jj) * (nx + 1) + ii];
    }
}

static const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

/* the piece's mid-plane half-space (keep <= 0) and the box face it bounds */
static int mid_half(int part, Half* h, int* face) {
    if (part == 0) return 0;
    const int d = (part - 1) / 2, upper = (part - 1) % 2;
    memset(h, 0, sizeof(*h));
    h->c[d] = upper ? -1.0 : 1.0;
    h->c0 = upper ? 0.5 : -0.5;
    *face = 2 * d + (upper ? 0 : 1);
    return 1;
}

/* physical gradient of c0 + c . u (the outward direction of a half-space) */
static void half_normal(const Half* h, const double del[3], double n[3]) {
    for (int d = 0; d < 3; ++d) n[d] = h->c[d] / del[d];
}

static void add_face(BoxOut* o, int f, const PolyInt* r) {
    o->fa[f] += r->A;
    for (int d = 0; d < 3; ++d) o->fm[f][d] += r->m[d];
}

/* EB facet piece with area vector pointing into the fluid */
static void add_eb(BoxOut* o, const PolyInt* r, double sign) {
    if (!(r->A > 0.0)) return;
    for (int d = 0; d < 3; ++d) o->av[d] += sign * r->a[d];
    o->area += r->A;
    for (int d = 0; d < 3; ++d) o->em[d] += r->m[d];
}

static void clip_all(const LPoly* in, const Half* hs, int nh, LPoly* out) {
    LPoly a = *in, b;
    for (int q = 0; q < nh; ++q) {
        lclip(&a, hs[q].c0, hs[q].c, hs[q].cf, &b);
        a = b;
    }
    *out = a;
}

/* Fluid part of tetrahedron s of the cell inside box piece `part`. */
static void tet_piece(const orc_grid* g, const double ph[8], int s, int part, int bottom, BoxOut* o) {
    const double del[3] = {g->dx[0], g->dx[1], g->dx[2]};
    const int* P = kPerm[s];
    /* vertices */
    LV V[4];
    int node[4] = {0, 1 << P[0], (1 << P[0]) | (1 << P[1]), 7};
    for (int m = 0; m < 4; ++m) {
        for (int d = 0; d < 3; ++d) V[m].u[d] = (node[m] >> d) & 1;
        V[m].f = ph[node[m]];
    }
    int npos = 0, nneg = 0;
    for (int m = 0; m < 4; ++m) {
        npos += V[m].f > 0.0;
        nneg += V[m].f < 0.0;
    }
    if (npos == 0) return; /* no fluid (its zero faces belong to the other side) */
    /* linear level set of the tetrahedron: f = f0 + sum_m (f_m - f_{m-1}) u[P[m-1]] */
    double gu[3] = {0, 0, 0};
    for (int m = 1; m < 4; ++m) gu[P[m - 1]] = V[m].f - V[m - 1].f;
    const double f0 = V[0].f;
    double gphys[3];
    for (int d = 0; d < 3; ++d) gphys[d] = gu[d] / del[d];
    /* half-spaces: the four faces (face m opposite vertex m), the mid-plane,
     * the fluid */
    Half H[6];
    memset(H, 0, sizeof(H));
    H[0].c[P[0]] = 1.0; H[0].c0 = -1.0;     /* u[s0] <= 1: cell face +s0 */
    H[1].c[P[1]] = 1.0; H[1].c[P[0]] = -1.0; /* u[s1] <= u[s0]            */
    H[2].c[P[2]] = 1.0; H[2].c[P[1]] = -1.0; /* u[s2] <= u[s1]            */
    H[3].c[P[2]] = -1.0;                     /* u[s2] >= 0: cell face -s2 */
    int mid_face = -1;
    const int has_mid = mid_half(part, &H[4], &mid_face);
    H[5].cf = -1.0;                          /* f >= 0                    */
    const int cut = nneg > 0;                /* the fluid plane cuts T    */
    const int cell_face[4] = {2 * P[0] + 1, -1, -1, 2 * P[2]};
    double vol = 0.0, mv[3] = {0, 0, 0};
    /* faces of T */
    for (int m = 0; m < 4; ++m) {
        LPoly F, C;
        F.n = 3;
        int q = 0;
        int zero = 1;
        for (int v = 0; v < 4; ++v) {
            if (v == m) continue;
            F.v[q++] = V[v];
            zero = zero && V[v].f == 0.0;
        }
        Half hs[2];
        int nh = 0;
        if (has_mid) hs[nh++] = H[4];
        if (cut) hs[nh++] = H[5];
        clip_all(&F, hs, nh, &C);
        double n[3];
        half_normal(&H[m], del, n);
        PolyInt r;
        poly_int(&C, del, n, &r);
        add_to_volume(&r, &vol, mv);
        const int on_bottom = bottom && m == 3 && P[2] == 2;
        if (zero && !on_bottom) {
            add_eb(o, &r, -1.0); /* facet bounding T's fluid: into T */
        } else if (cell_face[m] >= 0) {
            add_face(o, cell_face[m], &r);
        }
    }
    /* the mid-plane cross-section */
    if (has_mid) {
        const int d = (part - 1) / 2, a = (d + 1) % 3, b = (d + 2) % 3;
        LPoly Q, C;
        Q.n = 4;
        const int corner[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
        for (int v = 0; v < 4; ++v) {
            Q.v[v].u[d] = 0.5;
            Q.v[v].u[a] = corner[v][0];
            Q.v[v].u[b] = corner[v][1];
            Q.v[v].f = f0 + gu[0] * Q.v[v].u[0] + gu[1] * Q.v[v].u[1] + gu[2] * Q.v[v].u[2];
        }
        Half hs[5];
        int nh = 0;
        for (int m = 0; m < 4; ++m) hs[nh++] = H[m];
        if (cut) hs[nh++] = H[5];
        clip_all(&Q, hs, nh, &C);
        double n[3];
        half_normal(&H[4], del, n);
        PolyInt r;
        poly_int(&C, del, n, &r);
        add_to_volume(&r, &vol, mv);
        add_face(o, mid_face, &r);
    }
    /* the zero-set cross-section of T */
    if (cut) {
        LPoly X, C;
        X.n = 0;
        for (int m = 0; m < 4; ++m)
            if (V[m].f == 0.0) X.v[X.n++] = V[m];
        for (int p = 0; p < 4; ++p)
            for (int q = p + 1; q < 4; ++q) {
                const LV* A = &V[p];
                const LV* B = &V[q];
                if (!((A->f > 0.0 && B->f < 0.0) || (A->f < 0.0 && B->f > 0.0))) continue;
                /* from the positive end, so that the point does not depend on
                 * the order of the pair */
                const LV* Pp = A->f > 0.0 ? A : B;
                const LV* Pn = A->f > 0.0 ? B : A;
                const double t = Pp->f / (Pp->f - Pn->f);
                LV r;
                for (int d = 0; d < 3; ++d) r.u[d] = (1.0 - t) * Pp->u[d] + t * Pn->u[d];
                r.f = 0.0;
                X.v[X.n++] = r;
            }
        /* order the points around their centroid in the plane */
        double c[3] = {0, 0, 0};
        double x[8][3];
        for (int v = 0; v < X.n; ++v)
            for (int d = 0; d < 3; ++d) {
                x[v][d] = X.v[v].u[d] * del[d];
                c[d] += x[v][d] / X.n;
            }
        const double gn = sqrt(gphys[0] * gphys[0] + gphys[1] * gphys[1] + gphys[2] * gphys[2]);
        double e1[3], e2[3];
        {
            const double nn[3] = {gphys[0] / gn, gphys[1] / gn, gphys[2] / gn};
            const int ax = fabs(nn[0]) < 0.5 ? 0 : (fabs(nn[1]) < 0.5 ? 1 : 2);
            double t[3] = {0, 0, 0};
            t[ax] = 1.0;
            e1[0] = nn[1] * t[2] - nn[2] * t[1];
            e1[1] = nn[2] * t[0] - nn[0] * t[2];
            e1[2] = nn[0] * t[1] - nn[1] * t[0];
            const double l = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
            for (int d = 0; d < 3; ++d) e1[d] /= l;
            e2[0] = nn[1] * e1[2] - nn[2] * e1[1];
            e2[1] = nn[2] * e1[0] - nn[0] * e1[2];
            e2[2] = nn[0] * e1[1] - nn[1] * e1[0];
        }
        double ang[8];
        for (int v = 0; v < X.n; ++v) {
            double p1 = 0, p2 = 0;
            for (int d = 0; d < 3; ++d) {
                p1 += (x[v][d] - c[d]) * e1[d];
                p2 += (x[v][d] - c[d]) * e2[d];
            }
            ang[v] = atan2(p2, p1);
        }
        for (int a = 1; a < X.n; ++a)
            for (int b = a; b > 0 && ang[b] < ang[b - 1]; --b) {
                const double ta = ang[b];
                ang[b] = ang[b - 1];
                ang[b - 1] = ta;
                const LV tv = X.v[b];
                X.v[b] = X.v[b - 1];
                X.v[b - 1] = tv;
            }
        Half hs[1];
        int nh = 0;
        if (has_mid) hs[nh++] = H[4];
        clip_all(&X, hs, nh, &C);
        const double n[3] = {-gphys[0], -gphys[1], -gphys[2]};
        PolyInt r;
        poly_int(&C, del, n, &r);
        add_to_volume(&r, &vol, mv);
        add_eb(o, &r, -1.0);
    }
    o->vol += vol;
    for (int d = 0; d < 3; ++d) o->mv[d] += mv[d];
}

static void ls_piece(const PieceSrc* S, int i, int j, int k, int part, BoxOut* o) {
    const NodeData* d = (const NodeData*)S->data;
    const LsCtx Lc = {d->g, d->v};
    const LsCtx* L = &Lc;
    double ph[8];
    cell_phi(L, i, j, k, ph);
    memset(o, 0, sizeof(*o));
    const int bottom = k == 0 && part != 6;
    for (int s = 0; s < 6; ++s) tet_piece(L->g, ph, s, part, bottom, o);
}

/* 0 covered, 1 regular, 2 cut: the extreme values of the interpolant over
 * the piece are among its nodes and, for a half cell, the midpoints of the
 * tetrahedron edges that cross the mid-plane (node pairs a <= b
 * componentwise that differ in the split coordinate).  Samples on the domain
 * bottom count as fluid when >= 0. */
static int ls_type(const PieceSrc* S, int i, int j, int k, int part) {
    const NodeData* d = (const NodeData*)S->data;
    const LsCtx Lc = {d->g, d->v};
    const LsCtx* L = &Lc;
    double ph[8];
    cell_phi(L, i, j, k, ph);
    double smp[20];
    int onb[20];
    int n = 0;
    const int bottom = k == 0;
    if (part == 0) {
        for (int c = 0; c < 8; ++c) {
            smp[n] = ph[c];
            onb[n++] = bottom && !(c & 4);
        }
    } else {
        const int d = (part - 1) / 2, upper = (part - 1) % 2;
        for (int c = 0; c < 8; ++c) {
            if (((c >> d) & 1) != upper) continue;
            smp[n] = ph[c];
            onb[n++] = bottom && !(c & 4);
        }
        for (int a = 0; a < 8; ++a) {
            if ((a >> d) & 1) continue;
            for (int b = 0; b < 8; ++b) {
                if (!((b >> d) & 1) || (a & b) != a) continue;
                smp[n] = 0.5 * ph[a] + 0.5 * ph[b];
                onb[n++] = bottom && !(a & 4) && !(b & 4);
            }
        }
    }
    int covered = 1, regular = 1;
    for (int q = 0; q < n; ++q) {
        if (smp[q] > 0.0) covered = 0;
        if (onb[q] ? !(smp[q] >= 0.0) : !(smp[q] > 0.0)) regular = 0;
    }
    if (covered) return 0;
    if (regular) return 1;
    return 2;
}

int orc_geometry_levelset(const orc_grid* g, const double* phi, double* const geo[4],
                          int8_t* const ctype[4]) {
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= ny; ++j)
            for (int i = 0; i <= nx; ++i) {
                const size_t a = ((size_t)k * (ny + 1) + j) * (nx + 1) + i;
                const size_t b = a + (size_t)(ny + 1) * (nx + 1);
                if (!(phi[b] >= phi[a])) return 1;
            }
    const NodeData d = {g, phi};
    PieceSrc S;
    orc_levelset_src(&d, &S);
    return orc_assemble(&S, geo, ctype);
}

void orc_levelset_src(const NodeData* d, PieceSrc* s) {
    s->g = d->g;
    s->data = d;
    s->piece = ls_piece;
    s->type = ls_type;
}

int orc_levelset_piece(const orc_grid* g, const double* phi, int i, int j, int k, int part,
                       double* out) {
    const NodeData d = {g, phi};
    PieceSrc S;
    orc_levelset_src(&d, &S);
    BoxOut o;
    ls_piece(&S, i, j, k, part, &o);
    out[0] = o.vol;
    for (int d = 0; d < 3; ++d) {
        out[1 + d] = o.mv[d];
        out[4 + d] = o.av[d];
    }
    out[7] = o.area;
    for (int f = 0; f < 6; ++f) out[8 + f] = o.fa[f];
    out[14] = ls_type(&S, i, j, k, part);
    return 0;
}
