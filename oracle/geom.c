/*
 * Oracle geometry builder (TEST INFRASTRUCTURE ONLY; see oracle.h).
 *
 * Follows the construction of Section 3.2 of the paper: the embedded boundary
 * is the zero set of the level set phi = z - h(x,y), reconstructed as planar
 * facets inside each cell; the cell-centred data set is built first, then each
 * staggered control volume is assembled from two half-cells of neighbouring
 * cells, summing volumes, face areas and EB areas and averaging centroids with
 * volume / area weights.
 *
 * Reading of the facet reconstruction (the paper defers to the AMReX EB
 * module): inside the xy-cell (i,j) the terrain is the continuous piecewise
 * linear interpolant of the four nodal heights on the two triangles
 * a(i,j) b(i+1,j) c(i+1,j+1) and a c d(i,j+1).  Fluid is {z > h}.  A face
 * lying exactly on the terrain carries no fluid; an EB facet lying exactly on
 * an interior grid plane belongs to the control volume above it; a facet on
 * the domain bottom is dropped (the wall takes precedence).
 *
 * Algorithm here (chosen to be generic and obviously correct, not fast):
 * each triangle is clipped against the box footprint and against the two
 * height levels by Sutherland-Hodgman; every resulting convex polygon is fan
 * triangulated and integrated with the three-edge-midpoint rule, which is
 * exact for the (at most quadratic) integrands that occur.  Faces are clipped
 * as polygons in their own plane.
 */
#include "geom_piece.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double x, y;  /* position in the clipping plane                         */
    double h;     /* absolute terrain height (used for every in/out decision) */
    double hl;    /* terrain height relative to the cell's lower node plane   */
} Vtx;

typedef struct {
    int n;
    Vtx v[32];
} Poly;

/* Keep the part of a convex polygon where c0 + cx*x + cy*y + ch*h is < 0
 * (strict) or <= 0.  New vertices interpolate every attribute with the convex
 * combination (1-t) p + t q. */
static void clip(const Poly* in, double c0, double cx, double cy, double ch, int strict,
                 Poly* out) {
    out->n = 0;
    const int n = in->n;
    for (int a = 0; a < n; ++a) {
        const Vtx* p = &in->v[a];
        const Vtx* q = &in->v[(a + 1) % n];
        const double fp = c0 + cx * p->x + cy * p->y + ch * p->h;
        const double fq = c0 + cx * q->x + cy * q->y + ch * q->h;
        const int ip = strict ? (fp < 0.0) : (fp <= 0.0);
        const int iq = strict ? (fq < 0.0) : (fq <= 0.0);
        if (ip) out->v[out->n++] = *p;
        if (ip != iq) {
            const double t = fp / (fp - fq);
            Vtx r;
            r.x = (1.0 - t) * p->x + t * q->x;
            r.y = (1.0 - t) * p->y + t * q->y;
            r.h = (1.0 - t) * p->h + t * q->h;
            r.hl = (1.0 - t) * p->hl + t * q->hl;
            out->v[out->n++] = r;
        }
    }
}

/* Integrals over a polygon of 1, x, y, hl, x*hl, y*hl, hl*hl, x*x, x*y, y*y. */
typedef struct {
    double a, x, y, h, xh, yh, hh, xx, xy, yy;
} Mom;

static void poly_moments(const Poly* P, Mom* m) {
    memset(m, 0, sizeof(*m));
    for (int t = 1; t + 1 < P->n; ++t) {
        const Vtx* A = &P->v[0];
        const Vtx* B = &P->v[t];
        const Vtx* C = &P->v[t + 1];
        const double S =
            0.5 * ((B->x - A->x) * (C->y - A->y) - (C->x - A->x) * (B->y - A->y));
        const Vtx* E[3][2] = {{A, B}, {B, C}, {C, A}};
        for (int e = 0; e < 3; ++e) {
            const double x = 0.5 * (E[e][0]->x + E[e][1]->x);
            const double y = 0.5 * (E[e][0]->y + E[e][1]->y);
            const double h = 0.5 * (E[e][0]->hl + E[e][1]->hl);
            const double w = S / 3.0;
            m->a += w;
            m->x += w * x;
            m->y += w * y;
            m->h += w * h;
            m->xh += w * x * h;
            m->yh += w * y * h;
            m->hh += w * h * h;
            m->xx += w * x * x;
            m->xy += w * x * y;
            m->yy += w * y * y;
        }
    }
}

typedef struct {
    double DX, DY;
    double hn[4];  /* nodal heights a, b, c, d (absolute)                  */
    double zk;     /* lower node plane of the cell (origin for hl)        */
} CellCtx;

/* The two triangles of the xy-cell as polygons carrying their nodal heights. */
static void make_triangle(const CellCtx* c, int which, Poly* T) {
    const double ha = c->hn[0], hb = c->hn[1], hc = c->hn[2], hd = c->hn[3];
    T->n = 3;
    Vtx a = {0.0, 0.0, ha, ha - c->zk};
    Vtx b = {c->DX, 0.0, hb, hb - c->zk};
    Vtx cc = {c->DX, c->DY, hc, hc - c->zk};
    Vtx d = {0.0, c->DY, hd, hd - c->zk};
    if (which == 0) {
        T->v[0] = a; T->v[1] = b; T->v[2] = cc;
    } else {
        T->v[0] = a; T->v[1] = cc; T->v[2] = d;
    }
}

/* terrain gradient on triangle `which` */
static void tri_grad(const CellCtx* c, int which, double* gx, double* gy) {
    const double ha = c->hn[0], hb = c->hn[1], hc = c->hn[2], hd = c->hn[3];
    if (which == 0) {
        *gx = (hb - ha) / c->DX;
        *gy = (hc - hb) / c->DY;
    } else {
        *gx = (hc - hd) / c->DX;
        *gy = (hd - ha) / c->DY;
    }
}

/* Segment of the vertical line {x = xf} (if dir == 0) or {y = yf} (dir == 1)
 * inside triangle `which`, as two end points with their heights.  Returns 0 if
 * the intersection has zero length. */
static int tri_line(const CellCtx* c, int which, int dir, double f, double* s0, double* h0,
                    double* s1, double* h1) {
    Poly T;
    make_triangle(c, which, &T);
    double smin = 0, smax = 0, hmin = 0, hmax = 0;
    int found = 0;
    for (int e = 0; e < 3; ++e) {
        const Vtx* p = &T.v[e];
        const Vtx* q = &T.v[(e + 1) % 3];
        const double pf = dir == 0 ? p->x : p->y, qf = dir == 0 ? q->x : q->y;
        const double ps = dir == 0 ? p->y : p->x, qs = dir == 0 ? q->y : q->x;
        double pts[2], hs[2];
        int np = 0;
        if (pf == f && qf == f) {
            pts[0] = ps; hs[0] = p->h;
            pts[1] = qs; hs[1] = q->h;
            np = 2;
        } else if ((pf <= f && f <= qf) || (qf <= f && f <= pf)) {
            if (pf == qf) continue;
            const double lam = (f - pf) / (qf - pf);
            pts[0] = (1.0 - lam) * ps + lam * qs;
            hs[0] = (1.0 - lam) * p->h + lam * q->h;
            np = 1;
        }
        for (int k = 0; k < np; ++k) {
            if (!found) {
                smin = smax = pts[k];
                hmin = hmax = hs[k];
                found = 1;
            } else {
                if (pts[k] < smin) { smin = pts[k]; hmin = hs[k]; }
                if (pts[k] > smax) { smax = pts[k]; hmax = hs[k]; }
            }
        }
    }
    if (!found || !(smax > smin)) return 0;
    *s0 = smin; *h0 = hmin; *s1 = smax; *h1 = hmax;
    return 1;
}

/* Fluid part of a vertical face {x = f} (dir 0) or {y = f} (dir 1) of a box,
 * restricted to s in [sa, sb] (the other horizontal coordinate) and z in
 * [za, zb].  Accumulates area and the moments of (s, z - zk). */
static void vertical_face(const CellCtx* c, int dir, double f, double sa, double sb,
                          double za, double zb, double* area, double* ms, double* mz) {
    *area = 0.0; *ms = 0.0; *mz = 0.0;
    for (int which = 0; which < 2; ++which) {
        double s0, h0, s1, h1;
        if (!tri_line(c, which, dir, f, &s0, &h0, &s1, &h1)) continue;
        /* restrict to [sa, sb], interpolating the (linear) height along it */
        double lo = s0 > sa ? s0 : sa;
        double hi = s1 < sb ? s1 : sb;
        if (!(hi > lo)) continue;
        const double mlo = (lo - s0) / (s1 - s0), mhi = (hi - s0) / (s1 - s0);
        const double hlo = (1.0 - mlo) * h0 + mlo * h1;
        const double hhi = (1.0 - mhi) * h0 + mhi * h1;
        /* rectangle in the (s, z) plane; fluid where z > h(s) */
        Poly R, Pf;
        R.n = 4;
        Vtx v0 = {lo, za, hlo, 0}, v1 = {hi, za, hhi, 0}, v2 = {hi, zb, hhi, 0},
            v3 = {lo, zb, hlo, 0};
        R.v[0] = v0; R.v[1] = v1; R.v[2] = v2; R.v[3] = v3;
        clip(&R, 0.0, 0.0, -1.0, 1.0, 1, &Pf); /* keep h - z < 0 */
        for (int t = 1; t + 1 < Pf.n; ++t) {
            const Vtx* A = &Pf.v[0];
            const Vtx* B = &Pf.v[t];
            const Vtx* C = &Pf.v[t + 1];
            const double S =
                0.5 * ((B->x - A->x) * (C->y - A->y) - (C->x - A->x) * (B->y - A->y));
            *area += S;
            *ms += S * (A->x + B->x + C->x) / 3.0;
            *mz += S * ((A->y - c->zk) + (B->y - c->zk) + (C->y - c->zk)) / 3.0;
        }
    }
}

/* Moments of the fluid part of the box [xa,xb] x [ya,yb] x [za,zb] of the cell;
 * x, y local to the cell node, z absolute.  `bottom` marks a box whose lower
 * face is the domain bottom. */
static void box_moments(const CellCtx* c, double xa, double xb, double ya, double yb,
                        double za, double zb, int bottom, BoxOut* o) {
    memset(o, 0, sizeof(*o));
    const double zal = za - c->zk, zbl = zb - c->zk;
    for (int which = 0; which < 2; ++which) {
        Poly T, P1, P2, P3, P, Pl, Pm1, Pm, Pe1, Pe, Pz;
        make_triangle(c, which, &T);
        clip(&T, xa, -1.0, 0.0, 0.0, 0, &P1);   /* x >= xa */
        clip(&P1, -xb, 1.0, 0.0, 0.0, 0, &P2);  /* x <= xb */
        clip(&P2, ya, 0.0, -1.0, 0.0, 0, &P3);  /* y >= ya */
        clip(&P3, -yb, 0.0, 1.0, 0.0, 0, &P);   /* y <= yb */
        Mom m;
        /* terrain at or below the bottom level: full column height */
        clip(&P, -za, 0.0, 0.0, 1.0, 0, &Pl);   /* h <= za */
        poly_moments(&Pl, &m);
        const double H = zbl - zal;
        o->vol += H * m.a;
        o->mv[0] += H * m.x;
        o->mv[1] += H * m.y;
        o->mv[2] += 0.5 * (zbl * zbl - zal * zal) * m.a;
        /* terrain between the levels: column from h to zb */
        clip(&P, za, 0.0, 0.0, -1.0, 1, &Pm1);  /* h > za */
        clip(&Pm1, -zb, 0.0, 0.0, 1.0, 1, &Pm); /* h < zb */
        poly_moments(&Pm, &m);
        o->vol += zbl * m.a - m.h;
        o->mv[0] += zbl * m.x - m.xh;
        o->mv[1] += zbl * m.y - m.yh;
        o->mv[2] += 0.5 * (zbl * zbl * m.a - m.hh);
        /* EB facet: za <= h < zb (za < h at the domain bottom) */
        clip(&P, za, 0.0, 0.0, -1.0, bottom ? 1 : 0, &Pe1);
        clip(&Pe1, -zb, 0.0, 0.0, 1.0, 1, &Pe);
        poly_moments(&Pe, &m);
        double gx, gy;
        tri_grad(c, which, &gx, &gy);
        const double sq = sqrt(1.0 + gx * gx + gy * gy);
        o->av[0] += -gx * m.a;
        o->av[1] += -gy * m.a;
        o->av[2] += m.a;
        o->area += sq * m.a;
        o->em[0] += sq * m.x;
        o->em[1] += sq * m.y;
        o->em[2] += sq * m.h;
        /* horizontal faces: fluid where h < level (h <= level on the domain bottom) */
        clip(&P, -za, 0.0, 0.0, 1.0, bottom ? 0 : 1, &Pz);
        poly_moments(&Pz, &m);
        o->fa[4] += m.a;
        o->fm[4][0] += m.x;
        o->fm[4][1] += m.y;
        o->fm[4][2] += zal * m.a;
        clip(&P, -zb, 0.0, 0.0, 1.0, 1, &Pz);
        poly_moments(&Pz, &m);
        o->fa[5] += m.a;
        o->fm[5][0] += m.x;
        o->fm[5][1] += m.y;
        o->fm[5][2] += zbl * m.a;
    }
    /* vertical faces */
    const double xs[2] = {xa, xb}, ys[2] = {ya, yb};
    for (int s = 0; s < 2; ++s) {
        double a, ms, mz;
        vertical_face(c, 0, xs[s], ya, yb, za, zb, &a, &ms, &mz);
        o->fa[0 + s] = a;
        o->fm[0 + s][0] = xs[s] * a;
        o->fm[0 + s][1] = ms;
        o->fm[0 + s][2] = mz;
        vertical_face(c, 1, ys[s], xa, xb, za, zb, &a, &ms, &mz);
        o->fa[2 + s] = a;
        o->fm[2 + s][0] = ms;
        o->fm[2 + s][1] = ys[s] * a;
        o->fm[2 + s][2] = mz;
    }
}

/* Shift all moments of a box result by (sx, sy, sz) (new origin = old - s). */
static void shift(BoxOut* o, double sx, double sy, double sz) {
    const double s[3] = {sx, sy, sz};
    for (int d = 0; d < 3; ++d) {
        o->mv[d] += s[d] * o->vol;
        o->em[d] += s[d] * o->area;
        for (int f = 0; f < 6; ++f) o->fm[f][d] += s[d] * o->fa[f];
    }
}

/* Union of two boxes adjacent along direction d (A below B). */
static void combine(const BoxOut* A, const BoxOut* B, int d, BoxOut* o) {
    memset(o, 0, sizeof(*o));
    o->vol = A->vol + B->vol;
    o->area = A->area + B->area;
    for (int e = 0; e < 3; ++e) {
        o->mv[e] = A->mv[e] + B->mv[e];
        o->av[e] = A->av[e] + B->av[e];
        o->em[e] = A->em[e] + B->em[e];
    }
    for (int f = 0; f < 6; ++f) {
        const int fd = f / 2, hi = f % 2;
        const BoxOut* src[2] = {A, B};
        if (fd == d) {
            const BoxOut* S = src[hi];
            o->fa[f] = S->fa[f];
            for (int e = 0; e < 3; ++e) o->fm[f][e] = S->fm[f][e];
        } else {
            o->fa[f] = A->fa[f] + B->fa[f];
            for (int e = 0; e < 3; ++e) o->fm[f][e] = A->fm[f][e] + B->fm[f][e];
        }
    }
}

typedef struct {
    const orc_grid* g;
    const double* h;
} GeoCtx;

static double node_h(const GeoCtx* G, int i, int j) {
    const int nx = G->g->n[0], ny = G->g->n[1];
    i = ((i % nx) + nx) % nx;
    j = ((j % ny) + ny) % ny;
    return G->h[(size_t)j * (nx + 1) + i];
}

static void cell_ctx(const GeoCtx* G, int i, int j, int k, CellCtx* c) {
    const int nx = G->g->n[0], ny = G->g->n[1];
    i = ((i % nx) + nx) % nx;
    j = ((j % ny) + ny) % ny;
    c->DX = G->g->dx[0];
    c->DY = G->g->dx[1];
    c->hn[0] = G->h[(size_t)j * (nx + 1) + i];
    c->hn[1] = G->h[(size_t)j * (nx + 1) + i + 1];
    c->hn[2] = G->h[(size_t)(j + 1) * (nx + 1) + i + 1];
    c->hn[3] = G->h[(size_t)(j + 1) * (nx + 1) + i];
    c->zk = G->g->lo[2] + (double)k * G->g->dx[2];
}

/* Plane z coordinates: node planes lo + k dz, mid planes lo + (k + 1/2) dz. */
static double zplane(const orc_grid* g, int k) { return g->lo[2] + (double)k * g->dx[2]; }
static double zmid(const orc_grid* g, int k) { return g->lo[2] + ((double)k + 0.5) * g->dx[2]; }

/* Box pieces of cell (i,j,k): part 0 full, 1/2 x-lo/hi half, 3/4 y halves, 5/6 z halves */
static void piece(const GeoCtx* G, int i, int j, int k, int part, BoxOut* o) {
    CellCtx c;
    cell_ctx(G, i, j, k, &c);
    const double DX = c.DX, DY = c.DY;
    double xa = 0, xb = DX, ya = 0, yb = DY;
    double za = zplane(G->g, k), zb = zplane(G->g, k + 1);
    int bottom = (k == 0);
    switch (part) {
        case 1: xb = 0.5 * DX; break;
        case 2: xa = 0.5 * DX; break;
        case 3: yb = 0.5 * DY; break;
        case 4: ya = 0.5 * DY; break;
        case 5: zb = zmid(G->g, k); break;
        case 6: za = zmid(G->g, k); bottom = 0; break;
        default: break;
    }
    box_moments(&c, xa, xb, ya, yb, za, zb, bottom, o);
}

/* Sample heights that bound the terrain over a box piece (vertices of the
 * linear pieces of the interpolant), as used by the level-set classification. */
static int piece_samples(const GeoCtx* G, int i, int j, int part, double* s) {
    CellCtx c;
    cell_ctx(G, i, j, 0, &c);
    const double ha = c.hn[0], hb = c.hn[1], hc = c.hn[2], hd = c.hn[3];
    const double mac = 0.5 * ha + 0.5 * hc;
    switch (part) {
        case 1: /* x in [0, dx/2]: a, mid(ab), mid(ac), mid(dc), d */
            s[0] = ha; s[1] = 0.5 * ha + 0.5 * hb; s[2] = mac; s[3] = 0.5 * hd + 0.5 * hc; s[4] = hd;
            return 5;
        case 2:
            s[0] = 0.5 * ha + 0.5 * hb; s[1] = hb; s[2] = hc; s[3] = 0.5 * hd + 0.5 * hc; s[4] = mac;
            return 5;
        case 3: /* y in [0, dy/2]: a, b, mid(bc), mid(ac), mid(ad) */
            s[0] = ha; s[1] = hb; s[2] = 0.5 * hb + 0.5 * hc; s[3] = mac; s[4] = 0.5 * ha + 0.5 * hd;
            return 5;
        case 4:
            s[0] = 0.5 * ha + 0.5 * hd; s[1] = mac; s[2] = 0.5 * hb + 0.5 * hc; s[3] = hc; s[4] = hd;
            return 5;
        default:
            s[0] = ha; s[1] = hb; s[2] = hc; s[3] = hd;
            return 4;
    }
}

/* 0 covered, 1 regular, 2 cut for one box piece */
static int piece_type(const GeoCtx* G, int i, int j, int k, int part) {
    double s[5];
    const int ns = piece_samples(G, i, j, part, s);
    double za = zplane(G->g, k), zb = zplane(G->g, k + 1);
    int bottom = (k == 0);
    if (part == 5) zb = zmid(G->g, k);
    if (part == 6) { za = zmid(G->g, k); bottom = 0; }
    int all_above = 1, all_below = 1;
    for (int q = 0; q < ns; ++q) {
        if (!(s[q] >= zb)) all_above = 0;
        if (bottom ? !(s[q] <= za) : !(s[q] < za)) all_below = 0;
    }
    if (all_above) return 0;
    if (all_below) return 1;
    return 2;
}

static int combine_type(int a, int b) {
    if (a == 0 && b == 0) return 0;
    if (a == 1 && b == 1) return 1;
    return 2;
}

/* Store a control volume's data; (cx, cy, cz) is the CV centre relative to the
 * origin the moments refer to. */
static void store_cv(const orc_grid* g, const BoxOut* o, double cx, double cy, double cz,
                     double* geo, size_t NI, size_t idx) {
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    const double dv = dx * dy * dz;
    const double ctr[3] = {cx, cy, cz};
    const double del[3] = {dx, dy, dz};
    const double farea[3] = {dy * dz, dx * dz, dx * dy};
    geo[OQ_ALPHA * NI + idx] = o->vol / dv;
    /* lower faces: face centre = CV centre shifted by -dx_d/2 along d */
    const int tang[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    const int qb[3] = {OQ_BX, OQ_BY, OQ_BZ};
    const int qf[3] = {OQ_FX1, OQ_FY1, OQ_FZ1};
    for (int d = 0; d < 3; ++d) {
        const double a = o->fa[2 * d];
        geo[qb[d] * NI + idx] = a / farea[d];
        for (int t = 0; t < 2; ++t) {
            const int e = tang[d][t];
            geo[(qf[d] + t) * NI + idx] = a > 0 ? (o->fm[2 * d][e] / a - ctr[e]) / del[e] : 0.0;
        }
    }
    for (int d = 0; d < 3; ++d) {
        geo[(OQ_VCX + d) * NI + idx] = o->vol > 0 ? (o->mv[d] / o->vol - ctr[d]) / del[d] : 0.0;
        geo[(OQ_AX + d) * NI + idx] = o->av[d] / farea[d];
        geo[(OQ_EBX + d) * NI + idx] = o->area > 0 ? (o->em[d] / o->area - ctr[d]) / del[d] : 0.0;
    }
    geo[OQ_AREA * NI + idx] = o->area / (dx * dy);
}

/* store only the lower z-face data (for planes that are not CVs) */
static void store_zface(const orc_grid* g, const BoxOut* o, double cx, double cy, double* geo,
                        size_t NI, size_t idx) {
    const double dx = g->dx[0], dy = g->dx[1];
    const double a = o->fa[4];
    geo[OQ_BZ * NI + idx] = a / (dx * dy);
    geo[OQ_FZ1 * NI + idx] = a > 0 ? (o->fm[4][0] / a - cx) / dx : 0.0;
    geo[OQ_FZ2 * NI + idx] = a > 0 ? (o->fm[4][1] / a - cy) / dy : 0.0;
}

static void terrain_piece(const PieceSrc* s, int i, int j, int k, int part, BoxOut* o) {
    const NodeData* d = (const NodeData*)s->data;
    const GeoCtx G = {d->g, d->v};
    piece(&G, i, j, k, part, o);
}

static int terrain_type(const PieceSrc* s, int i, int j, int k, int part) {
    const NodeData* d = (const NodeData*)s->data;
    const GeoCtx G = {d->g, d->v};
    return piece_type(&G, i, j, k, part);
}

void orc_terrain_src(const NodeData* d, PieceSrc* s) {
    s->g = d->g;
    s->data = d;
    s->piece = terrain_piece;
    s->type = terrain_type;
}

int orc_geometry(const orc_grid* g, const double* h, double* const geo[4], int8_t* const ctype[4]) {
    const NodeData d = {g, h};
    PieceSrc S;
    orc_terrain_src(&d, &S);
    (void)node_h;
    return orc_assemble(&S, geo, ctype);
}

int orc_assemble(const PieceSrc* S, double* const geo[4], int8_t* const ctype[4]) {
    const orc_grid* g = S->g;
    const int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    const size_t NI = (size_t)(nz + 1) * ny * nx;
    const double dx = g->dx[0], dy = g->dx[1], dz = g->dx[2];
    for (int q = 0; q < 4; ++q) {
        memset(geo[q], 0, sizeof(double) * OQ_N * NI);
        memset(ctype[q], 0, NI);
    }
    /* every iteration writes only its own entries: planes run in parallel */
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k <= nz; ++k) {
        for (int j = 0; j < ny; ++j) {
            for (int i = 0; i < nx; ++i) {
                const size_t idx = ((size_t)k * ny + j) * nx + i;
                if (k == nz) {
                    /* domain top: lower z-face of the pseudo planes */
                    BoxOut top, A, B, C;
                    S->piece(S, i, j, nz - 1, 0, &top);
                    /* the top face of cell nz-1 is face 5; move it into slot 4 */
                    top.fa[4] = top.fa[5];
                    for (int e = 0; e < 3; ++e) top.fm[4][e] = top.fm[5][e];
                    store_zface(g, &top, 0.5 * dx, 0.5 * dy, geo[0], NI, idx);
                    S->piece(S, i - 1, j, nz - 1, 2, &A);
                    S->piece(S, i, j, nz - 1, 1, &B);
                    shift(&A, -dx, 0, 0);
                    combine(&A, &B, 0, &C);
                    C.fa[4] = C.fa[5];
                    for (int e = 0; e < 3; ++e) C.fm[4][e] = C.fm[5][e];
                    store_zface(g, &C, 0.0, 0.5 * dy, geo[1], NI, idx);
                    S->piece(S, i, j - 1, nz - 1, 4, &A);
                    S->piece(S, i, j, nz - 1, 3, &B);
                    shift(&A, 0, -dy, 0);
                    combine(&A, &B, 1, &C);
                    C.fa[4] = C.fa[5];
                    for (int e = 0; e < 3; ++e) C.fm[4][e] = C.fm[5][e];
                    store_zface(g, &C, 0.5 * dx, 0.0, geo[2], NI, idx);
                    /* z instance: lower face of pseudo CV nz = mid plane of cell nz-1 */
                    S->piece(S, i, j, nz - 1, 6, &A);
                    store_zface(g, &A, 0.5 * dx, 0.5 * dy, geo[3], NI, idx);
                    continue;
                }
                /* cell-centred instance */
                {
                    BoxOut o;
                    S->piece(S, i, j, k, 0, &o);
                    store_cv(g, &o, 0.5 * dx, 0.5 * dy, 0.5 * dz, geo[0], NI, idx);
                    ctype[0][idx] = (int8_t)S->type(S, i, j, k, 0);
                }
                /* x-face instance: hi-x half of cell i-1 + lo-x half of cell i */
                {
                    BoxOut A, B, C;
                    S->piece(S, i - 1, j, k, 2, &A);
                    S->piece(S, i, j, k, 1, &B);
                    shift(&A, -dx, 0, 0);
                    combine(&A, &B, 0, &C);
                    store_cv(g, &C, 0.0, 0.5 * dy, 0.5 * dz, geo[1], NI, idx);
                    ctype[1][idx] = (int8_t)combine_type(S->type(S, i - 1, j, k, 2),
                                                         S->type(S, i, j, k, 1));
                }
                /* y-face instance */
                {
                    BoxOut A, B, C;
                    S->piece(S, i, j - 1, k, 4, &A);
                    S->piece(S, i, j, k, 3, &B);
                    shift(&A, 0, -dy, 0);
                    combine(&A, &B, 1, &C);
                    store_cv(g, &C, 0.5 * dx, 0.0, 0.5 * dz, geo[2], NI, idx);
                    ctype[2][idx] = (int8_t)combine_type(S->type(S, i, j - 1, k, 4),
                                                         S->type(S, i, j, k, 3));
                }
                /* z-face instance: hi-z half of cell k-1 + lo-z half of cell k (k >= 1) */
                if (k >= 1) {
                    BoxOut A, B, C;
                    S->piece(S, i, j, k - 1, 6, &A);
                    S->piece(S, i, j, k, 5, &B);
                    shift(&A, 0, 0, -dz);
                    combine(&A, &B, 2, &C);
                    store_cv(g, &C, 0.5 * dx, 0.5 * dy, 0.0, geo[3], NI, idx);
                    ctype[3][idx] = (int8_t)combine_type(S->type(S, i, j, k - 1, 6),
                                                         S->type(S, i, j, k, 5));
                }
            }
        }
    }
    return 0;
}

int orc_box_moments(const orc_grid* g, const double* h, int ci, int cj, const double rect[4],
                    double za, double zb, int bottom, double* out) {
    GeoCtx G = {g, h};
    CellCtx c;
    cell_ctx(&G, ci, cj, 0, &c);
    c.zk = za;
    BoxOut o;
    box_moments(&c, rect[0], rect[1], rect[2], rect[3], za, zb, bottom, &o);
    out[0] = o.vol;
    out[1] = o.mv[0];
    out[2] = o.mv[1];
    out[3] = o.mv[2];
    out[4] = o.av[0];
    out[5] = o.av[1];
    out[6] = o.av[2];
    out[7] = o.area;
    for (int f = 0; f < 6; ++f) out[8 + f] = o.fa[f];
    return 0;
}
