// Geometry builder: classification of the four instances, the general region,
// and the moments of every CV in it (Section 3.2 of the paper).
//
// Formulation used here.  Inside an xy-cell the terrain is linear on the two
// triangles a b c and a c d (a = node (i,j), b = (i+1,j), c = (i+1,j+1),
// d = (i,j+1)).  Every box a control volume is made of (the whole cell, or a
// half-cell split at a mid plane) is covered by at most four sub-triangles
// whose corners lie on the half-grid {0, 1/2, 1}^2 of the cell.  With
// d(x,y) = level - h(x,y), the fluid column above the terrain between two
// levels is (zb - h)^+ - (za - h)^+, so every volume moment is a difference of
// positive-part integrals of a linear function over a triangle.  Those have
// closed forms: the positive part is the whole triangle, nothing, a corner
// triangle, or the whole triangle minus a corner triangle, and a linear (or
// squared linear) weight integrates exactly from its corner values.  Vertical
// faces use the same construction in one dimension.
//
// The file is compiled without floating-point contraction so that the
// heights at half-grid points, (0.5 p + 0.5 q), and the plane levels,
// lo + k dz, are rounded exactly as written: the discrete classification is
// made by comparing those values.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <vector>

#include "ebs_internal.h"

namespace ebs {
namespace {

// ------------------------------------------------------------ level planes
__host__ __device__ inline double zplane(double lo, double dz, int k) { return lo + (double)k * dz; }
__host__ __device__ inline double zmidp(double lo, double dz, int k) {
    return lo + ((double)k + 0.5) * dz;
}

struct Heights {
    double a, b, c, d;  // nodal heights
};

// height at half-grid point (s2, t2) in {0,1,2}^2 of the cell
__device__ inline double hhalf(const Heights& H, int s2, int t2) {
    const int key = s2 * 3 + t2;
    switch (key) {
        case 0: return H.a;                       // (0,0)
        case 6: return H.b;                       // (2,0)
        case 8: return H.c;                       // (2,2)
        case 2: return H.d;                       // (0,2)
        case 3: return 0.5 * H.a + 0.5 * H.b;     // (1,0)
        case 7: return 0.5 * H.b + 0.5 * H.c;     // (2,1)
        case 5: return 0.5 * H.d + 0.5 * H.c;     // (1,2)
        case 1: return 0.5 * H.a + 0.5 * H.d;     // (0,1)
        default: return 0.5 * H.a + 0.5 * H.c;    // (1,1) on the diagonal
    }
}

// sub-triangles of each box part: {triangle (0: a b c, 1: a c d), 3 half-grid corners}
// parts: 0 whole, 1 x-lower half, 2 x-upper half, 3 y-lower half, 4 y-upper half
struct Piece {
    int8_t tri, s[3], t[3];
};
__constant__ Piece kPieces[5][4] = {
    {{0, {0, 2, 2}, {0, 0, 2}}, {1, {0, 2, 0}, {0, 2, 2}}, {-1, {0}, {0}}, {-1, {0}, {0}}},
    {{0, {0, 1, 1}, {0, 0, 1}}, {1, {0, 1, 1}, {0, 1, 2}}, {1, {0, 1, 0}, {0, 2, 2}}, {-1, {0}, {0}}},
    {{0, {1, 2, 2}, {0, 0, 2}}, {0, {1, 2, 1}, {0, 2, 1}}, {1, {1, 2, 1}, {1, 2, 2}}, {-1, {0}, {0}}},
    {{0, {0, 2, 2}, {0, 0, 1}}, {0, {0, 2, 1}, {0, 1, 1}}, {1, {0, 1, 0}, {0, 1, 1}}, {-1, {0}, {0}}},
    {{0, {1, 2, 2}, {1, 1, 2}}, {1, {1, 2, 0}, {1, 2, 2}}, {1, {1, 0, 0}, {1, 2, 1}}, {-1, {0}, {0}}},
};

// positive-part integrals over a triangle
struct PP {
    double I, Ix, Iy, J;  // int d+, int x d+, int y d+, int (d+)^2
    double A, Ax, Ay;     // area of {d > 0} and its first moments
};

struct TriW {
    double x[3], y[3], d[3];
};

// exact integrals of a linear weight d over a triangle
__device__ inline void tri_int(const TriW& T, double& S, double& Id, double& Ixd, double& Iyd,
                               double& Idd, double& Ix, double& Iy) {
    S = 0.5 * fabs((T.x[1] - T.x[0]) * (T.y[2] - T.y[0]) - (T.x[2] - T.x[0]) * (T.y[1] - T.y[0]));
    const double sd = T.d[0] + T.d[1] + T.d[2];
    const double sx = T.x[0] + T.x[1] + T.x[2];
    const double sy = T.y[0] + T.y[1] + T.y[2];
    Id = S * sd / 3.0;
    Ix = S * sx / 3.0;
    Iy = S * sy / 3.0;
    Ixd = S / 12.0 * (T.x[0] * T.d[0] + T.x[1] * T.d[1] + T.x[2] * T.d[2] + sx * sd);
    Iyd = S / 12.0 * (T.y[0] * T.d[0] + T.y[1] * T.d[1] + T.y[2] * T.d[2] + sy * sd);
    Idd = S / 12.0 * (T.d[0] * T.d[0] + T.d[1] * T.d[1] + T.d[2] * T.d[2] + sd * sd);
}

// corner triangle at vertex v where d changes sign along both edges
__device__ inline TriW corner(const TriW& T, int v) {
    const int p = (v + 1) % 3, q = (v + 2) % 3;
    const double lp = T.d[v] / (T.d[v] - T.d[p]);
    const double lq = T.d[v] / (T.d[v] - T.d[q]);
    TriW C;
    C.x[0] = T.x[v]; C.y[0] = T.y[v]; C.d[0] = T.d[v];
    C.x[1] = T.x[v] + lp * (T.x[p] - T.x[v]);
    C.y[1] = T.y[v] + lp * (T.y[p] - T.y[v]);
    C.d[1] = 0.0;
    C.x[2] = T.x[v] + lq * (T.x[q] - T.x[v]);
    C.y[2] = T.y[v] + lq * (T.y[q] - T.y[v]);
    C.d[2] = 0.0;
    return C;
}

__device__ inline PP pos_part(const TriW& T) {
    PP r = {0, 0, 0, 0, 0, 0, 0};
    int np = 0, vpos = 0, vneg = 0;
    for (int v = 0; v < 3; ++v) {
        if (T.d[v] > 0.0) { ++np; vpos = v; } else { vneg = v; }
    }
    if (np == 0) return r;
    double S, Id, Ixd, Iyd, Idd, Ix, Iy;
    if (np == 3) {
        tri_int(T, S, Id, Ixd, Iyd, Idd, Ix, Iy);
        r.I = Id; r.Ix = Ixd; r.Iy = Iyd; r.J = Idd; r.A = S; r.Ax = Ix; r.Ay = Iy;
        return r;
    }
    if (np == 1) {
        const TriW C = corner(T, vpos);
        tri_int(C, S, Id, Ixd, Iyd, Idd, Ix, Iy);
        r.I = Id; r.Ix = Ixd; r.Iy = Iyd; r.J = Idd; r.A = S; r.Ax = Ix; r.Ay = Iy;
        return r;
    }
    // two positive corners: whole triangle minus the negative corner triangle
    tri_int(T, S, Id, Ixd, Iyd, Idd, Ix, Iy);
    const TriW C = corner(T, vneg);
    double S2, Id2, Ixd2, Iyd2, Idd2, Ix2, Iy2;
    tri_int(C, S2, Id2, Ixd2, Iyd2, Idd2, Ix2, Iy2);
    r.I = Id - Id2; r.Ix = Ixd - Ixd2; r.Iy = Iyd - Iyd2; r.J = Idd - Idd2;
    r.A = S - S2; r.Ax = Ix - Ix2; r.Ay = Iy - Iy2;
    return r;
}

// one-dimensional positive part over a segment u in [u0, u1] with d linear
struct PP1 {
    double I, Iu, J;
};
__device__ inline PP1 pos_part1(double u0, double d0, double u1, double d1) {
    PP1 r = {0, 0, 0};
    const double L = u1 - u0;
    if (!(L > 0.0)) return r;
    if (d0 > 0.0 && d1 > 0.0) {
        r.I = L * (d0 + d1) * 0.5;
        r.Iu = L / 6.0 * (u0 * (2.0 * d0 + d1) + u1 * (d0 + 2.0 * d1));
        r.J = L / 3.0 * (d0 * d0 + d0 * d1 + d1 * d1);
    } else if (d0 > 0.0) {
        const double lam = d0 / (d0 - d1);
        const double ue = u0 + lam * L;
        r.I = lam * L * d0 * 0.5;
        r.Iu = lam * L / 6.0 * (2.0 * u0 * d0 + ue * d0);
        r.J = lam * L * d0 * d0 / 3.0;
    } else if (d1 > 0.0) {
        const double lam = d1 / (d1 - d0);
        const double us = u1 - lam * L;
        r.I = lam * L * d1 * 0.5;
        r.Iu = lam * L / 6.0 * (us * d1 + 2.0 * u1 * d1);
        r.J = lam * L * d1 * d1 / 3.0;
    }
    return r;
}

// Moments of the fluid part of one box, relative to the cell node (X_i, Y_j, Z_k).
struct BoxM {
    double vol, m[3];
    double fa[6], ft[6][2];  // face areas; moments of the two tangential coordinates
    double fz[6];            // (unused slot kept for z-faces symmetry)
    double av[3], area, em[3];
};

// Evaluate a box: part 0..4 (footprint), z-range [za, zb]; zk is the cell's lower
// node plane; bottom marks the domain bottom.
__device__ void box_eval(const Heights& H, double DX, double DY, int part, double za, double zb,
                         double zk, bool bottom, BoxM& o) {
    for (int q = 0; q < 6; ++q) { o.fa[q] = 0; o.ft[q][0] = o.ft[q][1] = 0; o.fz[q] = 0; }
    o.vol = o.m[0] = o.m[1] = o.m[2] = 0;
    o.av[0] = o.av[1] = o.av[2] = o.area = o.em[0] = o.em[1] = o.em[2] = 0;
    const double hx = 0.5 * DX, hy = 0.5 * DY;
    const double gx[2] = {(H.b - H.a) / DX, (H.c - H.d) / DX};
    const double gy[2] = {(H.c - H.b) / DY, (H.d - H.a) / DY};
    const double zal = za - zk;
    for (int p = 0; p < 4; ++p) {
        const Piece& P = kPieces[part][p];
        if (P.tri < 0) break;
        TriW Tb, Tt;
        double hv[3];
        for (int v = 0; v < 3; ++v) {
            Tb.x[v] = Tt.x[v] = P.s[v] * hx;
            Tb.y[v] = Tt.y[v] = P.t[v] * hy;
            hv[v] = hhalf(H, P.s[v], P.t[v]);
            Tb.d[v] = za - hv[v];
            Tt.d[v] = zb - hv[v];
        }
        const PP lo = pos_part(Tb), hi = pos_part(Tt);
        // volume and moments (z relative to za, shifted below)
        o.vol += hi.I - lo.I;
        o.m[0] += hi.Ix - lo.Ix;
        o.m[1] += hi.Iy - lo.Iy;
        o.m[2] += (zb - za) * hi.I - 0.5 * hi.J + 0.5 * lo.J;
        // area below each level: A{h < level}; at the domain bottom the lower
        // face also counts terrain lying exactly on it (flat piece at za)
        double Alo = lo.A, Axlo = lo.Ax, Aylo = lo.Ay;
        const bool flat = (hv[0] == hv[1]) && (hv[1] == hv[2]);
        double S, Id, Ixd, Iyd, Idd, Ix, Iy;
        tri_int(Tb, S, Id, Ixd, Iyd, Idd, Ix, Iy);
        if (bottom && flat && hv[0] == za) { Alo = S; Axlo = Ix; Aylo = Iy; }
        o.fa[4] += Alo;
        o.ft[4][0] += Axlo;
        o.ft[4][1] += Aylo;
        o.fa[5] += hi.A;
        o.ft[5][0] += hi.Ax;
        o.ft[5][1] += hi.Ay;
        // EB facet: za <= h < zb (za < h at the domain bottom)
        const double pa = hi.A - Alo;
        if (pa > 0.0) {
            const double sq = sqrt(1.0 + gx[P.tri] * gx[P.tri] + gy[P.tri] * gy[P.tri]);
            o.av[0] += -gx[P.tri] * pa;
            o.av[1] += -gy[P.tri] * pa;
            o.av[2] += pa;
            o.area += sq * pa;
            o.em[0] += sq * (hi.Ax - Axlo);
            o.em[1] += sq * (hi.Ay - Aylo);
            // integral of (h - zk) over the facet footprint:
            // int_{h<c} (h - zk) = (c - zk) A - I(c)
            const double hlo = (bottom && flat && hv[0] == za) ? (zal * Alo - lo.I) : (zal * lo.A - lo.I);
            o.em[2] += sq * (((zb - zk) * hi.A - hi.I) - hlo);
        }
    }
    o.m[2] += zal * o.vol;
    // vertical faces: x-faces at the footprint's x bounds, y-faces at its y bounds
    int s_lo = 0, s_hi = 2, t_lo = 0, t_hi = 2;
    if (part == 1) s_hi = 1;
    if (part == 2) s_lo = 1;
    if (part == 3) t_hi = 1;
    if (part == 4) t_lo = 1;
    for (int side = 0; side < 2; ++side) {
        // x-face at s = S: triangle abc covers t in [0, S], acd covers [S, 2]
        {
            const int S2 = side ? s_hi : s_lo;
            const int br[3] = {t_lo, std::min(std::max(S2, t_lo), t_hi), t_hi};
            for (int seg = 0; seg < 2; ++seg) {
                const int ta = br[seg], tb = br[seg + 1];
                if (tb <= ta) continue;
                const double u0 = ta * hy, u1 = tb * hy;
                const double h0 = hhalf(H, S2, ta), h1 = hhalf(H, S2, tb);
                const PP1 L = pos_part1(u0, za - h0, u1, za - h1);
                const PP1 U = pos_part1(u0, zb - h0, u1, zb - h1);
                const int f = 0 + side;
                o.fa[f] += U.I - L.I;
                o.ft[f][0] += U.Iu - L.Iu;
                o.ft[f][1] += (zb - za) * U.I - 0.5 * U.J + 0.5 * L.J + zal * (U.I - L.I);
            }
        }
        // y-face at t = T: triangle acd covers s in [0, T], abc covers [T, 2]
        {
            const int T2 = side ? t_hi : t_lo;
            const int br[3] = {s_lo, std::min(std::max(T2, s_lo), s_hi), s_hi};
            for (int seg = 0; seg < 2; ++seg) {
                const int sa = br[seg], sb = br[seg + 1];
                if (sb <= sa) continue;
                const double u0 = sa * hx, u1 = sb * hx;
                const double h0 = hhalf(H, sa, T2), h1 = hhalf(H, sb, T2);
                const PP1 L = pos_part1(u0, za - h0, u1, za - h1);
                const PP1 U = pos_part1(u0, zb - h0, u1, zb - h1);
                const int f = 2 + side;
                o.fa[f] += U.I - L.I;
                o.ft[f][0] += U.Iu - L.Iu;
                o.ft[f][1] += (zb - za) * U.I - 0.5 * U.J + 0.5 * L.J + zal * (U.I - L.I);
            }
        }
    }
}

__device__ inline void shift_box(BoxM& o, double sx, double sy, double sz) {
    o.m[0] += sx * o.vol; o.m[1] += sy * o.vol; o.m[2] += sz * o.vol;
    o.em[0] += sx * o.area; o.em[1] += sy * o.area; o.em[2] += sz * o.area;
    // tangential coordinates of the faces: x-faces (y, z), y-faces (x, z), z-faces (x, y)
    const double s[3] = {sx, sy, sz};
    const int tg[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    for (int f = 0; f < 6; ++f) {
        const int d = f / 2;
        o.ft[f][0] += s[tg[d][0]] * o.fa[f];
        o.ft[f][1] += s[tg[d][1]] * o.fa[f];
    }
}

// union of two boxes adjacent along d (A lower, B upper)
__device__ inline void combine_box(const BoxM& A, const BoxM& B, int d, BoxM& o) {
    o.vol = A.vol + B.vol;
    o.area = A.area + B.area;
    for (int e = 0; e < 3; ++e) {
        o.m[e] = A.m[e] + B.m[e];
        o.av[e] = A.av[e] + B.av[e];
        o.em[e] = A.em[e] + B.em[e];
    }
    for (int f = 0; f < 6; ++f) {
        if (f / 2 == d) {
            const BoxM& S = (f % 2) ? B : A;
            o.fa[f] = S.fa[f]; o.ft[f][0] = S.ft[f][0]; o.ft[f][1] = S.ft[f][1];
        } else {
            o.fa[f] = A.fa[f] + B.fa[f];
            o.ft[f][0] = A.ft[f][0] + B.ft[f][0];
            o.ft[f][1] = A.ft[f][1] + B.ft[f][1];
        }
    }
}

// ------------------------------------------------------ general level sets
//
// Fluid is {phi > 0} for the piecewise linear interpolant of nodal phi over
// the six Kuhn tetrahedra of the cell, T_s = {1 >= u[s0] >= u[s1] >= u[s2]
// >= 0} in unit cell coordinates, with vertices 0, e[s0], e[s0] + e[s1] and
// (1,1,1).  The fluid part of a tetrahedron inside a box piece is cut into
// tetrahedra in two steps, by the piece's mid-plane and then by phi = 0; a
// tetrahedron cut by a plane leaves one corner tetrahedron or a prism of
// three.  Every vertex carries the set of planes it lies on: the faces of
// its Kuhn tetrahedron (bit m: the face opposite vertex m), the mid-plane and
// the zero set.  A face of a final tetrahedron lies on a plane exactly when
// all three of its vertices do, which books it to a box face, to the EB or
// to the interior with no geometric tolerance.  Ties follow the terrain
// rules: a face carries fluid where phi > 0 (phi >= 0 on the domain bottom),
// a piece of the zero set belongs to the fluid it bounds, and on the domain
// bottom the wall takes precedence.

struct TV {
    double x[3];  // offset from the cell's lower node
    double f;     // the tetrahedron's linear level set
    unsigned m;   // planes the point lies on
};

constexpr unsigned LS_F0 = 1u, LS_F3 = 8u, LS_MID = 16u, LS_ZERO = 32u;

__constant__ int kKuhn[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// point where the plane g = 0 crosses edge (a inside, g < 0; b outside, g >= 0)
__device__ inline TV ls_cross(const TV& a, const TV& b, double ga, double gb, unsigned bit, bool zero_set) {
    TV r;
    if (gb == 0.0) {  // b lies on the plane
        r = b;
        r.m |= bit;
        return r;
    }
    const double t = ga / (ga - gb);
    for (int d = 0; d < 3; ++d) r.x[d] = (1.0 - t) * a.x[d] + t * b.x[d];
    if (zero_set) {
        r.f = 0.0;
        r.m = (a.m & b.m) | bit;
    } else {
        r.f = (1.0 - t) * a.f + t * b.f;
        r.m = (a.m & b.m) | bit | (r.f == 0.0 ? LS_ZERO : 0u);
    }
    return r;
}

// the part {g < 0} of tetrahedron v as at most three tetrahedra
template <class Emit>
__device__ inline void ls_cut(const TV* v, const double* g, unsigned bit, bool zero_set, Emit&& emit) {
    int in[4], out[4], ni = 0, no = 0;
    for (int q = 0; q < 4; ++q) {
        if (g[q] < 0.0) in[ni++] = q;
        else out[no++] = q;
    }
    if (ni == 0) return;
    if (ni == 4) {
        emit(v[0], v[1], v[2], v[3]);
        return;
    }
    auto X = [&](int a, int b) { return ls_cross(v[a], v[b], g[a], g[b], bit, zero_set); };
    if (ni == 1) {
        const int a = in[0];
        emit(v[a], X(a, out[0]), X(a, out[1]), X(a, out[2]));
        return;
    }
    // a prism p0 p1 p2 - q0 q1 q2 with lateral edges p_i q_i, as three
    // tetrahedra
    TV p0, p1, p2, q0, q1, q2;
    if (ni == 3) {
        const int d = out[0];
        p0 = v[in[0]]; p1 = v[in[1]]; p2 = v[in[2]];
        q0 = X(in[0], d); q1 = X(in[1], d); q2 = X(in[2], d);
    } else {
        const int a = in[0], b = in[1];
        p0 = v[a]; p1 = X(a, out[0]); p2 = X(a, out[1]);
        q0 = v[b]; q1 = X(b, out[0]); q2 = X(b, out[1]);
    }
    emit(p0, p1, p2, q2);
    emit(p0, p1, q1, q2);
    emit(p0, q0, q1, q2);
}

__device__ inline bool same_point(const TV& a, const TV& b) {
    return a.x[0] == b.x[0] && a.x[1] == b.x[1] && a.x[2] == b.x[2];
}

__device__ inline void ls_add_face(BoxM& o, int f, double A, const double c[3]) {
    const int tg[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    const int d = f / 2;
    o.fa[f] += A;
    o.ft[f][0] += A * c[tg[d][0]];
    o.ft[f][1] += A * c[tg[d][1]];
}

// one fluid tetrahedron of Kuhn tetrahedron s: volume moments and its faces
__device__ void ls_accumulate(const TV* p, const int* s, int mid_face, bool bottom, BoxM& o) {
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
            if (same_point(p[a], p[b])) return;
    double e[3][3];
    for (int q = 0; q < 3; ++q)
        for (int d = 0; d < 3; ++d) e[q][d] = p[q + 1].x[d] - p[0].x[d];
    const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                       e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                       e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    const double vol = fabs(det) / 6.0;
    if (vol == 0.0) return;
    o.vol += vol;
    for (int d = 0; d < 3; ++d) o.m[d] += vol * 0.25 * (p[0].x[d] + p[1].x[d] + p[2].x[d] + p[3].x[d]);
    for (int j = 0; j < 4; ++j) {
        const TV& A = p[(j + 1) & 3];
        const TV& B = p[(j + 2) & 3];
        const TV& C = p[(j + 3) & 3];
        const unsigned mk = A.m & B.m & C.m;
        if (!(mk & (LS_F0 | LS_F3 | LS_MID | LS_ZERO))) continue;
        const double u[3] = {B.x[0] - A.x[0], B.x[1] - A.x[1], B.x[2] - A.x[2]};
        const double w[3] = {C.x[0] - A.x[0], C.x[1] - A.x[1], C.x[2] - A.x[2]};
        double cr[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        const double area = 0.5 * sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        const double c[3] = {(A.x[0] + B.x[0] + C.x[0]) / 3.0, (A.x[1] + B.x[1] + C.x[1]) / 3.0,
                             (A.x[2] + B.x[2] + C.x[2]) / 3.0};
        if (mk & LS_ZERO) {
            if (bottom && (mk & LS_F3) && s[2] == 2) {
                ls_add_face(o, 4, area, c);
            } else {
                // a piece of the zero set bounding this fluid: its area
                // vector points into the tetrahedron
                const double* P = p[j].x;
                const double side = cr[0] * (P[0] - A.x[0]) + cr[1] * (P[1] - A.x[1]) + cr[2] * (P[2] - A.x[2]);
                const double sg = side > 0.0 ? 0.5 : -0.5;
                for (int d = 0; d < 3; ++d) o.av[d] += sg * cr[d];
                o.area += area;
                for (int d = 0; d < 3; ++d) o.em[d] += area * c[d];
            }
        } else if (mk & LS_MID) {
            ls_add_face(o, mid_face, area, c);
        } else if (mk & LS_F0) {
            ls_add_face(o, 2 * s[0] + 1, area, c);
        } else {
            ls_add_face(o, 2 * s[2], area, c);
        }
    }
}

// Moments of box piece `part` (0 the cell; 1 / 2 lower / upper half in x,
// 3 / 4 in y, 5 / 6 in z) of a cell with nodal values ph (bit 0 = x, bit 1 =
// y, bit 2 = z), relative to the cell's lower node; bottom marks a cell on
// the domain bottom.
__device__ void box_eval_ls(const double ph[8], double DX, double DY, double DZ, int part, bool bottom, BoxM& o) {
    for (int q = 0; q < 6; ++q) { o.fa[q] = 0; o.ft[q][0] = o.ft[q][1] = 0; o.fz[q] = 0; }
    o.vol = o.m[0] = o.m[1] = o.m[2] = 0;
    o.av[0] = o.av[1] = o.av[2] = o.area = o.em[0] = o.em[1] = o.em[2] = 0;
    const double del[3] = {DX, DY, DZ};
    const int md = part ? (part - 1) / 2 : 0;
    const bool upper = part && ((part - 1) % 2);
    const int mid_face = part ? 2 * md + (upper ? 0 : 1) : -1;
    const bool touches_bottom = bottom && part != 6;
    for (int t = 0; t < 6; ++t) {
        const int s[3] = {kKuhn[t][0], kKuhn[t][1], kKuhn[t][2]};
        const int node[4] = {0, 1 << s[0], (1 << s[0]) | (1 << s[1]), 7};
        TV v[4];
        bool any = false;
        for (int q = 0; q < 4; ++q) {
            for (int d = 0; d < 3; ++d) v[q].x[d] = ((node[q] >> d) & 1) ? del[d] : 0.0;
            v[q].f = ph[node[q]];
            v[q].m = (0xFu & ~(1u << q)) | (v[q].f == 0.0 ? LS_ZERO : 0u);
            any = any || v[q].f > 0.0;
        }
        if (!any) continue;
        auto fluid = [&](const TV& a, const TV& b, const TV& c, const TV& d) {
            const TV w[4] = {a, b, c, d};
            const double g[4] = {-a.f, -b.f, -c.f, -d.f};
            ls_cut(w, g, LS_ZERO, true, [&](const TV& p0, const TV& p1, const TV& p2, const TV& p3) {
                const TV p[4] = {p0, p1, p2, p3};
                ls_accumulate(p, s, mid_face, touches_bottom, o);
            });
        };
        if (!part) {
            fluid(v[0], v[1], v[2], v[3]);
        } else {
            double g[4];
            for (int q = 0; q < 4; ++q) g[q] = (upper ? -1.0 : 1.0) * (v[q].x[md] - 0.5 * del[md]);
            ls_cut(v, g, LS_MID, false, fluid);
        }
    }
}

// nodal values of cell (i, j, k) (i and j wrap periodically)
__device__ inline void cell_phi(const double* phi, int nx, int ny, int i, int j, int k, double ph[8]) {
    i = wrapi(i, nx);
    j = wrapi(j, ny);
    for (int c = 0; c < 8; ++c)
        ph[c] = phi[((size_t)(k + ((c >> 2) & 1)) * (ny + 1) + j + ((c >> 1) & 1)) * (nx + 1) + i + (c & 1)];
}

// 0 covered, 1 regular, 2 cut for box piece `part`: the extremes of the
// interpolant over the piece lie among its nodes and, for a half cell, the
// midpoints of the tetrahedron edges crossing its mid-plane (node pairs
// a <= b componentwise that differ in the split coordinate); samples on the
// domain bottom count as fluid when >= 0.
__device__ inline int ls_piece_type(const double ph[8], int part, bool bottom) {
    bool covered = true, regular = true;
    auto sample = [&](double v, bool onb) {
        if (v > 0.0) covered = false;
        if (onb ? !(v >= 0.0) : !(v > 0.0)) regular = false;
    };
    if (!part) {
        for (int c = 0; c < 8; ++c) sample(ph[c], bottom && !(c & 4));
    } else {
        const int d = (part - 1) / 2, up = (part - 1) % 2;
        for (int c = 0; c < 8; ++c)
            if (((c >> d) & 1) == up) sample(ph[c], bottom && !(c & 4));
        for (int a = 0; a < 8; ++a) {
            if ((a >> d) & 1) continue;
            for (int b = 0; b < 8; ++b) {
                if (!((b >> d) & 1) || (a & b) != a) continue;
                sample(0.5 * ph[a] + 0.5 * ph[b], bottom && !(a & 4) && !(b & 4));
            }
        }
    }
    return covered ? 0 : (regular ? 1 : 2);
}

struct GeomArgs {
    int nx, ny, nz;
    double dx, dy, dz, lo_z;
    const double* h;   // terrain: nodes (ny+1) x (nx+1); null for a level set
    const double* phi; // level set: nodes (nz+1) x (ny+1) x (nx+1); null for a terrain
    int merged;        // 1: h / phi hold the nodes of the grid refined by 2, and every
                       // CV is the union of its eight fine cells (Section 4.3)
    int32_t* kf;       // [4][ncol]
    int32_t* kr;
    int32_t* g0;
    int32_t* g1;
    const int32_t* stop;  // [ncol] highest level of a small CV, -1 if none (null: not yet known)
    const int32_t* ftop;  // [ncol] highest level the redistribution touches, -1 if none (null: unknown)
};

__device__ inline Heights cell_heights(const double* h, int nx, int ny, int i, int j) {
    i = wrapi(i, nx);
    j = wrapi(j, ny);
    Heights H;
    H.a = h[(size_t)j * (nx + 1) + i];
    H.b = h[(size_t)j * (nx + 1) + i + 1];
    H.c = h[(size_t)(j + 1) * (nx + 1) + i + 1];
    H.d = h[(size_t)(j + 1) * (nx + 1) + i];
    return H;
}

// min / max of the terrain over a half cell (its piece corners)
__device__ inline void half_range(const Heights& H, int part, double& mn, double& mx) {
    mn = INFINITY;
    mx = -INFINITY;
    for (int p = 0; p < 4; ++p) {
        const Piece& P = kPieces[part][p];
        if (P.tri < 0) break;
        for (int v = 0; v < 3; ++v) {
            const double x = hhalf(H, P.s[v], P.t[v]);
            mn = fmin(mn, x);
            mx = fmax(mx, x);
        }
    }
}

// first fluid and first regular level of instance inst in column (i, j)
__global__ void k_classify(GeomArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = a.nx * a.ny;
    if (c >= ncol) return;
    const int i = c % a.nx, j = c / a.nx;
    const Heights H = cell_heights(a.h, a.nx, a.ny, i, j);
    double mn[4], mx[4];
    half_range(H, 0, mn[0], mx[0]);
    mn[3] = mn[0];
    mx[3] = mx[0];
    {
        double m1, x1, m2, x2;
        half_range(cell_heights(a.h, a.nx, a.ny, i - 1, j), 2, m1, x1);
        half_range(H, 1, m2, x2);
        mn[1] = fmin(m1, m2); mx[1] = fmax(x1, x2);
        half_range(cell_heights(a.h, a.nx, a.ny, i, j - 1), 4, m1, x1);
        half_range(H, 3, m2, x2);
        mn[2] = fmin(m1, m2); mx[2] = fmax(x1, x2);
    }
    int gmin = a.nz;
    for (int inst = 0; inst < 4; ++inst) {
        int kf = -1, kr = -1;
        const int k0 = inst == 3 ? 1 : 0, k1 = inst == 3 ? a.nz - 1 : a.nz - 1;
        for (int k = k0; k <= k1; ++k) {
            bool covered, regular;
            if (inst == 3) {
                covered = mn[3] >= zmidp(a.lo_z, a.dz, k);
                regular = mx[3] < zmidp(a.lo_z, a.dz, k - 1);
            } else {
                covered = mn[inst] >= zplane(a.lo_z, a.dz, k + 1);
                regular = (k == 0) ? (mx[inst] <= zplane(a.lo_z, a.dz, 0))
                                   : (mx[inst] < zplane(a.lo_z, a.dz, k));
            }
            if (kf < 0 && !covered) kf = k;
            if (kr < 0 && regular) { kr = k; break; }
        }
        if (kf < 0) kf = k1 + 1;
        if (kr < 0) kr = k1 + 1;
        if (kf > kr) kf = kr;
        a.kf[inst * ncol + c] = kf;
        a.kr[inst * ncol + c] = kr;
        gmin = min(gmin, kf);
    }
    a.g0[c] = gmin;
}

// Type of CV (inst, i, j, k) of a level set: the staggered CV is regular
// (covered) when both halves are.
__device__ inline int ls_cv_type(const GeomArgs& a, int inst, int i, int j, int k) {
    double ph[8];
    cell_phi(a.phi, a.nx, a.ny, i, j, k, ph);
    if (inst == 0) return ls_piece_type(ph, 0, k == 0);
    const int d = inst - 1;
    double pn[8];
    cell_phi(a.phi, a.nx, a.ny, i - (d == 0), j - (d == 1), k - (d == 2), pn);
    const int ta = ls_piece_type(pn, 2 + 2 * d, k - (d == 2) == 0);
    const int tb = ls_piece_type(ph, 1 + 2 * d, k == 0);
    if (ta == 0 && tb == 0) return 0;
    if (ta == 1 && tb == 1) return 1;
    return 2;
}

// first fluid and first regular level of every instance in column (i, j),
// for a level set nondecreasing along z (every column covered, cut, then
// regular from the bottom up)
__global__ void k_classify_ls(GeomArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = a.nx * a.ny;
    if (c >= ncol) return;
    const int i = c % a.nx, j = c / a.nx;
    int gmin = a.nz;
    for (int inst = 0; inst < 4; ++inst) {
        int kf = -1, kr = -1;
        const int k0 = inst == 3 ? 1 : 0, k1 = a.nz - 1;
        for (int k = k0; k <= k1; ++k) {
            const int ty = ls_cv_type(a, inst, i, j, k);
            if (kf < 0 && ty != 0) kf = k;
            if (ty == 1) {
                kr = k;
                break;
            }
        }
        if (kf < 0) kf = k1 + 1;
        if (kr < 0) kr = k1 + 1;
        if (kf > kr) kf = kr;
        a.kf[inst * ncol + c] = kf;
        a.kr[inst * ncol + c] = kr;
        gmin = min(gmin, kf);
    }
    a.g0[c] = gmin;
}

// ------------------------------------------------- merged coarse geometry
//
// With refinement ratio 2 every CV of every instance of the coarse grid is
// the union of eight fine cells: the x-face CV around coarse face I spans
// the coarse cell centres on either side, which are fine nodes, so it holds
// fine cells 2I - 1 and 2I in x (likewise y and z), and a cell-centred CV
// holds 2I and 2I + 1.  Its moments are the sums of the fine cells' (shifted
// to the coarse node), its faces the fine faces on its boundary; it is
// covered (regular) when all eight fine cells are.

// first fine cell of coarse CV (inst, I, J, K) along each axis
__device__ inline void merged_first(int inst, int I, int J, int K, int& fi, int& fj, int& fk) {
    fi = 2 * I - (inst == 1);
    fj = 2 * J - (inst == 2);
    fk = 2 * K - (inst == 3);
}

// type of fine cell (fi, fj, fk): terrain samples against the fine levels,
// or the level-set samples of the cell
__device__ inline int fine_cell_type(const GeomArgs& a, int fi, int fj, int fk) {
    if (a.phi) {
        double ph[8];
        cell_phi(a.phi, 2 * a.nx, 2 * a.ny, fi, fj, fk, ph);
        return ls_piece_type(ph, 0, fk == 0);
    }
    const double fdz = 0.5 * a.dz;
    double mn, mx;
    half_range(cell_heights(a.h, 2 * a.nx, 2 * a.ny, fi, fj), 0, mn, mx);
    if (mn >= zplane(a.lo_z, fdz, fk + 1)) return 0;
    const bool regular = fk == 0 ? (mx <= zplane(a.lo_z, fdz, 0)) : (mx < zplane(a.lo_z, fdz, fk));
    return regular ? 1 : 2;
}

__device__ inline int merged_cv_type(const GeomArgs& a, int inst, int I, int J, int K) {
    int fi, fj, fk;
    merged_first(inst, I, J, K, fi, fj, fk);
    bool cov = true, reg = true;
    for (int c = 0; c < 2; ++c)
        for (int b = 0; b < 2; ++b)
            for (int q = 0; q < 2; ++q) {
                const int t = fine_cell_type(a, fi + q, fj + b, fk + c);
                cov = cov && t == 0;
                reg = reg && t == 1;
            }
    return cov ? 0 : (reg ? 1 : 2);
}

// first fluid and first regular level of every instance in coarse column
// (I, J) of a merged geometry
__global__ void k_classify_merged(GeomArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = a.nx * a.ny;
    if (c >= ncol) return;
    const int I = c % a.nx, J = c / a.nx;
    int gmin = a.nz;
    for (int inst = 0; inst < 4; ++inst) {
        int kf = -1, kr = -1;
        const int k0 = inst == 3 ? 1 : 0, k1 = a.nz - 1;
        for (int K = k0; K <= k1; ++K) {
            const int ty = merged_cv_type(a, inst, I, J, K);
            if (kf < 0 && ty != 0) kf = K;
            if (ty == 1) {
                kr = K;
                break;
            }
        }
        if (kf < 0) kf = k1 + 1;
        if (kr < 0) kr = k1 + 1;
        if (kf > kr) kf = kr;
        a.kf[inst * ncol + c] = kf;
        a.kr[inst * ncol + c] = kr;
        gmin = min(gmin, kf);
    }
    a.g0[c] = gmin;
}

// Top g1 of the general range of a column.  At and above it the
// regular-region kernel applies the plain formulas, which needs
//  (a) every CV of the cell regular (full faces, no cut-face interpolation);
//  (b) every CV its stencils read fluid (no order reduction; face densities
//      average both sides).  At the cell's own level they lie from GEN_RXY
//      columns below to GEN_RXY - 1 above in x and y (a staggered velocity
//      reads the densities on both sides of its face), and a vertical
//      velocity there reads the density one cell lower; in the own column
//      they reach GEN_RZ - 1 cells down, where the vertical velocity reads the
//      density GEN_RZ down and the horizontal ones the densities of the -x
//      and -y neighbours;
//  (c) the cell outside the redistribution footprint of every small CV
//      (neighbourhood members and least-squares fit points reach WSRD_RXY
//      columns and WSRD_RZ cells above a small CV).
// Before the volume fractions are known, every CV below kr counts as
// possibly small; once they are (a.stop), the footprint of the actual small
// CVs is used (the reach of the cut-face interpolation is covered by the
// face range, see build_range).  Once the
// redistribution tables exist (a.ftop), the range only has to contain the
// cells they read or write in its own column.  A column whose
// whole neighbourhood is regular down to the bottom wall has an empty range.
// "Fluid from level e" uses e = 0 for an instance that is fluid from its
// lowest CV level (nothing to require there).
__global__ void k_g1(GeomArgs a) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = a.nx * a.ny;
    if (c >= ncol) return;
    const int i = c % a.nx, j = c / a.nx;
    auto eff = [&](int s, int cc) {
        const int kf = a.kf[s * ncol + cc];
        return kf == (s == 3 ? 1 : 0) ? 0 : kf;
    };
    auto eff_all = [&](int cc) { return max(max(eff(0, cc), eff(1, cc)), max(eff(2, cc), eff(3, cc))); };
    auto need = [](int e, int d) { return e > 0 ? e + d : 0; };
    int own = 0;   // (a)
    int fl = 0;    // (b)
    int wsrd = 0;  // (c)
    bool flat = true;  // every CV of every instance in the window is regular
    for (int dj = -GEN_RXY; dj <= GEN_RXY; ++dj)
        for (int di = -GEN_RXY; di <= GEN_RXY; ++di) {
            const int cc = wrapi(j + dj, a.ny) * a.nx + wrapi(i + di, a.nx);
            const bool near = abs(di) <= WSRD_RXY && abs(dj) <= WSRD_RXY;
            if (di < GEN_RXY && dj < GEN_RXY) fl = max(fl, need(eff_all(cc), 1));
            for (int inst = 0; inst < 4; ++inst) {
                const int low = inst == 3 ? 1 : 0;  // lowest CV level of the instance
                const int kr = a.kr[inst * ncol + cc];
                flat = flat && kr == low;
                if (near && !a.stop && !a.ftop && kr > low) wsrd = max(wsrd, kr + WSRD_RZ);
                if (di == 0 && dj == 0) own = max(own, kr);
            }
            if (near && a.stop && a.stop[cc] >= 0) wsrd = max(wsrd, a.stop[cc] + WSRD_RZ + 1);
        }
    if (a.ftop && a.ftop[c] >= 0) wsrd = max(wsrd, a.ftop[c] + 1);
    // own column, and the -x / -y neighbours at the depth of the z stencils
    fl = max(fl, max(need(eff_all(c), GEN_RZ - 1), need(eff(0, c), GEN_RZ)));
    fl = max(fl, need(eff(0, j * a.nx + wrapi(i - 1, a.nx)), GEN_RZ - 1));
    fl = max(fl, need(eff(0, wrapi(j - 1, a.ny) * a.nx + i), GEN_RZ - 1));
    a.g1[c] = flat ? a.g0[c] : min(a.nz, max(max(own, fl), max(wsrd, a.g0[c])));
}

struct RecArgs {
    GeomArgs a;
    const int32_t* goff;
    const int32_t* gcol;
    int32_t G;
    double* geo;   // [4][GQ_N][G]
    int8_t* type;  // [4][G]
};

__device__ inline void put(const RecArgs& r, int inst, int q, int g, double v) {
    r.geo[((size_t)inst * GQ_N + q) * r.G + g] = v;
}

// Per general cell: the four instance types in one word (byte s = instance s)
// and the lower-face flags (area fraction > 0, area fraction == 1) of every
// instance and direction; planes without CVs of an instance have no faces.
__global__ void k_pack_types(RecArgs r, uint32_t* type4, uint32_t* fflag, const int4* col) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= r.G) return;
    const int c = r.gcol[g];
    const int k = col_g0(col[c]) + (g - col[c].z);
    uint32_t w = 0, f = 0;
    for (int s = 0; s < NINST; ++s) {
        w |= (uint32_t)(uint8_t)r.type[(size_t)s * r.G + g] << (8 * s);
        const bool plane = s == 3 ? (k >= 1 && k <= r.a.nz - 1) : (k >= 0 && k <= r.a.nz - 1);
        for (int d = 0; d < 3; ++d) {
            const double b = plane ? r.geo[((size_t)s * GQ_N + GQ_BX + d) * r.G + g] : 0.0;
            if (b > 0.0) f |= ff_pos(s, d);
            if (b == 1.0) f |= ff_full(s, d);
        }
    }
    type4[g] = w;
    fflag[g] = f;
}

// Type of CV (inst, c, k) from the column's kf / kr; writes it and, for
// non-cut CVs, their constant records.  Returns true for a cut CV.
__device__ inline bool record_type(const RecArgs& r, int inst, int g, int c, int k) {
    const GeomArgs& a = r.a;
    const int ncol = a.nx * a.ny;
    const bool is_cv = inst == 3 ? (k >= 1 && k <= a.nz - 1) : (k <= a.nz - 1);
    int ty;
    if (!is_cv || k < a.kf[inst * ncol + c]) ty = 0;
    else if (k >= a.kr[inst * ncol + c]) ty = 1;
    else ty = 2;
    r.type[(size_t)inst * r.G + g] = (int8_t)ty;
    if (ty != 2) {
        for (int q = 0; q < GQ_N; ++q) put(r, inst, q, g, 0.0);
        if (ty == 1) {
            put(r, inst, GQ_ALPHA, g, 1.0);
            put(r, inst, GQ_BX, g, 1.0);
            put(r, inst, GQ_BY, g, 1.0);
            put(r, inst, GQ_BZ, g, 1.0);
        }
        return false;
    }
    return true;
}

// The record of a cut CV from its moments o (relative to the lower node of
// the cell the CV is centred in, the CV centre at (cx, cy, cz) from there).
__device__ inline void record_store(const RecArgs& r, int inst, int g, const BoxM& o, double cx, double cy,
                                    double cz) {
    const double DX = r.a.dx, DY = r.a.dy, DZ = r.a.dz;
    const double dv = DX * DY * DZ;
    const double del[3] = {DX, DY, DZ};
    const double ctr[3] = {cx, cy, cz};
    const double farea[3] = {DY * DZ, DX * DZ, DX * DY};
    const int tg[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    put(r, inst, GQ_ALPHA, g, o.vol / dv);
    for (int d = 0; d < 3; ++d) {
        const double fa = o.fa[2 * d];
        put(r, inst, GQ_BX + d, g, fa / farea[d]);
        for (int t = 0; t < 2; ++t) {
            const int e = tg[d][t];
            put(r, inst, GQ_FX1 + 2 * d + t, g, fa > 0.0 ? (o.ft[2 * d][t] / fa - ctr[e]) / del[e] : 0.0);
        }
        put(r, inst, GQ_VCX + d, g, o.vol > 0.0 ? (o.m[d] / o.vol - ctr[d]) / del[d] : 0.0);
        put(r, inst, GQ_AX + d, g, o.av[d] / farea[d]);
        put(r, inst, GQ_EBX + d, g, o.area > 0.0 ? (o.em[d] / o.area - ctr[d]) / del[d] : 0.0);
    }
    put(r, inst, GQ_AREA, g, o.area / (DX * DY));
}

__global__ void k_records(RecArgs r) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= r.G) return;
    const GeomArgs& a = r.a;
    const int c = r.gcol[g];
    const int i = c % a.nx, j = c / a.nx;
    const int k = a.g0[c] + (g - r.goff[c]);
    if (!record_type(r, inst, g, c, k)) return;
    const double DX = a.dx, DY = a.dy, DZ = a.dz;
    const Heights H = cell_heights(a.h, a.nx, a.ny, i, j);
    const double zk = zplane(a.lo_z, DZ, k);
    BoxM o;
    double cx = 0.5 * DX, cy = 0.5 * DY, cz = 0.5 * DZ;
    if (inst == 0) {
        box_eval(H, DX, DY, 0, zk, zplane(a.lo_z, DZ, k + 1), zk, k == 0, o);
    } else if (inst == 1) {
        BoxM A, B;
        box_eval(cell_heights(a.h, a.nx, a.ny, i - 1, j), DX, DY, 2, zk, zplane(a.lo_z, DZ, k + 1),
                 zk, k == 0, A);
        box_eval(H, DX, DY, 1, zk, zplane(a.lo_z, DZ, k + 1), zk, k == 0, B);
        shift_box(A, -DX, 0.0, 0.0);
        combine_box(A, B, 0, o);
        cx = 0.0;
    } else if (inst == 2) {
        BoxM A, B;
        box_eval(cell_heights(a.h, a.nx, a.ny, i, j - 1), DX, DY, 4, zk, zplane(a.lo_z, DZ, k + 1),
                 zk, k == 0, A);
        box_eval(H, DX, DY, 3, zk, zplane(a.lo_z, DZ, k + 1), zk, k == 0, B);
        shift_box(A, 0.0, -DY, 0.0);
        combine_box(A, B, 1, o);
        cy = 0.0;
    } else {
        BoxM A, B;
        const double zkm = zplane(a.lo_z, DZ, k - 1);
        box_eval(H, DX, DY, 0, zmidp(a.lo_z, DZ, k - 1), zk, zkm, false, A);
        box_eval(H, DX, DY, 0, zk, zmidp(a.lo_z, DZ, k), zk, k == 0, B);
        shift_box(A, 0.0, 0.0, -DZ);
        combine_box(A, B, 2, o);
        cz = 0.0;
    }
    record_store(r, inst, g, o, cx, cy, cz);
}

// The same records for a level set: the staggered CVs join the halves of
// the two cells they straddle.
__global__ void k_records_ls(RecArgs r) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= r.G) return;
    const GeomArgs& a = r.a;
    const int c = r.gcol[g];
    const int i = c % a.nx, j = c / a.nx;
    const int k = a.g0[c] + (g - r.goff[c]);
    if (!record_type(r, inst, g, c, k)) return;
    const double DX = a.dx, DY = a.dy, DZ = a.dz;
    double ph[8], pn[8];
    cell_phi(a.phi, a.nx, a.ny, i, j, k, ph);
    BoxM o;
    double cx = 0.5 * DX, cy = 0.5 * DY, cz = 0.5 * DZ;
    if (inst == 0) {
        box_eval_ls(ph, DX, DY, DZ, 0, k == 0, o);
    } else {
        BoxM A, B;
        const int d = inst - 1;
        cell_phi(a.phi, a.nx, a.ny, i - (d == 0), j - (d == 1), k - (d == 2), pn);
        box_eval_ls(pn, DX, DY, DZ, 2 + 2 * d, d != 2 && k == 0, A);
        box_eval_ls(ph, DX, DY, DZ, 1 + 2 * d, k == 0, B);
        shift_box(A, d == 0 ? -DX : 0.0, d == 1 ? -DY : 0.0, d == 2 ? -DZ : 0.0);
        combine_box(A, B, d, o);
        if (d == 0) cx = 0.0;
        if (d == 1) cy = 0.0;
        if (d == 2) cz = 0.0;
    }
    record_store(r, inst, g, o, cx, cy, cz);
}

// moments of fine cell (fi, fj, fk) relative to its lower node
__device__ inline void fine_box(const GeomArgs& a, int fi, int fj, int fk, BoxM& o) {
    const double fdx = 0.5 * a.dx, fdy = 0.5 * a.dy, fdz = 0.5 * a.dz;
    if (a.phi) {
        double ph[8];
        cell_phi(a.phi, 2 * a.nx, 2 * a.ny, fi, fj, fk, ph);
        box_eval_ls(ph, fdx, fdy, fdz, 0, fk == 0, o);
    } else {
        const double zk = zplane(a.lo_z, fdz, fk);
        box_eval(cell_heights(a.h, 2 * a.nx, 2 * a.ny, fi, fj), fdx, fdy, 0, zk, zplane(a.lo_z, fdz, fk + 1), zk,
                 fk == 0, o);
    }
}

// The records of a merged coarse geometry: the eight fine cells of each CV,
// shifted to the coarse node and joined along x, then y, then z.
__global__ void k_records_merged(RecArgs r) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= r.G) return;
    const GeomArgs& a = r.a;
    const int c = r.gcol[g];
    const int I = c % a.nx, J = c / a.nx;
    const int K = a.g0[c] + (g - r.goff[c]);
    if (!record_type(r, inst, g, c, K)) return;
    const double fdx = 0.5 * a.dx, fdy = 0.5 * a.dy, fdz = 0.5 * a.dz;
    int fi, fj, fk;
    merged_first(inst, I, J, K, fi, fj, fk);
    BoxM o, layer;
    for (int cz = 0; cz < 2; ++cz) {
        BoxM plane, row;
        for (int cy = 0; cy < 2; ++cy) {
            BoxM A, B;
            fine_box(a, fi, fj + cy, fk + cz, A);
            fine_box(a, fi + 1, fj + cy, fk + cz, B);
            const double sy = (fj + cy - 2 * J) * fdy, sz = (fk + cz - 2 * K) * fdz;
            shift_box(A, (fi - 2 * I) * fdx, sy, sz);
            shift_box(B, (fi + 1 - 2 * I) * fdx, sy, sz);
            if (cy == 0) {
                combine_box(A, B, 0, row);
            } else {
                BoxM row1;
                combine_box(A, B, 0, row1);
                combine_box(row, row1, 1, plane);
            }
        }
        if (cz == 0) layer = plane;
        else combine_box(layer, plane, 2, o);
    }
    const double DX = a.dx, DY = a.dy, DZ = a.dz;
    record_store(r, inst, g, o, inst == 1 ? 0.0 : 0.5 * DX, inst == 2 ? 0.0 : 0.5 * DY, inst == 3 ? 0.0 : 0.5 * DZ);
}

// highest level of a small CV (0 < volume fraction < vfrac, any instance) per
// column of the general range
__global__ void k_small_top(RecArgs r, double vfrac, int32_t* stop) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= r.G) return;
    bool small = false;
    for (int s = 0; s < NINST; ++s) {
        const double al = r.geo[((size_t)s * GQ_N + GQ_ALPHA) * r.G + g];
        small = small || (al > 0.0 && al < vfrac);
    }
    if (!small) return;
    const int c = r.gcol[g];
    const int k = r.a.g0[c] + (g - r.goff[c]);
    atomicMax(&stop[c], k);
}

// ------------------------------------------ general-range index on the GPU
//
// Per column: the general range [g0, g1) and the extended face range
// [g0, g1e), which also holds the lower faces that bound a general CV from
// above (+x, +y neighbours and the cell above the range) and the faces a
// cut-face interpolation reads (one column away and up to one level above a
// cut CV: up to level kr of every cut column in the 3 x 3 neighbourhood).
// Their offsets are exclusive prefix sums of the column lengths; the cell
// lists hold the column of every entry.

// length of the general range and the interpolation reach of a column
__global__ void k_range_len(const int32_t* g0, const int32_t* g1, const int32_t* kr, int ncol, int32_t* len,
                            int32_t* krcut) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    len[c] = g1[c] - g0[c];
    int r = 0;
    for (int s = 0; s < NINST; ++s) {
        const int k = kr[(size_t)s * ncol + c];
        if (k > (s == 3 ? 1 : 0)) r = max(r, k + 1);
    }
    krcut[c] = r;
}

__global__ void k_range_ext(const int32_t* g0, const int32_t* g1, const int32_t* krcut, int nx, int ny, int nz,
                            int32_t* g1e, int32_t* lene) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nx * ny) return;
    const int i = c % nx, j = c / nx;
    const int own = g1[c] > g0[c] ? g1[c] + 1 : g0[c];
    int interp = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) interp = max(interp, krcut[wrapi(j + dj, ny) * nx + wrapi(i + di, nx)]);
    const int e = min(nz, max(max(own, interp), max(g1[j * nx + wrapi(i - 1, nx)], g1[wrapi(j - 1, ny) * nx + i])));
    g1e[c] = e;
    lene[c] = e - g0[c];
}

// exclusive prefix sum of n values by one block, 1024 at a time with a
// running carry; out[n] receives the total (64-bit, checked by the caller)
__global__ void __launch_bounds__(1024) k_scan_excl(const int32_t* in, int n, int32_t* out, int64_t* total) {
    __shared__ int64_t part[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < n; base += 1024) {
        const int q = base + (int)threadIdx.x;
        const int64_t v = q < n ? in[q] : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const int64_t t = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (q < n) out[q] = (int32_t)(carry + part[threadIdx.x] - v);
        __syncthreads();
        if (threadIdx.x == 1023) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// column of every entry of both lists, and the packed column records
__global__ void k_range_fill(const int32_t* g0, const int32_t* g1, const int32_t* g1e, const int32_t* goff,
                             const int32_t* goffe, int ncol, int32_t* gcol, int32_t* gcole, int4* col) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncol) return;
    for (int k = g0[c]; k < g1[c]; ++k) gcol[goff[c] + (k - g0[c])] = c;
    for (int k = g0[c]; k < g1e[c]; ++k) gcole[goffe[c] + (k - g0[c])] = c;
    col[c] = col_pack(g0[c], g1[c], g1e[c], goff[c], goffe[c]);
}

}  // namespace

static ebs_status build_range(ebs_ctx* cx, const GeomArgs& a);

ebs_status build_geometry(ebs_ctx* cx, const double* d_h, const double* d_phi) {
    const int ncol = cx->ncol;
    GeomArgs a;
    a.nx = cx->nx; a.ny = cx->ny; a.nz = cx->nz;
    a.dx = cx->g.dx[0]; a.dy = cx->g.dx[1]; a.dz = cx->g.dx[2];
    a.lo_z = cx->g.lo[2];
    a.h = d_h;
    a.phi = d_phi;
    a.merged = cx->geo_merged;
    a.kf = cx->d_kf; a.kr = cx->d_kr; a.g0 = cx->d_g0; a.g1 = cx->d_g1;
    a.stop = nullptr;
    a.ftop = nullptr;
    const int tb = 256;
    if (a.merged)
        hipLaunchKernelGGL(k_classify_merged, dim3((ncol + tb - 1) / tb), dim3(tb), 0, cx->stream, a);
    else if (d_phi)
        hipLaunchKernelGGL(k_classify_ls, dim3((ncol + tb - 1) / tb), dim3(tb), 0, cx->stream, a);
    else
        hipLaunchKernelGGL(k_classify, dim3((ncol + tb - 1) / tb), dim3(tb), 0, cx->stream, a);
    EBS_HIP(cx, hipGetLastError());
    if (cx->range_mode == 2) {
        // one pass with the redistribution footprint of an earlier build
        int32_t* d_ftop = nullptr;
        if ((int)cx->h_ftop.size() != ncol || hipMalloc(&d_ftop, sizeof(int32_t) * ncol) != hipSuccess) {
            cx->err = "general range: no redistribution footprint";
            return EBS_E_UNSUPPORTED;
        }
        hipError_t e = hipMemcpyAsync(d_ftop, cx->h_ftop.data(), sizeof(int32_t) * ncol, hipMemcpyHostToDevice,
                                      cx->stream);
        a.ftop = d_ftop;
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_g1, dim3((ncol + tb - 1) / tb), dim3(tb), 0, cx->stream, a);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(cx->stream);
        (void)hipFree(d_ftop);
        if (e != hipSuccess) {
            cx->err = std::string("general range: ") + hipGetErrorString(e);
            return EBS_E_HIP;
        }
        a.ftop = nullptr;
        return build_range(cx, a);
    }
    // pass 1: every CV below kr may be small
    hipLaunchKernelGGL(k_g1, dim3((ncol + tb - 1) / tb), dim3(tb), 0, cx->stream, a);
    EBS_HIP(cx, hipGetLastError());
    ebs_status st = build_range(cx, a);
    if (st != EBS_OK || cx->G == 0 || cx->range_mode == 0) return st;
    // pass 2: the footprint of the small CVs found in pass 1 (they all lie in
    // its range); the range can only shrink
    int32_t* d_stop = nullptr;
    if (hipMalloc(&d_stop, sizeof(int32_t) * ncol) != hipSuccess) {
        cx->err = "device allocation of geometry tables failed";
        return EBS_E_OOM;
    }
    std::vector<int32_t> g1_first = cx->h_g1;
    hipError_t e = hipMemsetAsync(d_stop, 0xFF, sizeof(int32_t) * ncol, cx->stream);
    if (e == hipSuccess) {
        RecArgs r;
        r.a = a;
        r.goff = cx->d_goff;
        r.gcol = cx->d_gcol;
        r.G = cx->G;
        r.geo = cx->d_geo;
        r.type = cx->d_type;
        hipLaunchKernelGGL(k_small_top, dim3((cx->G + 255) / 256), dim3(256), 0, cx->stream, r,
                           cx->g.small_vfrac, d_stop);
        a.stop = d_stop;
        hipLaunchKernelGGL(k_g1, dim3((ncol + tb - 1) / tb), dim3(tb), 0, cx->stream, a);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(cx->h_g1.data(), cx->d_g1, sizeof(int32_t) * ncol,
                                            hipMemcpyDeviceToHost, cx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(cx->stream);
    (void)hipFree(d_stop);
    if (e != hipSuccess) {
        cx->err = std::string("general range: ") + hipGetErrorString(e);
        return EBS_E_HIP;
    }
    a.stop = nullptr;
    if (cx->h_g1 == g1_first) return EBS_OK;
    return build_range(cx, a);
}

// the general range from the column ranges in d_g0 / d_g1: index tables, per
// cell allocations, geometry records, packed types and face flags
static ebs_status build_range(ebs_ctx* cx, const GeomArgs& a) {
    const int ncol = cx->ncol;
    const int tb = 256, nb = (ncol + tb - 1) / tb;
    // the index is computed on the device; the host keeps copies of the
    // per-column ranges for the set-up steps that run there
    int32_t *d_len = nullptr, *d_krcut = nullptr, *d_g1e = nullptr, *d_lene = nullptr, *d_goffe = nullptr;
    int64_t* d_tot = nullptr;
    auto release = [&]() {
        for (void* p : {(void*)d_len, (void*)d_krcut, (void*)d_g1e, (void*)d_lene, (void*)d_goffe, (void*)d_tot})
            if (p) (void)hipFree(p);
    };
    bool ok = hipMalloc(&d_len, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&d_krcut, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&d_g1e, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&d_lene, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&d_goffe, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&d_tot, sizeof(int64_t) * 2) == hipSuccess;
    if (cx->d_goff) (void)hipFree(cx->d_goff);
    cx->d_goff = nullptr;
    ok = ok && hipMalloc(&cx->d_goff, sizeof(int32_t) * ncol) == hipSuccess;
    if (!ok) {
        release();
        cx->err = "device allocation of geometry tables failed";
        return EBS_E_OOM;
    }
    int64_t tot[2] = {0, 0};
    hipLaunchKernelGGL(k_range_len, dim3(nb), dim3(tb), 0, cx->stream, cx->d_g0, cx->d_g1, cx->d_kr, ncol, d_len,
                       d_krcut);
    hipLaunchKernelGGL(k_range_ext, dim3(nb), dim3(tb), 0, cx->stream, cx->d_g0, cx->d_g1, d_krcut, cx->nx, cx->ny,
                       cx->nz, d_g1e, d_lene);
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, cx->stream, d_len, ncol, cx->d_goff, d_tot);
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, cx->stream, d_lene, ncol, d_goffe, d_tot + 1);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(tot, d_tot, sizeof(tot), hipMemcpyDeviceToHost, cx->stream);
    cx->h_g0.assign(ncol, 0);
    cx->h_g1.assign(ncol, 0);
    cx->h_goff.assign(ncol, 0);
    cx->h_g1e.assign(ncol, 0);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cx->h_g0.data(), cx->d_g0, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, cx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cx->h_g1.data(), cx->d_g1, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, cx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cx->h_goff.data(), cx->d_goff, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, cx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(cx->h_g1e.data(), d_g1e, sizeof(int32_t) * ncol, hipMemcpyDeviceToHost, cx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(cx->stream);
    if (e != hipSuccess) {
        release();
        cx->err = std::string("general range: ") + hipGetErrorString(e);
        return EBS_E_HIP;
    }
    const int64_t G = tot[0], Ge = tot[1];
    if (G > INT32_MAX / 8 || Ge > INT32_MAX / 16) {
        release();
        cx->err = "general region too large";
        return EBS_E_UNSUPPORTED;
    }
    cx->G = (int32_t)G;
    cx->Ge = (int32_t)Ge;
    const size_t Gs = (size_t)std::max<int64_t>(G, 1);
    const size_t Ges = (size_t)std::max<int64_t>(Ge, 1);
    auto alloc = [&](void** p, size_t bytes) -> bool {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        return hipMalloc(p, bytes) == hipSuccess;
    };
    ok = true;
    ok &= alloc((void**)&cx->d_col, sizeof(int4) * ncol);
    ok &= alloc((void**)&cx->d_gcol, sizeof(int32_t) * Gs);
    ok &= alloc((void**)&cx->d_geo, sizeof(double) * NINST * GQ_N * Gs);
    ok &= alloc((void**)&cx->d_type, NINST * Gs);
    ok &= alloc((void**)&cx->d_mask, sizeof(int32_t) * NINST * Gs);
    ok &= alloc((void**)&cx->d_small, NINST * Gs);
    ok &= alloc((void**)&cx->d_tier, NINST * Gs);
    ok &= alloc((void**)&cx->d_w, sizeof(double) * NINST * WQ_COUNT * Gs);
    ok &= alloc((void**)&cx->d_smalllist, sizeof(int32_t) * NINST * Gs);
    ok &= alloc((void**)&cx->d_actlist, sizeof(int32_t) * NINST * Gs);
    ok &= alloc((void**)&cx->d_uhat, sizeof(double) * 5 * Gs);
    ok &= alloc((void**)&cx->d_qhat, sizeof(double) * 5 * Gs);
    ok &= alloc((void**)&cx->d_sig, sizeof(double) * 15 * Gs);
    ok &= alloc((void**)&cx->d_prim, sizeof(double) * 4 * Gs);
    ok &= alloc((void**)&cx->d_fh, sizeof(double) * 15 * Ges);
    ok &= alloc((void**)&cx->d_gcole, sizeof(int32_t) * Ges);
    ok &= alloc((void**)&cx->d_fflag, sizeof(uint32_t) * Gs);
    ok &= alloc((void**)&cx->d_type4, sizeof(uint32_t) * Gs);
    if (!ok) {
        release();
        cx->err = "device allocation of geometry tables failed";
        return EBS_E_OOM;
    }
    hipLaunchKernelGGL(k_range_fill, dim3(nb), dim3(tb), 0, cx->stream, cx->d_g0, cx->d_g1, d_g1e, cx->d_goff,
                       d_goffe, ncol, cx->d_gcol, cx->d_gcole, cx->d_col);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(cx->stream);
    release();
    if (e != hipSuccess) {
        cx->err = std::string("general range: ") + hipGetErrorString(e);
        return EBS_E_HIP;
    }
    EBS_HIP(cx, hipMemsetAsync(cx->d_uhat, 0, sizeof(double) * 5 * Gs, cx->stream));
    if (G > 0) {
        RecArgs r;
        r.a = a;
        r.goff = cx->d_goff;
        r.gcol = cx->d_gcol;
        r.G = cx->G;
        r.geo = cx->d_geo;
        r.type = cx->d_type;
        if (a.merged)
            hipLaunchKernelGGL(k_records_merged, dim3((G + 127) / 128, NINST), dim3(128), 0, cx->stream, r);
        else if (a.phi)
            hipLaunchKernelGGL(k_records_ls, dim3((G + 127) / 128, NINST), dim3(128), 0, cx->stream, r);
        else
            hipLaunchKernelGGL(k_records, dim3((G + 127) / 128, NINST), dim3(128), 0, cx->stream, r);
        hipLaunchKernelGGL(k_pack_types, dim3((G + 255) / 256), dim3(256), 0, cx->stream, r, cx->d_type4,
                           cx->d_fflag, cx->d_col);
        EBS_HIP(cx, hipGetLastError());
    }
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    return EBS_OK;
}

}  // namespace ebs
