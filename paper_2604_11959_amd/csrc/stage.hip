// Explicit stage update of the four instances (Eqs. update-cc / update-fc of
// Section 3.1 with the advective flux of Section 4.1; Algorithm 1 steps 1-3).
//
// The regular region (every cell at or above its column's general range) is
// updated by the kernel in bulk.hip; this file holds the passes over the
// general range of each column (the cut band and a margin), in double
// precision with the full rules: area / volume fractions, covered stencil
// ends (order reduction), interpolation to the cut-face centroid, walls.  They
// also keep a double-precision copy of the provisional state there for the
// redistribution.  The two parts may run concurrently on two streams.
//
// Readings where the paper is silent: the mass flux advecting momentum on a
// staggered face is the mean of the two stored face momenta next to it; face
// velocities divide by the mean density of the fluid cells on either side;
// the momentum flux of the z-face instance through the mid planes of the
// bottom and top cell layers is zero; the EB flux is zero (test mode: minus
// the area vector dotted with the CV's mean provisional flux).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ebs_internal.h"
#include "stage_common.h"
#include "xcd.h"

namespace ebs {
namespace {

// --------------------------------------------------------------- general
//
// The general range is processed in four passes, in double precision: the
// advected quantities (prims) of every general cell and of every position
// above the range that a flux stencil reads; the provisional fluxes on the
// three lower faces of every cell of the extended face range (fhat); area
// fraction x flux moved to the centroid on every partial face (cut, from the
// static cut-face records); and the update, which takes the divergence over
// the six faces.
//
// A stencil position is general (an index into the range), below its column's
// range (no instance is fluid) or above it.  The range's top is chosen so that
// a position above it is regular and every CV within three cells in x and y
// and three below it is fluid; its advected quantities and fluxes therefore
// follow the plain formulas (two-sided face densities, full faces).  Every
// neighbour a cut-face interpolation reads lies within one cell of a CV that is
// not regular, hence inside or below its column's range.  Since the geometry
// is static, the positions the flux and update passes read are resolved once
// at set-up into two tables (build_stencils), so those passes gather directly.
template <typename T>
struct GenArgs {
    Dims D;
    GeoView v;
    const T* un[5];
    const T* cur[5];
    T* out[5];
    double* uhat;  // [5][G]
    double* prim;  // [G + naux][4] theta, u, v, w: general cells, then aux positions
    const uint32_t* sten;  // [10][Ge] stencil table of the face range
    int32_t naux;
    const int4* ptab;      // [G + naux] {i, j, k, fluid bits | lower-neighbour fluid bits << 4}
    const int4* ftab;      // [Ge] {i, j, k, lower-face flags} of the face range
    const int4* utab;      // [G] {i, j, k | fluid bits << 16, index in the face range}
    const int32_t* upd;    // [9][G] update table: the three upper neighbours' lower faces
    double* fh;    // [5][3][Ge] provisional flux on the lower faces
    const int32_t* cbase;  // [G] first cut-face record of each general cell
    // cut-face records: {n0, n1, n2, own | (instance * 3 + direction) << 28}
    // and [5][ncut] {b, c0, c1, c2, c3}
    const int4* cut_n;
    const double* cut_w;
    double* bfc;           // [2][ncut] area fraction x interpolated flux per record
    int32_t ncut;
    double cdt;
    double rdel[3];
    int eb_mode;
    // momentum sources (null when off): {p', rho'} per position of the prims
    // pass, the FP64 per-level table [5][nz] (p0, rho theta0, -, -, rho0) and
    // the equation-of-state constants
    double* srcv;
    const double* sref;
    double sP00, sR, sgam, sg;
};

// Interpolation of the flux on one cut face (area fraction b in (0, 1), or not
// exactly 1) to its centroid, fixed by the geometry: area fraction x flux =
// b (c[0] F(own face) + sum_q c[q+1] F(face n[q])) over the lower faces of the
// same direction at the neighbouring CVs n[q] (indices into the extended face
// range, -1 when unused), summed in that order.  A cell's records are
// consecutive, in the order of (instance, direction) of its partial faces.
struct CutRec {
    int32_t n[3];
    int32_t own;  // extended index of the face's own CV
    int32_t sd;   // instance * 3 + direction
    int32_t pad;
    double b;
    double c[4];
};

// bit s set <=> plane k holds CVs of instance s
__device__ inline int plane_mask(int nz, int k) {
    return (k >= 0 && k <= nz - 1 ? 0x7 : 0) | (k >= 1 && k <= nz - 1 ? 0x8 : 0);
}
__device__ inline int finst(int f) { return f < 2 ? 0 : f - 1; }

// a resolved stencil position: wrapped (i, j), plane k, general index (>= 0)
// or -1 above / -2 below the column's range, index in the extended face range
// (-1 beyond it), fluid bits per instance, lower-face flags (when loaded)
struct Pt {
    int i, j, k, g, ge, fl;
    uint32_t ff;
};
// a stencil position from the face-range table: wrapped (i, j), plane k, fluid
// bits per instance, index into the advected-quantity array
struct SPt {
    int i, j, k, fl;
    uint32_t pi;
};
// a lower face from the update table: index in the extended face range,
// lower-face flags of its CV, first cut-face record of that CV
struct UPt {
    int ge;
    uint32_t ff;
    int rb;
};

template <typename T>
struct Gen {
    const GenArgs<T>& a;
    __device__ __forceinline__ explicit Gen(const GenArgs<T>& a_) : a(a_) {}

    __device__ __forceinline__ int wx(int i) const { return wrapi(i, a.D.nx); }
    __device__ __forceinline__ int wy(int j) const { return wrapi(j, a.D.ny); }
    __device__ __forceinline__ int4 colinfo(int i, int j) const { return a.v.col[j * a.D.nx + i]; }
    // position without fluid bits (face data only)
    __device__ __forceinline__ Pt atf(int i, int j, int k, const int4& ci) const {
        Pt p;
        p.i = i;
        p.j = j;
        p.k = k;
        const int g0 = col_g0(ci);
        p.g = k < g0 ? -2 : (k >= col_g1(ci) ? -1 : ci.z + (k - g0));
        p.ge = k < g0 ? -2 : (k >= ci.y ? -1 : ci.w + (k - g0));
        p.fl = 0;
        p.ff = 0;
        return p;
    }
    // lower-face flags of a position (general: stored; above the range: full
    // faces on the planes that hold CVs; below: none)
    __device__ __forceinline__ uint32_t fflags(const Pt& p) const {
        if (p.g >= 0) return a.v.fflag[p.g];
        if (p.g == -2) return 0u;
        const int pm = plane_mask(a.D.nz, p.k);
        uint32_t f = 0;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if ((pm >> s) & 1) f |= (ff_pos(s, 0) | ff_pos(s, 1) | ff_pos(s, 2)) * 0x10001u;
        return f;
    }
    __device__ __forceinline__ Pt at(int i, int j, int k, const int4& ci) const {
        Pt p = atf(i, j, k, ci);
        int fl = p.g == -1 ? 0xF : 0;
        if (p.g >= 0) {
            const uint32_t t4 = a.v.type4[p.g];
            fl = ((t4 & 0xFFu) ? 1 : 0) | ((t4 & 0xFF00u) ? 2 : 0) | ((t4 & 0xFF0000u) ? 4 : 0) |
                 ((t4 >> 24) ? 8 : 0);
        }
        p.fl = fl & plane_mask(a.D.nz, k);
        return p;
    }
    __device__ __forceinline__ Pt at(int i, int j, int k) const { return at(i, j, k, colinfo(i, j)); }
    __device__ __forceinline__ double st(const T* const (&U)[5], int f, int i, int j, int k) const {
        return (double)pick5(U, f)[fidx(a.D, f, i, j, k)];
    }
    __device__ __forceinline__ double geo(int s, int q, int g) const { return gq(a.v, s, q, g); }

    // advected quantity of field F (1 theta, 2..4 velocity) at a fluid CV from
    // the state; the density of the face is the mean over the fluid cells on
    // either side (lo_fluid: the cell below / left of the face is fluid)
    template <int F>
    __device__ __forceinline__ double phi_state(const Pt& p, bool lo_fluid) const {
        if (F == 1) return st(a.cur, 1, p.i, p.j, p.k) / st(a.cur, 0, p.i, p.j, p.k);
        int i0 = p.i, j0 = p.j, k0 = p.k;
        if (F == 2) i0 = wx(p.i - 1);
        if (F == 3) j0 = wy(p.j - 1);
        if (F == 4) k0 = p.k - 1;
        double s = 0.0;
        int cnt = 0;
        if (lo_fluid) { s += st(a.cur, 0, i0, j0, k0); ++cnt; }
        if (p.fl & 1) { s += st(a.cur, 0, p.i, p.j, p.k); ++cnt; }
        if (cnt == 0) return 0.0;
        // the mean over one or two cells: halving is exact, so this equals s / cnt
        return st(a.cur, F, p.i, p.j, p.k) / (cnt == 2 ? 0.5 * s : s);
    }
    // advected quantity at any stencil position
    template <int F>
    __device__ __forceinline__ double phi(const Pt& p) const {
        if (!((p.fl >> finst(F)) & 1)) return 0.0;
        if (p.g >= 0) return a.prim[4 * (size_t)p.g + (F - 1)];
        return phi_state<F>(p, true);  // above the range: the lower neighbour is fluid
    }
    // momentum component D at a position, zero where its CV is not fluid
    template <int D>
    __device__ __forceinline__ double mom(const Pt& p) const {
        return ((p.fl >> (D + 1)) & 1) ? st(a.cur, 2 + D, p.i, p.j, p.k) : 0.0;
    }
    // provisional flux of field F on the lower D-face of the CV at P, from the
    // four stencil positions (LL, L, P, RR) and the position below P along the
    // staggering direction of the field's instance (ls)
    template <int F, int D>
    __device__ __forceinline__ double fhat(const Pt& LL, const Pt& L, const Pt& P, const Pt& RR,
                                           const Pt& ls) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        if (D == 2) {
            if (s != 3 && (P.k == 0 || P.k == a.D.nz)) return 0.0;
            if (s == 3 && (P.k == 1 || P.k == a.D.nz)) return 0.0;
        }
        // staggered face: mean of the two face momenta next to it over those
        // whose CV holds fluid (mom gives 0 for the others)
        const bool both = ((ls.fl & P.fl) >> (D + 1)) & 1;
        const double m = s == 0 ? mom<D>(P) : (both ? 0.5 * (mom<D>(ls) + mom<D>(P)) : mom<D>(ls) + mom<D>(P));
        if (F == 0) return m;
        return m * upw<double>(m, phi<F>(LL), phi<F>(L), phi<F>(P), phi<F>(RR), (LL.fl >> s) & 1,
                               (RR.fl >> s) & 1);
    }
    // stencil of the lower D-face of P
    template <int D>
    __device__ __forceinline__ void stencil(const Pt& P, Pt& LL, Pt& L, Pt& RR) const {
        if (D == 0) {
            LL = at(wx(P.i - 2), P.j, P.k);
            L = at(wx(P.i - 1), P.j, P.k);
            RR = at(wx(P.i + 1), P.j, P.k);
        } else if (D == 1) {
            LL = at(P.i, wy(P.j - 2), P.k);
            L = at(P.i, wy(P.j - 1), P.k);
            RR = at(P.i, wy(P.j + 1), P.k);
        } else {
            const int4 ci = colinfo(P.i, P.j);
            LL = at(P.i, P.j, P.k - 2, ci);
            L = at(P.i, P.j, P.k - 1, ci);
            RR = at(P.i, P.j, P.k + 1, ci);
        }
    }
    // the position below P along the staggering direction of instance S
    template <int S>
    __device__ __forceinline__ Pt stag(const Pt& P) const {
        if (S == 1) return at(wx(P.i - 1), P.j, P.k);
        if (S == 2) return at(P.i, wy(P.j - 1), P.k);
        return at(P.i, P.j, P.k - 1, colinfo(P.i, P.j));
    }
    // provisional flux on the lower D-face of any CV (computed from scratch)
    template <int F, int D>
    __device__ __forceinline__ double fhat_at(const Pt& P) const {
        Pt LL, L, RR;
        stencil<D>(P, LL, L, RR);
        constexpr int s = F < 2 ? 0 : F - 1;
        const Pt ls = s == 0 ? P : stag<s == 0 ? 3 : s>(P);
        return fhat<F, D>(LL, L, P, RR, ls);
    }
    // provisional flux on the lower D-face of a CV in the range (pass-2 buffer)
    // or above it
    template <int F, int D>
    __device__ __forceinline__ double fhat_any(const Pt& P) const {
        if (P.ge >= 0) return a.fh[((size_t)F * 3 + D) * a.v.Ge + P.ge];
        return fhat_at<F, D>(P);
    }
    // area fraction of the lower D-face of the CV of instance S at P
    template <int S, int D>
    __device__ __forceinline__ double beta(const Pt& P) const {
        if (P.k == a.D.nz) return D == 2 ? 1.0 : 0.0;
        if (!((plane_mask(a.D.nz, P.k) >> S) & 1)) return 0.0;
        if (P.g == -2) return 0.0;
        if (P.g == -1) return 1.0;
        return geo(S, GQ_BX + D, P.g);
    }
    // area fraction x flux on the lower D-face of the CV at P, the flux moved
    // to the face centroid when the face is cut (precomputed record)
    template <int F, int D>
    __device__ __forceinline__ double bface(const Pt& P) const {
        return bface_pre<F, D>(P, a.fh[((size_t)F * 3 + D) * a.v.Ge + max(P.ge, 0)]);
    }
    // the same from the provisional flux F0 loaded beforehand (unconditionally,
    // from a valid index, so that all loads of a cell are issued together)
    template <int F, int D>
    __device__ __forceinline__ double bface_pre(const Pt& P, double F0) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        if (P.k == a.D.nz) return 0.0;  // top wall: zero flux
        if (!(P.ff & ff_pos(s, D))) return 0.0;
        // (every face read here lies in the stored face range: g1e is at least
        // the -x and -y neighbours' g1, and g1 + 1 for a non-empty range)
        if (P.ff & ff_full(s, D)) return F0;
        // partial face: interpolated by the cut-face pass (record order)
        const uint32_t part = (P.ff & 0xFFFu) & ~(P.ff >> 16);
        const int r = a.cbase[P.g] + __popc(part & (ff_pos(s, D) - 1u));
        return a.bfc[(F == 1 ? (size_t)a.ncut : 0) + r];
    }
    // area fraction with a runtime instance (set-up only)
    template <int D>
    __device__ double beta_rt(int s, const Pt& P) const {
        if (P.k == a.D.nz) return D == 2 ? 1.0 : 0.0;
        if (!((plane_mask(a.D.nz, P.k) >> s) & 1)) return 0.0;
        if (P.g == -2) return 0.0;
        if (P.g == -1) return 1.0;
        return geo(s, GQ_BX + D, P.g);
    }
    // Builds the record of the partial lower D-face of instance s at the general
    // CV P: neighbours chosen by the signs of the face-centroid offsets (first
    // tangential axis y for x-faces and x otherwise, second y for z-faces and z
    // otherwise), weights from their magnitudes, all-or-nothing when a
    // neighbour face has no fluid or lies beyond a wall.  Returns false if a
    // neighbour face lies outside the stored face range.
    template <int D>
    __device__ bool cut_record(int s, const Pt& P, CutRec& r) const {
        const double b = geo(s, GQ_BX + D, P.g);
        r.n[0] = r.n[1] = r.n[2] = -1;
        r.own = P.ge;
        r.sd = s * 3 + D;
        r.pad = 0;
        r.b = b;
        r.c[0] = 1.0;
        r.c[1] = r.c[2] = r.c[3] = 0.0;
        if (!(b < 1.0)) return true;
        const double g1 = geo(s, GQ_FX1 + 2 * D, P.g), g2 = geo(s, GQ_FX1 + 2 * D + 1, P.g);
        // offsets within 1e-12 of zero count as none (a face cut by a
        // vertical wall has its centroid at mid-height up to rounding)
        const int s1 = g1 > 1e-12 ? 1 : (g1 < -1e-12 ? -1 : 0);
        const int s2 = g2 > 1e-12 ? 1 : (g2 < -1e-12 ? -1 : 0);
        if (s1 == 0 && s2 == 0) return true;
        const int ax = D == 0 ? 0 : s1, ay = D == 0 ? s1 : 0;
        const int by = D == 2 ? s2 : 0, bz = D == 2 ? 0 : s2;
        const bool u1 = s1 != 0, u2 = s2 != 0, u12 = u1 && u2;
        if (u2 && bz != 0 && !((plane_mask(a.D.nz, P.k + bz) >> s) & 1)) return true;
        Pt N1, N2, N12;
        if (u1) {
            N1 = at(wx(P.i + ax), wy(P.j + ay), P.k);
            if (!(beta_rt<D>(s, N1) > 0.0)) return true;
        }
        if (u2) {
            N2 = at(P.i, wy(P.j + by), P.k + bz);
            if (!(beta_rt<D>(s, N2) > 0.0)) return true;
        }
        if (u12) {
            N12 = at(wx(P.i + ax), wy(P.j + ay + by), P.k + bz);
            if (!(beta_rt<D>(s, N12) > 0.0)) return true;
        }
        const double w1 = u1 ? fabs(g1) : 0.0, w2 = u2 ? fabs(g2) : 0.0;
        r.c[0] = (1.0 - w1) * (1.0 - w2);
        bool ok = true;
        if (u1) { r.n[0] = N1.ge; r.c[1] = w1 * (1.0 - w2); ok &= N1.ge >= 0; }
        if (u2) { r.n[1] = N2.ge; r.c[2] = (1.0 - w1) * w2; ok &= N2.ge >= 0; }
        if (u12) { r.n[2] = N12.ge; r.c[3] = w1 * w2; ok &= N12.ge >= 0; }
        return ok;
    }
    template <int F, int D, bool EB>
    __device__ __forceinline__ double div_pre(const Pt& P, const Pt& U, int g, double Fp, double Fu) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        const double rd = a.rdel[D];
        double br = (bface_pre<F, D>(U, Fu) - bface_pre<F, D>(P, Fp)) * rd;
        if (EB) {
            const double blo = beta<s, D>(P), bhi = beta<s, D>(U);
            double sm = 0.0;
            int cnt = 0;
            if (blo > 0.0) { sm += fhat_any<F, D>(P); ++cnt; }
            if (bhi > 0.0) { sm += U.k == a.D.nz ? 0.0 : fhat_any<F, D>(U); ++cnt; }
            const double fb = cnt ? sm / cnt : 0.0;
            br -= geo(s, GQ_AX + D, g) * fb * rd;
        }
        return br;
    }
    template <int F, bool EB>
    __device__ __forceinline__ void update(const Pt& P, const Pt& Ux, const Pt& Uy, const Pt& Uz, int g) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        // every load of this field first, from valid indices
        const size_t Ge = a.v.Ge;
        const double* f0 = a.fh + ((size_t)F * 3 + 0) * Ge;
        const double* f1 = a.fh + ((size_t)F * 3 + 1) * Ge;
        const double* f2 = a.fh + ((size_t)F * 3 + 2) * Ge;
        const int pe = max(P.ge, 0);
        const double Fp0 = f0[pe], Fp1 = f1[pe], Fp2 = f2[pe];
        const double Fu0 = f0[max(Ux.ge, 0)], Fu1 = f1[max(Uy.ge, 0)], Fu2 = f2[max(Uz.ge, 0)];
        const double al = geo(s, GQ_ALPHA, g);
        const double unv = st(a.un, F, P.i, P.j, P.k);
        double val = 0.0;
        if ((P.fl >> s) & 1) {
            double br = div_pre<F, 0, EB>(P, Ux, g, Fp0, Fu0);
            br += div_pre<F, 1, EB>(P, Uy, g, Fp1, Fu1);
            br += div_pre<F, 2, EB>(P, Uz, g, Fp2, Fu2);
            val = unv - a.cdt * br / al;
        }
        a.uhat[(size_t)F * a.v.G + g] = val;
        put_field<T>(a.D, a.out, F, P.i, P.j, P.k, (T)val);
    }
    // ---- update from the update table (no test-mode EB flux)
    // area fraction x flux on the lower D-face described by u (zero without
    // fluid; the stored flux on a full face; the interpolated one otherwise)
    template <int F, int D>
    __device__ __forceinline__ double bface_u(const UPt& u, double F0) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        if (!(u.ff & ff_pos(s, D))) return 0.0;
        if (u.ff & ff_full(s, D)) return F0;
        const uint32_t part = (u.ff & 0xFFFu) & ~(u.ff >> 16);
        return a.bfc[(F == 1 ? (size_t)a.ncut : 0) + u.rb + __popc(part & (ff_pos(s, D) - 1u))];
    }
    template <int F>
    __device__ __forceinline__ void update_t(int fl, const UPt& P, const UPt (&U)[3], int i, int j, int k,
                                             int g, double src = 0.0) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        const size_t Ge = a.v.Ge;
        const double* f0 = a.fh + ((size_t)F * 3 + 0) * Ge;
        const double* f1 = a.fh + ((size_t)F * 3 + 1) * Ge;
        const double* f2 = a.fh + ((size_t)F * 3 + 2) * Ge;
        const double Fp0 = f0[P.ge], Fp1 = f1[P.ge], Fp2 = f2[P.ge];
        const double Fu0 = f0[U[0].ge], Fu1 = f1[U[1].ge], Fu2 = f2[U[2].ge];
        const double al = geo(s, GQ_ALPHA, g);
        const double unv = st(a.un, F, i, j, k);
        double val = 0.0;
        if ((fl >> s) & 1) {
            double br = (bface_u<F, 0>(U[0], Fu0) - bface_u<F, 0>(P, Fp0)) * a.rdel[0];
            br += (bface_u<F, 1>(U[1], Fu1) - bface_u<F, 1>(P, Fp1)) * a.rdel[1];
            br += (bface_u<F, 2>(U[2], Fu2) - bface_u<F, 2>(P, Fp2)) * a.rdel[2];
            val = unv - a.cdt * br / al;
            if (F >= 2 && a.srcv) val += a.cdt * src;
        }
        a.uhat[(size_t)F * a.v.G + g] = val;
        put_field<T>(a.D, a.out, F, i, j, k, (T)val);
    }

    // ---- provisional fluxes from the stencil table: every advected quantity
    // a face-range stencil reads is a load from the advected-quantity array
    struct PV {
        double q[4];
    };
    __device__ __forceinline__ PV loadpv(const SPt& p) const {
        const double* b = a.prim + 4 * (size_t)p.pi;
        PV v;
        v.q[0] = b[0];
        v.q[1] = b[1];
        v.q[2] = b[2];
        v.q[3] = b[3];
        return v;
    }
    template <int F>
    __device__ __forceinline__ double phit(const SPt& p, const PV& v) const {
        return ((p.fl >> finst(F)) & 1) ? v.q[F - 1] : 0.0;
    }
    // momentum component D, loaded unconditionally from a clamped plane
    template <int D>
    __device__ __forceinline__ double momt(const SPt& p) const {
        const double v = st(a.cur, 2 + D, p.i, p.j, min(max(p.k, 0), a.D.nz - 1));
        return ((p.fl >> (D + 1)) & 1) ? v : 0.0;
    }
    // mass flux of a staggered face: mean of the two face momenta next to it
    // over those whose CV holds fluid (momt gives 0 for the others), so one
    // fluid CV gives its own momentum
    template <int F, int D>
    __device__ __forceinline__ double fhatt(const SPt& LL, const SPt& L, const SPt& P, const SPt& RR,
                                            const PV& vLL, const PV& vL, const PV& vP, const PV& vRR,
                                            double m0, double mls, bool both) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        if (D == 2) {
            if (s != 3 && (P.k == 0 || P.k == a.D.nz)) return 0.0;
            if (s == 3 && (P.k == 1 || P.k == a.D.nz)) return 0.0;
        }
        const double m = s == 0 ? m0 : (both ? 0.5 * (mls + m0) : mls + m0);
        if (F == 0) return m;
        return m * upw<double>(m, phit<F>(LL, vLL), phit<F>(L, vL), phit<F>(P, vP), phit<F>(RR, vRR),
                               (LL.fl >> s) & 1, (RR.fl >> s) & 1);
    }
    // the 15 lower-face fluxes of direction D at table slot set S (slot 0 the
    // CV, 1 + 3 D .. 3 + 3 D the positions -2, -1, +1 along D)
    template <int D>
    __device__ __forceinline__ void fhat_dirt(const SPt (&S)[10], const PV& vP, uint32_t ff, int e) const {
        const SPt& P = S[0];
        const SPt& LL = S[1 + 3 * D];
        const SPt& L = S[2 + 3 * D];
        const SPt& RR = S[3 + 3 * D];
        const size_t G = a.v.Ge;
        const PV vLL = loadpv(LL), vL = loadpv(L), vRR = loadpv(RR);
        // mass fluxes: component D at P and below P along x, y, z
        const double m0 = momt<D>(P), mx = momt<D>(S[2]), my = momt<D>(S[5]), mz = momt<D>(S[8]);
        // are the D-momentum CVs at P and below P along x, y, z all fluid
        const int f0 = (P.fl >> (D + 1)) & 1;
        const bool bx = f0 & (S[2].fl >> (D + 1)), by = f0 & (S[5].fl >> (D + 1)), bz = f0 & (S[8].fl >> (D + 1));
        a.fh[(0 * 3 + D) * G + e] = (ff & ff_pos(0, D)) ? fhatt<0, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, m0, true) : 0.0;
        a.fh[(1 * 3 + D) * G + e] = (ff & ff_pos(0, D)) ? fhatt<1, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, m0, true) : 0.0;
        a.fh[(2 * 3 + D) * G + e] = (ff & ff_pos(1, D)) ? fhatt<2, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, mx, bx) : 0.0;
        a.fh[(3 * 3 + D) * G + e] = (ff & ff_pos(2, D)) ? fhatt<3, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, my, by) : 0.0;
        a.fh[(4 * 3 + D) * G + e] = (ff & ff_pos(3, D)) ? fhatt<4, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, mz, bz) : 0.0;
    }
    // table code of a stencil position (set-up): index into the
    // advected-quantity array | fluid bits << 28; 0 where no instance is
    // fluid (below the range, beyond the walls).  ok is cleared when an aux
    // position beyond its column's aux range is needed.
    __device__ uint32_t sten_code(int i, int j, int k, const int32_t* gp, const int32_t* aoff, bool& ok) const {
        if (k < 0 || k >= a.D.nz) return 0u;
        const int c = j * a.D.nx + i;
        const int4 ci = a.v.col[c];
        const Pt p = at(i, j, k, ci);
        if (p.g >= 0) return (uint32_t)p.g | ((uint32_t)p.fl << 28);
        if (p.g == -2) return 0u;
        if (k >= gp[c]) {
            ok = false;
            return 0u;
        }
        return (uint32_t)(a.v.G + aoff[c] + (k - col_g1(ci))) | ((uint32_t)p.fl << 28);
    }
};

// slot offsets of the stencil table: the CV, then -2, -1, +1 along x, y, z
constexpr int8_t kStenOff[10][3] = {{0, 0, 0},  {-2, 0, 0}, {-1, 0, 0}, {1, 0, 0},  {0, -2, 0},
                                             {0, -1, 0}, {0, 1, 0},  {0, 0, -2}, {0, 0, -1}, {0, 0, 1}};

__device__ inline void gen_cell(const GeoView& v, int g, int& i, int& j, int& k, int4& ci) {
    const int c = v.gcol[g];
    ci = v.col[c];
    i = c % v.nx;
    j = c / v.nx;
    k = col_g0(ci) + (g - ci.z);
}
// cell of the extended face range
__device__ inline void face_cell(const GeoView& v, int e, int& i, int& j, int& k, int4& ci) {
    const int c = v.gcole[e];
    ci = v.col[c];
    i = c % v.nx;
    j = c / v.nx;
    k = col_g0(ci) + (e - ci.w);
}

// Positions per thread of the prims pass: every load of both is issued
// before the arithmetic of either, so a wave keeps twice the gathers in
// flight (the pass uses few registers, so occupancy does not drop).
constexpr int GEN_CO = 2;

// the state values the advected quantities of a position read: rho, rho
// theta, the three momenta at the position and rho below it along x, y, z
struct PrimIn {
    double r, rt, mu, mv, mw, rx, ry, rz;
};

template <typename T>
__global__ void __launch_bounds__(256) k_gen_prims(GenArgs<T> a) {
    const int n = a.v.G + a.naux;
    const int base = xcd_block() * (GEN_CO * 256) + threadIdx.x;
    const Gen<T> G(a);
    int4 t[GEN_CO];
    PrimIn in[GEN_CO];
#pragma unroll
    for (int u = 0; u < GEN_CO; ++u) {
        const int p = base + u * 256;
        t[u] = a.ptab[min(p, n - 1)];
    }
#pragma unroll
    for (int u = 0; u < GEN_CO; ++u) {
        const int i = t[u].x, j = t[u].y, k = t[u].z;
        in[u].r = G.st(a.cur, 0, i, j, k);
        in[u].rt = G.st(a.cur, 1, i, j, k);
        in[u].mu = G.st(a.cur, 2, i, j, k);
        in[u].mv = G.st(a.cur, 3, i, j, k);
        in[u].mw = G.st(a.cur, 4, i, j, k);
        in[u].rx = G.st(a.cur, 0, G.wx(i - 1), j, k);
        in[u].ry = G.st(a.cur, 0, i, G.wy(j - 1), k);
        in[u].rz = G.st(a.cur, 0, i, j, max(k - 1, 0));
    }
#pragma unroll
    for (int u = 0; u < GEN_CO; ++u) {
        const int p = base + u * 256;
        if (p >= n) break;
        const int fl = t[u].w & 0xF;
        const PrimIn& v = in[u];
        // face density: mean over the fluid cells on either side (the lower
        // one flagged in bits 4-6); halving is exact, so this equals s / cnt
        auto face = [&](double lo, int lbit) -> double {
            const bool l = (t[u].w >> lbit) & 1, o = fl & 1;
            if (l && o) return 0.5 * (lo + v.r);
            return l ? lo : v.r;
        };
        auto vel = [&](double m, double lo, int lbit) -> double {
            const bool l = (t[u].w >> lbit) & 1, o = fl & 1;
            if (!l && !o) return 0.0;
            return m / face(lo, lbit);
        };
        double* o = a.prim + 4 * (size_t)p;
        o[0] = (fl & 1) ? v.rt / v.r : 0.0;
        o[1] = (fl & 2) ? vel(v.mu, v.rx, 4) : 0.0;
        o[2] = (fl & 4) ? vel(v.mv, v.ry, 5) : 0.0;
        o[3] = (fl & 8) ? vel(v.mw, v.rz, 6) : 0.0;
        if (a.srcv) {
            // perturbation pressure (equation of state) and density of a fluid cell
            double pp = 0.0, rp = 0.0;
            if (fl & 1) {
                const int k = t[u].z;
                const double rt0 = a.sref[a.D.nz + k];
                pp = a.sref[k] * expm1(a.sgam * log1p((v.rt - rt0) / rt0));
                rp = v.r - a.sref[4 * a.D.nz + k];
            }
            a.srcv[2 * (size_t)p] = pp;
            a.srcv[2 * (size_t)p + 1] = rp;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_gen_fhat(GenArgs<T> a) {
    const int e = xcd_block() * blockDim.x + threadIdx.x;  // extended face range
    if (e >= a.v.Ge) return;
    const Gen<T> G(a);
    const int4 t = a.ftab[e];
    const int i = t.x, j = t.y, k = t.z;
    const uint32_t ff = (uint32_t)t.w;  // lower-face flags of the CV
    SPt S[10];
#pragma unroll
    for (int q = 0; q < 10; ++q) {
        const uint32_t cd = a.sten[(size_t)q * a.v.Ge + e];
        S[q].i = G.wx(i + kStenOff[q][0]);
        S[q].j = G.wy(j + kStenOff[q][1]);
        S[q].k = k + kStenOff[q][2];
        S[q].fl = (int)(cd >> 28);
        S[q].pi = cd & 0x0FFFFFFFu;
    }
    const auto vP = G.loadpv(S[0]);
    G.template fhat_dirt<0>(S, vP, ff, e);
    G.template fhat_dirt<1>(S, vP, ff, e);
    G.template fhat_dirt<2>(S, vP, ff, e);
}

// update with the test-mode embedded-boundary flux (positions resolved from
// the column ranges; the production update below reads the update table)
template <typename T>
__global__ void __launch_bounds__(256) k_gen_update_eb(GenArgs<T> a) {
    constexpr bool EB = true;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.v.G) return;
    const Gen<T> G(a);
    int i, j, k;
    int4 ci;
    gen_cell(a.v, g, i, j, k, ci);
    Pt P = G.at(i, j, k, ci);
    P.ff = G.fflags(P);
    // the upper neighbours: their lower faces are this CV's upper faces
    const int ip = G.wx(i + 1), jp = G.wy(j + 1);
    Pt Ux = G.atf(ip, j, k, G.colinfo(ip, j)), Uy = G.atf(i, jp, k, G.colinfo(i, jp)), Uz = G.atf(i, j, k + 1, ci);
    Ux.ff = G.fflags(Ux);
    Uy.ff = G.fflags(Uy);
    Uz.ff = G.fflags(Uz);
    G.template update<0, EB>(P, Ux, Uy, Uz, g);
    G.template update<1, EB>(P, Ux, Uy, Uz, g);
    G.template update<2, EB>(P, Ux, Uy, Uz, g);
    G.template update<3, EB>(P, Ux, Uy, Uz, g);
    G.template update<4, EB>(P, Ux, Uy, Uz, g);
}

// the update (EB flux zero), from the update table
template <typename T>
__global__ void __launch_bounds__(256) k_gen_update(GenArgs<T> a) {
    const int g = xcd_block() * blockDim.x + threadIdx.x;
    if (g >= a.v.G) return;
    const Gen<T> G(a);
    const int Gn = a.v.G;
    UPt U[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        U[d].ge = a.upd[(size_t)d * Gn + g];
        U[d].ff = (uint32_t)a.upd[(size_t)(3 + d) * Gn + g];
        U[d].rb = a.upd[(size_t)(6 + d) * Gn + g];
    }
    const int4 t = a.utab[g];
    const int i = t.x, j = t.y, k = t.z & 0xFFFF, fl = t.z >> 16;
    const UPt P{t.w, a.v.fflag[g], a.cbase[g]};
    // momentum sources: p' and rho' of this cell and of its lower neighbours
    // along x, y, z (stencil-table slots 2, 5, 8 name their positions and
    // whether they are fluid cells)
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (a.srcv) {
        const size_t Ge = a.v.Ge;
        const uint32_t cx = a.sten[2 * Ge + t.w], cy = a.sten[5 * Ge + t.w], cz = a.sten[8 * Ge + t.w];
        const bool fo = fl & 1, fx = (cx >> 28) & 1u, fy = (cy >> 28) & 1u, fz = (cz >> 28) & 1u;
        const double po = fo ? a.srcv[2 * (size_t)g] : 0.0, ro = fo ? a.srcv[2 * (size_t)g + 1] : 0.0;
        const double pz = fz ? a.srcv[2 * (size_t)(cz & 0x0FFFFFFFu)] : 0.0;
        const double rz = fz ? a.srcv[2 * (size_t)(cz & 0x0FFFFFFFu) + 1] : 0.0;
        if (fo && fx) sx = -(po - a.srcv[2 * (size_t)(cx & 0x0FFFFFFFu)]) * a.rdel[0];
        if (fo && fy) sy = -(po - a.srcv[2 * (size_t)(cy & 0x0FFFFFFFu)]) * a.rdel[1];
        if (fo && fz) sz = -(po - pz) * a.rdel[2];
        const int cnt = (int)fo + (int)fz;
        if (cnt) sz -= a.sg * ((ro + rz) / cnt);
    }
    G.template update_t<0>(fl, P, U, i, j, k, g);
    G.template update_t<1>(fl, P, U, i, j, k, g);
    G.template update_t<2>(fl, P, U, i, j, k, g, sx);
    G.template update_t<3>(fl, P, U, i, j, k, g, sy);
    G.template update_t<4>(fl, P, U, i, j, k, g, sz);
}

// Area fraction x flux moved to the centroid on every partial face, for the
// field(s) of the face's instance (slot 1: rho theta of the cell-centred CVs).
// The records are stored as structure of arrays, so each of their loads
// reads consecutive words across the wave.
template <typename T>
__global__ void __launch_bounds__(256) k_gen_cut(GenArgs<T> a) {
    const int r = xcd_block() * blockDim.x + threadIdx.x;
    if (r >= a.ncut) return;
    const size_t N = a.ncut;
    const int4 nn = a.cut_n[r];
    const int own = nn.w & 0x0FFFFFFF, sd = (int)((uint32_t)nn.w >> 28);
    const double b = a.cut_w[r], c0 = a.cut_w[N + r], c1 = a.cut_w[2 * N + r], c2 = a.cut_w[3 * N + r],
                 c3 = a.cut_w[4 * N + r];
    const int s = sd / 3, d = sd - 3 * s;
    const int n0 = max(nn.x, 0), n1 = max(nn.y, 0), n2 = max(nn.z, 0);
    for (int q = 0; q < (s == 0 ? 2 : 1); ++q) {
        const int f = s == 0 ? q : s + 1;
        const double* fhd = a.fh + ((size_t)f * 3 + d) * a.v.Ge;
        const double F0 = fhd[own], F1 = fhd[n0], F2 = fhd[n1], F3 = fhd[n2];
        double Fv = c0 * F0;
        if (nn.x >= 0) Fv += c1 * F1;
        if (nn.y >= 0) Fv += c2 * F2;
        if (nn.z >= 0) Fv += c3 * F3;
        a.bfc[(size_t)q * N + r] = b * Fv;
    }
}

// the records as structure of arrays (set-up)
__global__ void __launch_bounds__(256) k_cut_soa(const CutRec* rec, int32_t n, int4* cn, double* cw) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const CutRec c = rec[r];
    cn[r] = make_int4(c.n[0], c.n[1], c.n[2], (int32_t)((uint32_t)c.own | ((uint32_t)c.sd << 28)));
    const size_t N = n;
    cw[r] = c.b;
    for (int q = 0; q < 4; ++q) cw[(q + 1) * N + r] = c.c[q];
}

// number of partial lower faces (area fraction > 0 and not exactly 1) per general cell
__global__ void __launch_bounds__(256) k_cut_count(GeoView v, int32_t* cnt) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= v.G) return;
    const uint32_t ff = v.fflag[g];
    cnt[g] = __popc((ff & 0xFFFu) & ~(ff >> 16));
}

__global__ void __launch_bounds__(128) k_cut_fill(GenArgs<double> a, CutRec* rec, int32_t* bad) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.v.G) return;
    const Gen<double> G(a);
    int i, j, k;
    int4 ci;
    gen_cell(a.v, g, i, j, k, ci);
    const Pt P = G.at(i, j, k, ci);
    const uint32_t ff = a.v.fflag[g];
    const uint32_t part = (ff & 0xFFFu) & ~(ff >> 16);
    int r = a.cbase[g];
    bool ok = true;
    for (int s = 0; s < 4; ++s) {
        if (part & ff_pos(s, 0)) ok &= G.template cut_record<0>(s, P, rec[r++]);
        if (part & ff_pos(s, 1)) ok &= G.template cut_record<1>(s, P, rec[r++]);
        if (part & ff_pos(s, 2)) ok &= G.template cut_record<2>(s, P, rec[r++]);
    }
    if (!ok) atomicAdd(bad, 1);
}

// stencil table of the face range (set-up)
__global__ void __launch_bounds__(256) k_sten_fill(GenArgs<double> a, const int32_t* gp, const int32_t* aoff,
                                                   uint32_t* sten, int4* ftab, int32_t* bad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.v.Ge) return;
    const Gen<double> G(a);
    int i, j, k;
    int4 ci;
    face_cell(a.v, e, i, j, k, ci);
    // lower-face flags (stored in the general range; above it every face of a
    // plane holding CVs is full)
    ftab[e] = make_int4(i, j, k, (int)G.fflags(G.atf(i, j, k, ci)));
    bool ok = true;
    for (int q = 0; q < 10; ++q)
        sten[(size_t)q * a.v.Ge + e] =
            G.sten_code(G.wx(i + kStenOff[q][0]), G.wy(j + kStenOff[q][1]), k + kStenOff[q][2], gp, aoff, ok);
    if (!ok) atomicAdd(bad, 1);
}

// update table (set-up): for each general cell, the lower faces of its +x, +y
// and +z neighbours (its own upper faces)
__global__ void __launch_bounds__(256) k_upd_fill(GenArgs<double> a, int32_t* upd, int4* utab, int32_t* bad) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.v.G) return;
    const Gen<double> G(a);
    int i, j, k;
    int4 ci;
    gen_cell(a.v, g, i, j, k, ci);
    utab[g] = make_int4(i, j, k | (G.at(i, j, k, ci).fl << 16), ci.w + (k - col_g0(ci)));
    const int ip = G.wx(i + 1), jp = G.wy(j + 1);
    const Pt U[3] = {G.atf(ip, j, k, G.colinfo(ip, j)), G.atf(i, jp, k, G.colinfo(i, jp)),
                     G.atf(i, j, k + 1, ci)};
    const size_t Gn = a.v.G;
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
        const uint32_t ff = G.fflags(U[d]);
        // a face with fluid must lie in the stored face range
        if (ff != 0u && U[d].ge < 0) ok = false;
        upd[d * Gn + g] = max(U[d].ge, 0);
        upd[(3 + d) * Gn + g] = (int32_t)ff;
        upd[(6 + d) * Gn + g] = U[d].g >= 0 ? a.cbase[U[d].g] : 0;
    }
    if (!ok) atomicAdd(bad, 1);
}

// cell table of the prims pass (set-up): general cells, then aux positions
__global__ void __launch_bounds__(256) k_ptab_fill(GenArgs<double> a, const int2* aux, int4* ptab) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.v.G + a.naux) return;
    const Gen<double> G(a);
    int i, j, k, bits;
    if (p < a.v.G) {
        int4 ci;
        gen_cell(a.v, p, i, j, k, ci);
        const int lx = G.at(G.wx(i - 1), j, k).fl & 1;
        const int ly = G.at(i, G.wy(j - 1), k).fl & 1;
        const int lz = G.at(i, j, k - 1, ci).fl & 1;
        bits = G.at(i, j, k, ci).fl | lx << 4 | ly << 5 | lz << 6;
    } else {
        // above the general range: every CV there and below it is fluid
        const int2 ck = aux[p - a.v.G];
        i = ck.x % a.v.nx;
        j = ck.x / a.v.nx;
        k = ck.y;
        bits = G.at(i, j, k, a.v.col[ck.x]).fl | 0x70;
    }
    ptab[p] = make_int4(i, j, k, bits);
}

}  // namespace

// ------------------------------------------------------------- host side
ebs_status build_cut_faces(ebs_ctx* cx) {
    const int32_t G = cx->G;
    if (cx->d_cbase) (void)hipFree(cx->d_cbase);
    if (cx->d_cut_n) (void)hipFree(cx->d_cut_n);
    if (cx->d_cut_w) (void)hipFree(cx->d_cut_w);
    cx->d_cbase = nullptr;
    cx->d_cut_n = nullptr;
    cx->d_cut_w = nullptr;
    cx->ncut = 0;
    if (G == 0) return EBS_OK;
    int32_t* d_bad = nullptr;
    if (hipMalloc(&cx->d_cbase, sizeof(int32_t) * G) != hipSuccess ||
        hipMalloc(&d_bad, sizeof(int32_t)) != hipSuccess) {
        if (d_bad) (void)hipFree(d_bad);
        cx->err = "cut-face table allocation failed";
        return EBS_E_OOM;
    }
    const GeoView v = geo_view(cx);
    hipLaunchKernelGGL(k_cut_count, dim3((G + 255) / 256), dim3(256), 0, cx->stream, v, cx->d_cbase);
    EBS_HIP(cx, hipGetLastError());
    std::vector<int32_t> cnt(G);
    EBS_HIP(cx, hipMemcpyAsync(cnt.data(), cx->d_cbase, sizeof(int32_t) * G, hipMemcpyDeviceToHost, cx->stream));
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    int64_t tot = 0;
    for (int32_t g = 0; g < G; ++g) {
        const int32_t n = cnt[g];
        cnt[g] = (int32_t)tot;
        tot += n;
    }
    if (tot > INT32_MAX / 2) {
        (void)hipFree(d_bad);
        cx->err = "too many cut faces";
        return EBS_E_UNSUPPORTED;
    }
    if (cx->Ge >= (1 << 28)) {  // face-range indices share a word with (instance, direction)
        (void)hipFree(d_bad);
        cx->err = "face range too large for the cut-face records";
        return EBS_E_UNSUPPORTED;
    }
    cx->ncut = (int32_t)tot;
    if (cx->d_bfc) (void)hipFree(cx->d_bfc);
    cx->d_bfc = nullptr;
    const int64_t n1 = std::max<int64_t>(tot, 1);
    CutRec* rec = nullptr;  // the records as built (set-up only)
    auto fail = [&](ebs_status st, const char* msg) {
        if (rec) (void)hipFree(rec);
        (void)hipFree(d_bad);
        cx->err = msg;
        return st;
    };
    if (hipMalloc(&rec, sizeof(CutRec) * n1) != hipSuccess || hipMalloc(&cx->d_bfc, sizeof(double) * 2 * n1) != hipSuccess ||
        hipMalloc(&cx->d_cut_n, sizeof(int4) * n1) != hipSuccess ||
        hipMalloc(&cx->d_cut_w, sizeof(double) * 5 * n1) != hipSuccess)
        return fail(EBS_E_OOM, "cut-face table allocation failed");
    auto hip_ok = [&](hipError_t e) { return e == hipSuccess; };
    if (!hip_ok(hipMemcpyAsync(cx->d_cbase, cnt.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, cx->stream)) ||
        !hip_ok(hipMemsetAsync(d_bad, 0, sizeof(int32_t), cx->stream)))
        return fail(EBS_E_HIP, "cut-face table upload failed");
    GenArgs<double> a{};
    a.D = Dims{cx->nx, cx->ny, cx->nz};
    a.v = v;
    a.cbase = cx->d_cbase;
    hipLaunchKernelGGL(k_cut_fill, dim3((G + 127) / 128), dim3(128), 0, cx->stream, a, rec, d_bad);
    int32_t bad = 0;
    if (!hip_ok(hipGetLastError()) ||
        !hip_ok(hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, cx->stream)) ||
        !hip_ok(hipStreamSynchronize(cx->stream)))
        return fail(EBS_E_HIP, "cut-face record build failed");
    if (bad != 0) return fail(EBS_E_UNSUPPORTED, "a cut-face interpolation neighbour lies outside the stored face range");
    if (tot > 0) {
        hipLaunchKernelGGL(k_cut_soa, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, cx->stream, rec, (int32_t)tot,
                           cx->d_cut_n, cx->d_cut_w);
        if (!hip_ok(hipGetLastError()) || !hip_ok(hipStreamSynchronize(cx->stream)))
            return fail(EBS_E_HIP, "cut-face record build failed");
    }
    (void)hipFree(rec);
    (void)hipFree(d_bad);
    return EBS_OK;
}

// Stencil and update tables.  Every position a provisional-flux stencil
// of the face range reads (the CV and -2, -1, +1 along each axis) is resolved
// once: general cells by their index, positions above their column's general
// range by an index in a list of aux positions appended to the general range
// (whose advected quantities the prims pass computes as well), and positions
// with no fluid CV by code 0.  The aux range of a column is [g1, gp), gp the
// highest plane any face-range stencil reads there, plus one.  The update
// table holds, for each general cell, the lower faces of its +x, +y and +z
// neighbours: their index in the face range, their flags and the first
// cut-face record of their CV.
ebs_status build_stencils(ebs_ctx* cx) {
    for (void** q : {(void**)&cx->d_sten, (void**)&cx->d_upd, (void**)&cx->d_ptab, (void**)&cx->d_ftab,
                     (void**)&cx->d_utab, (void**)&cx->d_acol}) {
        if (*q) (void)hipFree(*q);
        *q = nullptr;
    }
    cx->naux = 0;
    const int nx = cx->nx, ny = cx->ny, nz = cx->nz, ncol = nx * ny;
    const int32_t G = cx->G, Ge = cx->Ge;
    const std::vector<int32_t>& g0 = cx->h_g0;
    const std::vector<int32_t>& g1 = cx->h_g1;
    const std::vector<int32_t>& g1e = cx->h_g1e;
    std::vector<int32_t> gp(g1);
    auto cid = [&](int i, int j) { return ((j % ny + ny) % ny) * nx + ((i % nx + nx) % nx); };
    for (int c = 0; c < ncol; ++c) {
        if (g1e[c] <= g0[c]) continue;  // empty face range: reads nothing
        const int i = c % nx, j = c / nx;
        gp[c] = std::max(gp[c], std::min(nz, g1e[c] + 1));
        for (int d : {-2, -1, 1}) {
            int& a = gp[cid(i + d, j)];
            a = std::max(a, g1e[c]);
            int& b = gp[cid(i, j + d)];
            b = std::max(b, g1e[c]);
        }
    }
    // With diffusion the fits of the general cells' faces and facets, and
    // the centred differences, read theta and velocities up to two cells
    // away in every direction (diagonals included): up to level g1 + 1 of
    // every column within two columns of a general one.
    if (cx->visc_on || cx->diff_on)
        for (int c = 0; c < ncol; ++c) {
            if (g1[c] <= g0[c]) continue;
            const int i = c % nx, j = c / nx, top = std::min(nz, g1[c] + 2);
            for (int dj = -2; dj <= 2; ++dj)
                for (int di = -2; di <= 2; ++di) {
                    int& a = gp[cid(i + di, j + dj)];
                    a = std::max(a, top);
                }
        }
    std::vector<int32_t> aoff(ncol);
    int64_t A = 0;
    for (int c = 0; c < ncol; ++c) {
        aoff[c] = (int32_t)A;
        A += gp[c] - g1[c];
    }
    if ((int64_t)G + A >= (int64_t)1 << 28) {
        cx->err = "general region too large for the stencil table";
        return EBS_E_UNSUPPORTED;
    }
    std::vector<int2> aux((size_t)std::max<int64_t>(A, 1));
    for (int c = 0; c < ncol; ++c)
        for (int k = g1[c]; k < gp[c]; ++k) aux[aoff[c] + (k - g1[c])] = make_int2(c, k);
    cx->naux = (int32_t)A;
    cx->h_gp = gp;
    cx->h_aoff = aoff;
    const size_t P = (size_t)std::max<int64_t>(G + A, 1);
    const size_t Gs = (size_t)std::max(G, 1), Ges = (size_t)std::max(Ge, 1);
    if (cx->d_prim) (void)hipFree(cx->d_prim);
    cx->d_prim = nullptr;
    if (cx->d_srcv) (void)hipFree(cx->d_srcv);
    cx->d_srcv = nullptr;
    int32_t *d_gp = nullptr, *d_aoff = nullptr, *d_bad = nullptr;
    int2* d_aux = nullptr;
    bool ok = hipMalloc(&cx->d_prim, sizeof(double) * 4 * P) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_srcv, sizeof(double) * 2 * P) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_ptab, sizeof(int4) * P) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_sten, sizeof(uint32_t) * 10 * Ges) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_ftab, sizeof(int4) * Ges) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_upd, sizeof(int32_t) * 9 * Gs) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_utab, sizeof(int4) * Gs) == hipSuccess;
    ok = ok && hipMalloc(&d_aux, sizeof(int2) * aux.size()) == hipSuccess;
    ok = ok && hipMalloc(&d_gp, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&d_aoff, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&d_bad, sizeof(int32_t)) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_acol, sizeof(int2) * ncol) == hipSuccess;
    std::vector<int2> acol(ncol);
    for (int c = 0; c < ncol; ++c) acol[c] = make_int2(aoff[c], gp[c]);
    int32_t bad = 0;
    hipError_t e = ok ? hipSuccess : hipErrorOutOfMemory;
    auto chk = [&](hipError_t r) {
        if (e == hipSuccess) e = r;
    };
    if (ok) {
        chk(hipMemcpyAsync(d_aux, aux.data(), sizeof(int2) * aux.size(), hipMemcpyHostToDevice, cx->stream));
        chk(hipMemcpyAsync(d_gp, gp.data(), sizeof(int32_t) * ncol, hipMemcpyHostToDevice, cx->stream));
        chk(hipMemcpyAsync(d_aoff, aoff.data(), sizeof(int32_t) * ncol, hipMemcpyHostToDevice, cx->stream));
        chk(hipMemcpyAsync(cx->d_acol, acol.data(), sizeof(int2) * ncol, hipMemcpyHostToDevice, cx->stream));
        chk(hipMemsetAsync(d_bad, 0, sizeof(int32_t), cx->stream));
        GenArgs<double> a{};
        a.D = Dims{nx, ny, nz};
        a.v = geo_view(cx);
        a.cbase = cx->d_cbase;
        a.naux = cx->naux;
        if (G + A > 0)
            hipLaunchKernelGGL(k_ptab_fill, dim3((unsigned)((G + A + 255) / 256)), dim3(256), 0, cx->stream, a,
                               d_aux, cx->d_ptab);
        if (Ge > 0)
            hipLaunchKernelGGL(k_sten_fill, dim3((Ge + 255) / 256), dim3(256), 0, cx->stream, a, d_gp, d_aoff,
                               cx->d_sten, cx->d_ftab, d_bad);
        if (G > 0)
            hipLaunchKernelGGL(k_upd_fill, dim3((G + 255) / 256), dim3(256), 0, cx->stream, a, cx->d_upd,
                               cx->d_utab, d_bad);
        chk(hipGetLastError());
        chk(hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, cx->stream));
        chk(hipStreamSynchronize(cx->stream));
    }
    for (void* q : {(void*)d_aux, (void*)d_gp, (void*)d_aoff, (void*)d_bad})
        if (q) (void)hipFree(q);
    if (!ok) {
        cx->err = "stencil table allocation failed";
        return EBS_E_OOM;
    }
    if (e != hipSuccess) {
        cx->err = std::string("stencil tables: ") + hipGetErrorString(e);
        return EBS_E_HIP;
    }
    if (bad != 0) {
        cx->err = "a face-range stencil reads a position outside the stored ranges";
        return EBS_E_UNSUPPORTED;
    }
    return EBS_OK;
}

template <typename T>
static ebs_status advance_t(ebs_ctx* cx, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uh,
                            double cdt, bool defer_join) {
    // The regular-region kernel and the general-range passes write disjoint
    // cells and read U_cur (never an output), so the former runs on the side
    // stream, forked from and joined back into the context stream.
    const bool fork = cx->overlap && cx->side && cx->ntiles > 0 && cx->G > 0;
    hipStream_t bs = cx->stream;
    if (fork) {
        EBS_HIP(cx, hipEventRecord(cx->ev_fork, cx->stream));
        EBS_HIP(cx, hipStreamWaitEvent(cx->side, cx->ev_fork, 0));
        bs = cx->side;
    }
    const void* const un[5] = {Un->rho, Un->rhotheta, Un->rhou, Un->rhov, Un->rhow};
    const void* const cu[5] = {Ucur->rho, Ucur->rhotheta, Ucur->rhou, Ucur->rhov, Ucur->rhow};
    void* const ou[5] = {Uh->rho, Uh->rhotheta, Uh->rhou, Uh->rhov, Uh->rhow};
    Dims D{cx->nx, cx->ny, cx->nz};
    {
        ebs_status st = launch_bulk(cx, Un, Ucur, Uh, cdt, bs);
        if (st != EBS_OK) return st;
        if (cx->diff_on || cx->visc_on) {  // adds to what the regular-region kernel wrote
            st = launch_regular_diffusion(cx, Ucur, Uh, cdt, bs);
            if (st != EBS_OK) return st;
        }
        if (fork) EBS_HIP(cx, hipEventRecord(cx->ev_join, bs));
    }
    if (cx->G > 0) {
        GenArgs<T> a;
        a.D = D;
        a.v = geo_view(cx);
        for (int f = 0; f < 5; ++f) {
            a.un[f] = (const T*)un[f];
            a.cur[f] = (const T*)cu[f];
            a.out[f] = (T*)ou[f];
        }
        a.uhat = cx->d_uhat;
        a.prim = cx->d_prim;
        a.sten = cx->d_sten;
        a.ptab = cx->d_ptab;
        a.ftab = cx->d_ftab;
        a.utab = cx->d_utab;
        a.naux = cx->naux;
        a.upd = cx->d_upd;
        a.fh = cx->d_fh;
        a.cbase = cx->d_cbase;
        a.cut_n = cx->d_cut_n;
        a.cut_w = cx->d_cut_w;
        a.bfc = cx->d_bfc;
        a.ncut = cx->ncut;
        a.cdt = cdt;
        for (int d = 0; d < 3; ++d) a.rdel[d] = 1.0 / cx->g.dx[d];
        a.eb_mode = cx->g.eb_flux;
        a.srcv = cx->src_on ? cx->d_srcv : nullptr;
        a.sref = cx->d_srcd;
        a.sP00 = cx->src.P00;
        a.sR = cx->src.R;
        a.sgam = cx->src.gamma;
        a.sg = cx->src.g;
        // work-list passes spread over the XCDs in contiguous chunks (xcd.h);
        // the test-mode update keeps the plain mapping
        const dim3 grid((cx->G + 255) / 256), blk(256);
        // the first two passes only read the input state; the update writes
        // the output (which may alias U^n, never U_cur)
        hipLaunchKernelGGL(k_gen_prims<T>, dim3(xcd_grid((cx->G + cx->naux + GEN_CO * 256 - 1) / (GEN_CO * 256))),
                           blk, 0, cx->stream, a);
        hipLaunchKernelGGL(k_gen_fhat<T>, dim3(xcd_grid((cx->Ge + 255) / 256)), blk, 0, cx->stream, a);
        if (cx->ncut > 0)
            hipLaunchKernelGGL(k_gen_cut<T>, dim3(xcd_grid((cx->ncut + 255) / 256)), blk, 0, cx->stream, a);
        if (a.eb_mode == 1)
            hipLaunchKernelGGL(k_gen_update_eb<T>, grid, blk, 0, cx->stream, a);
        else
            hipLaunchKernelGGL(k_gen_update<T>, dim3(xcd_grid((cx->G + 255) / 256)), blk, 0, cx->stream, a);
        EBS_HIP(cx, hipGetLastError());
        if (cx->diff_on) {  // adds to what the update wrote
            const ebs_status st = launch_diffusion_general(cx, Ucur, Uh, cdt);
            if (st != EBS_OK) return st;
        }
        if (cx->visc_on) {
            const ebs_status st = launch_viscous_general(cx, Ucur, Uh, cdt);
            if (st != EBS_OK) return st;
        }
    }
    cx->join_pending = fork;
    if (fork && !defer_join) return join_side(cx);
    return EBS_OK;
}

ebs_status join_side(ebs_ctx* cx) {
    if (!cx->join_pending) return EBS_OK;
    cx->join_pending = false;
    EBS_HIP(cx, hipStreamWaitEvent(cx->stream, cx->ev_join, 0));
    return EBS_OK;
}

ebs_status launch_advance(ebs_ctx* cx, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uhat,
                          double cdt, bool defer_join) {
    if (cx->g.precision == EBS_F32_BULK) return advance_t<float>(cx, Un, Ucur, Uhat, cdt, defer_join);
    return advance_t<double>(cx, Un, Ucur, Uhat, cdt, defer_join);
}

}  // namespace ebs
