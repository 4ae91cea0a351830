// Explicit stage update of the four instances (Eqs. update-cc / update-fc of
// Section 3.1 with the advective flux of Section 4.1; Algorithm 1 steps 1-3).
//
// The regular region (every cell at or above its column's general range) is
// updated by the kernel in bulk.hip; this file holds the passes over the
// general range of each column (the cut band and a margin), in double
// precision with the full rules: area / volume fractions, covered stencil
// ends (order reduction), interpolation to the cut-face centroid, walls.  They
// also keep a double-precision copy of the provisional state there for the
// redistribution.  The two parts run concurrently on two streams.
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

namespace ebs {
namespace {

// --------------------------------------------------------------- general
//
// The general range is processed in three passes over its cells, in double
// precision: the advected quantities of every cell (prims), the provisional
// fluxes on its three lower faces (fhat), and the update, which moves the
// provisional flux of every cut face to the face centroid (bilinear
// interpolation of neighbouring provisional fluxes), multiplies by the area
// fraction and takes the divergence over the six faces.
//
// A stencil position is resolved through its column's range info (loaded once
// per neighbouring column): general (an index into the range), below the range
// (no instance is fluid) or above it.  The range's top is chosen so that a
// position above it has only regular CVs within three cells in x and y and
// below it; its advected quantities and fluxes therefore follow the plain
// formulas (every neighbour inside the domain is fluid, faces are full).  Every
// neighbour a cut-face interpolation reads lies within one cell of a CV that is
// not regular, hence inside or below its column's range.
template <typename T>
struct GenArgs {
    Dims D;
    GeoView v;
    const T* un[5];
    const T* cur[5];
    T* out[5];
    double* uhat;  // [5][G]
    double* prim;  // [G][4] theta, u, v, w
    double* fh;    // [5][3][Ge] provisional flux on the lower faces
    const int32_t* cbase;  // [G] first cut-face record of each general cell
    const struct CutRec* crec;
    double* bfc;           // [2][ncut] area fraction x interpolated flux per record
    int32_t ncut;
    double cdt;
    double rdel[3];
    int eb_mode;
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
        return st(a.cur, F, p.i, p.j, p.k) / (s / cnt);
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
        const double m = s == 0 ? mom<D>(P) : 0.5 * (mom<D>(ls) + mom<D>(P));
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
        const int s1 = g1 > 0.0 ? 1 : (g1 < 0.0 ? -1 : 0);
        const int s2 = g2 > 0.0 ? 1 : (g2 < 0.0 ? -1 : 0);
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
        const double w1 = fabs(g1), w2 = fabs(g2);
        r.c[0] = (1.0 - w1) * (1.0 - w2);
        bool ok = true;
        if (u1) { r.n[0] = N1.ge; r.c[1] = w1 * (1.0 - w2); ok &= N1.ge >= 0; }
        if (u2) { r.n[1] = N2.ge; r.c[2] = (1.0 - w1) * w2; ok &= N2.ge >= 0; }
        if (u12) { r.n[2] = N12.ge; r.c[3] = w1 * w2; ok &= N12.ge >= 0; }
        return ok;
    }
    template <int F, int D>
    __device__ __forceinline__ double div_pre(const Pt& P, const Pt& U, int g, double Fp, double Fu) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        const double rd = a.rdel[D];
        double br = (bface_pre<F, D>(U, Fu) - bface_pre<F, D>(P, Fp)) * rd;
        if (a.eb_mode == 1) {
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
    template <int F>
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
            double br = div_pre<F, 0>(P, Ux, g, Fp0, Fu0);
            br += div_pre<F, 1>(P, Uy, g, Fp1, Fu1);
            br += div_pre<F, 2>(P, Uz, g, Fp2, Fu2);
            val = unv - a.cdt * br / al;
        }
        a.uhat[(size_t)F * a.v.G + g] = val;
        put_field<T>(a.D, a.out, F, P.i, P.j, P.k, (T)val);
    }
    // advected quantities of a position loaded unconditionally (valid index;
    // used only where the position is general)
    struct PV {
        double q[4];
    };
    __device__ __forceinline__ PV loadpv(const Pt& p) const {
        const double* b = a.prim + 4 * (size_t)max(p.g, 0);
        PV v;
        v.q[0] = b[0];
        v.q[1] = b[1];
        v.q[2] = b[2];
        v.q[3] = b[3];
        return v;
    }
    template <int F>
    __device__ __forceinline__ double phiv(const Pt& p, const PV& v) const {
        if (!((p.fl >> finst(F)) & 1)) return 0.0;
        if (p.g >= 0) return v.q[F - 1];
        return phi_state<F>(p, true);
    }
    // momentum component D, loaded unconditionally from a clamped plane
    template <int D>
    __device__ __forceinline__ double momv(const Pt& p) const {
        const double v = st(a.cur, 2 + D, p.i, p.j, min(max(p.k, 0), a.D.nz - 1));
        return ((p.fl >> (D + 1)) & 1) ? v : 0.0;
    }
    template <int F, int D>
    __device__ __forceinline__ double fhatv(const Pt& LL, const Pt& L, const Pt& P, const Pt& RR,
                                            const PV& vLL, const PV& vL, const PV& vP, const PV& vRR,
                                            double m0, double mls) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        if (D == 2) {
            if (s != 3 && (P.k == 0 || P.k == a.D.nz)) return 0.0;
            if (s == 3 && (P.k == 1 || P.k == a.D.nz)) return 0.0;
        }
        const double m = s == 0 ? m0 : 0.5 * (mls + m0);
        if (F == 0) return m;
        return m * upw<double>(m, phiv<F>(LL, vLL), phiv<F>(L, vL), phiv<F>(P, vP), phiv<F>(RR, vRR),
                               (LL.fl >> s) & 1, (RR.fl >> s) & 1);
    }
    template <int D>
    __device__ __forceinline__ void fhat_dir(const Pt& P, const Pt& Lx, const Pt& Ly, const Pt& Lz,
                                             const int4& ci, int g, const PV& vP) const {
        Pt LL, RR;
        const Pt& L = D == 0 ? Lx : D == 1 ? Ly : Lz;
        if (D == 0) {
            LL = at(wx(P.i - 2), P.j, P.k);
            RR = at(wx(P.i + 1), P.j, P.k);
        } else if (D == 1) {
            LL = at(P.i, wy(P.j - 2), P.k);
            RR = at(P.i, wy(P.j + 1), P.k);
        } else {
            LL = at(P.i, P.j, P.k - 2, ci);
            RR = at(P.i, P.j, P.k + 1, ci);
        }
        const size_t G = a.v.Ge;
        const uint32_t ff = P.ff;  // lower faces with fluid (P.k < nz here)
        const PV vLL = loadpv(LL), vL = loadpv(L), vRR = loadpv(RR);
        // mass fluxes: component D at P and below P along x, y, z
        const double m0 = momv<D>(P), mx = momv<D>(Lx), my = momv<D>(Ly), mz = momv<D>(Lz);
        a.fh[(0 * 3 + D) * G + g] = (ff & ff_pos(0, D)) ? fhatv<0, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, m0) : 0.0;
        a.fh[(1 * 3 + D) * G + g] = (ff & ff_pos(0, D)) ? fhatv<1, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, m0) : 0.0;
        a.fh[(2 * 3 + D) * G + g] = (ff & ff_pos(1, D)) ? fhatv<2, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, mx) : 0.0;
        a.fh[(3 * 3 + D) * G + g] = (ff & ff_pos(2, D)) ? fhatv<3, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, my) : 0.0;
        a.fh[(4 * 3 + D) * G + g] = (ff & ff_pos(3, D)) ? fhatv<4, D>(LL, L, P, RR, vLL, vL, vP, vRR, m0, mz) : 0.0;
    }
};

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

template <typename T>
__global__ void __launch_bounds__(256) k_gen_prims(GenArgs<T> a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.v.G) return;
    const Gen<T> G(a);
    int i, j, k;
    int4 ci;
    gen_cell(a.v, g, i, j, k, ci);
    const Pt P = G.at(i, j, k, ci);
    const bool lx = G.at(G.wx(i - 1), j, k).fl & 1;
    const bool ly = G.at(i, G.wy(j - 1), k).fl & 1;
    const bool lz = G.at(i, j, k - 1, ci).fl & 1;
    double* o = a.prim + 4 * (size_t)g;
    o[0] = (P.fl & 1) ? G.template phi_state<1>(P, false) : 0.0;
    o[1] = (P.fl & 2) ? G.template phi_state<2>(P, lx) : 0.0;
    o[2] = (P.fl & 4) ? G.template phi_state<3>(P, ly) : 0.0;
    o[3] = (P.fl & 8) ? G.template phi_state<4>(P, lz) : 0.0;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gen_fhat(GenArgs<T> a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;  // extended face range
    if (g >= a.v.Ge) return;
    const Gen<T> G(a);
    int i, j, k;
    int4 ci;
    face_cell(a.v, g, i, j, k, ci);
    Pt P = G.at(i, j, k, ci);
    P.ff = G.fflags(P);
    // positions below P along x, y, z (the staggering neighbours of instances 1-3)
    const Pt Lx = G.at(G.wx(i - 1), j, k), Ly = G.at(i, G.wy(j - 1), k), Lz = G.at(i, j, k - 1, ci);
    const auto vP = G.loadpv(P);
    G.template fhat_dir<0>(P, Lx, Ly, Lz, ci, g, vP);
    G.template fhat_dir<1>(P, Lx, Ly, Lz, ci, g, vP);
    G.template fhat_dir<2>(P, Lx, Ly, Lz, ci, g, vP);
}

template <typename T>
__global__ void __launch_bounds__(256) k_gen_update(GenArgs<T> a) {
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
    G.template update<0>(P, Ux, Uy, Uz, g);
    G.template update<1>(P, Ux, Uy, Uz, g);
    G.template update<2>(P, Ux, Uy, Uz, g);
    G.template update<3>(P, Ux, Uy, Uz, g);
    G.template update<4>(P, Ux, Uy, Uz, g);
}

// Area fraction x flux moved to the centroid on every partial face, for the
// field(s) of the face's instance (slot 1: rho theta of the cell-centred CVs).
template <typename T>
__global__ void __launch_bounds__(256) k_gen_cut(GenArgs<T> a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.ncut) return;
    const CutRec c = a.crec[r];
    const int s = c.sd / 3, d = c.sd - 3 * s;
    const int n0 = max(c.n[0], 0), n1 = max(c.n[1], 0), n2 = max(c.n[2], 0);
    for (int q = 0; q < (s == 0 ? 2 : 1); ++q) {
        const int f = s == 0 ? q : s + 1;
        const double* fhd = a.fh + ((size_t)f * 3 + d) * a.v.Ge;
        const double F0 = fhd[c.own], F1 = fhd[n0], F2 = fhd[n1], F3 = fhd[n2];
        double Fv = c.c[0] * F0;
        if (c.n[0] >= 0) Fv += c.c[1] * F1;
        if (c.n[1] >= 0) Fv += c.c[2] * F2;
        if (c.n[2] >= 0) Fv += c.c[3] * F3;
        a.bfc[(size_t)q * a.ncut + r] = c.b * Fv;
    }
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

}  // namespace

// ------------------------------------------------------------- host side
ebs_status build_cut_faces(ebs_ctx* cx) {
    const int32_t G = cx->G;
    if (cx->d_cbase) (void)hipFree(cx->d_cbase);
    if (cx->d_crec) (void)hipFree(cx->d_crec);
    cx->d_cbase = nullptr;
    cx->d_crec = nullptr;
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
    cx->ncut = (int32_t)tot;
    if (cx->d_bfc) (void)hipFree(cx->d_bfc);
    cx->d_bfc = nullptr;
    if (hipMalloc(&cx->d_crec, sizeof(CutRec) * std::max<int64_t>(tot, 1)) != hipSuccess ||
        hipMalloc(&cx->d_bfc, sizeof(double) * 2 * std::max<int64_t>(tot, 1)) != hipSuccess) {
        (void)hipFree(d_bad);
        cx->err = "cut-face table allocation failed";
        return EBS_E_OOM;
    }
    EBS_HIP(cx, hipMemcpyAsync(cx->d_cbase, cnt.data(), sizeof(int32_t) * G, hipMemcpyHostToDevice, cx->stream));
    EBS_HIP(cx, hipMemsetAsync(d_bad, 0, sizeof(int32_t), cx->stream));
    GenArgs<double> a{};
    a.D = Dims{cx->nx, cx->ny, cx->nz};
    a.v = v;
    a.cbase = cx->d_cbase;
    hipLaunchKernelGGL(k_cut_fill, dim3((G + 127) / 128), dim3(128), 0, cx->stream, a, (CutRec*)cx->d_crec,
                       d_bad);
    EBS_HIP(cx, hipGetLastError());
    int32_t bad = 0;
    EBS_HIP(cx, hipMemcpyAsync(&bad, d_bad, sizeof(int32_t), hipMemcpyDeviceToHost, cx->stream));
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    (void)hipFree(d_bad);
    if (bad != 0) {
        cx->err = "a cut-face interpolation neighbour lies outside the stored face range";
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
        const ebs_status st = launch_bulk(cx, Un, Ucur, Uh, cdt, bs);
        if (st != EBS_OK) return st;
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
        a.fh = cx->d_fh;
        a.cbase = cx->d_cbase;
        a.crec = (const CutRec*)cx->d_crec;
        a.bfc = cx->d_bfc;
        a.ncut = cx->ncut;
        a.cdt = cdt;
        for (int d = 0; d < 3; ++d) a.rdel[d] = 1.0 / cx->g.dx[d];
        a.eb_mode = cx->g.eb_flux;
        const dim3 grid((cx->G + 255) / 256), gride((cx->Ge + 255) / 256), blk(256);
        // the first two passes only read the input state; the update writes
        // the output (which may alias U^n, never U_cur)
        hipLaunchKernelGGL(k_gen_prims<T>, grid, blk, 0, cx->stream, a);
        hipLaunchKernelGGL(k_gen_fhat<T>, gride, blk, 0, cx->stream, a);
        if (cx->ncut > 0)
            hipLaunchKernelGGL(k_gen_cut<T>, dim3((cx->ncut + 255) / 256), blk, 0, cx->stream, a);
        hipLaunchKernelGGL(k_gen_update<T>, grid, blk, 0, cx->stream, a);
        EBS_HIP(cx, hipGetLastError());
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
