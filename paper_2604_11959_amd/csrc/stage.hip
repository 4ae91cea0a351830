// Explicit stage update of the four instances (Eqs. update-cc / update-fc of
// Section 3.1 with the advective flux of Section 4.1; Algorithm 1 steps 1-3).
//
// Two kernels share the work:
//   * k_bulk streams the regular region (every cell position at or above the
//     column's general range, and the covered cells below it).  Every CV and
//     every stencil member there is a full cell, so the update needs no
//     geometry: face fractions are one, no flux is moved to a centroid, and
//     the only special cases are the top wall.  It runs over a tile list
//     derived from the box list, in the state precision.
//   * k_general handles the general range of each column (the cut band and a
//     margin) in double precision with the full rules: area / volume
//     fractions, covered stencil ends (order reduction), interpolation to the
//     cut-face centroid, walls.  It also keeps a double-precision copy of the
//     provisional state there for the redistribution.
//
// Readings where the paper is silent: the mass flux advecting momentum on a
// staggered face is the mean of the two stored face momenta next to it; face
// velocities divide by the mean density of the fluid cells on either side;
// the momentum flux of the z-face instance through the mid planes of the
// bottom and top cell layers is zero; the EB flux is zero (test mode: minus
// the area vector dotted with the CV's mean provisional flux).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ebs_internal.h"

namespace ebs {
namespace {

struct Dims {
    int nx, ny, nz;
};

__device__ inline size_t ic(const Dims& D, int i, int j, int k) { return ((size_t)k * D.ny + j) * D.nx + i; }
__device__ inline size_t iu(const Dims& D, int i, int j, int k) { return ((size_t)k * D.ny + j) * (D.nx + 1) + i; }
__device__ inline size_t iv(const Dims& D, int i, int j, int k) { return ((size_t)k * (D.ny + 1) + j) * D.nx + i; }

// index of field f at CV position (i, j, k) (i, j already wrapped)
__device__ inline size_t fidx(const Dims& D, int f, int i, int j, int k) {
    if (f == 2) return iu(D, i, j, k);
    if (f == 3) return iv(D, i, j, k);
    return ic(D, i, j, k);
}

// third-order upwind face value (fourth-order centred plus hyperviscosity),
// second-order centred when the upwind end of the stencil is unavailable
template <typename C>
__device__ inline C upw(C m, C pLL, C pL, C pR, C pRR, bool okLL, bool okRR) {
    const C sixth = C(1) / C(6);
    if (m >= C(0)) {
        if (!okLL) return C(0.5) * (pL + pR);
        return (C(5) * pL + C(2) * pR - pLL) * sixth;
    }
    if (!okRR) return C(0.5) * (pL + pR);
    return (C(2) * pL + C(5) * pR - pRR) * sixth;
}

// write helper covering the periodic repeats and the top wall plane
template <typename T>
__device__ inline void put_field(const Dims& D, T* const* out, int f, int i, int j, int k, T v) {
    out[f][fidx(D, f, i, j, k)] = v;
    if (f == 2 && i == 0) out[2][iu(D, D.nx, j, k)] = v;
    if (f == 3 && j == 0) out[3][iv(D, i, D.ny, k)] = v;
    if (f == 4 && k == D.nz - 1) out[4][ic(D, i, j, D.nz)] = T(0);
}

// ------------------------------------------------------------------ bulk
template <typename T>
struct BulkArgs {
    Dims D;
    const T* un[5];
    const T* cur[5];
    T* out[5];
    T cdt;
    T rdx, rdy, rdz;
    const int32_t* g0;
    const int32_t* g1;
    const ebs_tile* tiles;
    int32_t ntiles;
};

template <typename T>
struct BulkCell {
    const BulkArgs<T>& a;
    int i, j, k;
    __device__ BulkCell(const BulkArgs<T>& a_, int i_, int j_, int k_) : a(a_), i(i_), j(j_), k(k_) {}
    __device__ int X(int o) const { return wrapi(i + o, a.D.nx); }
    __device__ int Y(int o) const { return wrapi(j + o, a.D.ny); }
    __device__ T R(int ii, int jj, int kk) const { return a.cur[0][ic(a.D, ii, jj, kk)]; }
    __device__ T RU(int ii, int jj, int kk) const { return a.cur[2][iu(a.D, ii, jj, kk)]; }
    __device__ T RV(int ii, int jj, int kk) const { return a.cur[3][iv(a.D, ii, jj, kk)]; }
    __device__ T RW(int ii, int jj, int kk) const { return a.cur[4][ic(a.D, ii, jj, kk)]; }
    __device__ T TH(int ii, int jj, int kk) const {
        if (kk < 0 || kk >= a.D.nz) return T(0);
        return a.cur[1][ic(a.D, ii, jj, kk)] / R(ii, jj, kk);
    }
    __device__ T UU(int ii, int jj, int kk) const {
        if (kk < 0 || kk >= a.D.nz) return T(0);
        return RU(ii, jj, kk) / (T(0.5) * (R(wrapi(ii - 1, a.D.nx), jj, kk) + R(ii, jj, kk)));
    }
    __device__ T VV(int ii, int jj, int kk) const {
        if (kk < 0 || kk >= a.D.nz) return T(0);
        return RV(ii, jj, kk) / (T(0.5) * (R(ii, wrapi(jj - 1, a.D.ny), kk) + R(ii, jj, kk)));
    }
    __device__ T WW(int ii, int jj, int kk) const {
        if (kk < 1 || kk > a.D.nz - 1) return T(0);
        return RW(ii, jj, kk) / (T(0.5) * (R(ii, jj, kk - 1) + R(ii, jj, kk)));
    }
};

template <typename T>
__device__ void bulk_update(const BulkArgs<T>& a, int i, int j, int k) {
    const BulkCell<T> c(a, i, j, k);
    const int nz = a.D.nz;
    const int xm2 = c.X(-2), xm1 = c.X(-1), xp1 = c.X(1), xp2 = c.X(2);
    const int ym2 = c.Y(-2), ym1 = c.Y(-1), yp1 = c.Y(1), yp2 = c.Y(2);
    const bool top = (k + 1 == nz);
    // ---- cell-centred instance: rho and rho theta
    {
        T m, tf;
        T dr = 0, dt = 0;
        // x
        m = c.RU(i, j, k);
        tf = upw<T>(m, c.TH(xm2, j, k), c.TH(xm1, j, k), c.TH(i, j, k), c.TH(xp1, j, k), true, true);
        dr -= m * a.rdx; dt -= m * tf * a.rdx;
        m = c.RU(xp1, j, k);
        tf = upw<T>(m, c.TH(xm1, j, k), c.TH(i, j, k), c.TH(xp1, j, k), c.TH(xp2, j, k), true, true);
        dr += m * a.rdx; dt += m * tf * a.rdx;
        // y
        m = c.RV(i, j, k);
        tf = upw<T>(m, c.TH(i, ym2, k), c.TH(i, ym1, k), c.TH(i, j, k), c.TH(i, yp1, k), true, true);
        dr -= m * a.rdy; dt -= m * tf * a.rdy;
        m = c.RV(i, yp1, k);
        tf = upw<T>(m, c.TH(i, ym1, k), c.TH(i, j, k), c.TH(i, yp1, k), c.TH(i, yp2, k), true, true);
        dr += m * a.rdy; dt += m * tf * a.rdy;
        // z (the bulk range starts above the bottom margin)
        m = c.RW(i, j, k);
        tf = upw<T>(m, c.TH(i, j, k - 2), c.TH(i, j, k - 1), c.TH(i, j, k), c.TH(i, j, k + 1), true,
                    k + 1 <= nz - 1);
        dr -= m * a.rdz; dt -= m * tf * a.rdz;
        if (!top) {
            m = c.RW(i, j, k + 1);
            tf = upw<T>(m, c.TH(i, j, k - 1), c.TH(i, j, k), c.TH(i, j, k + 1), c.TH(i, j, k + 2), true,
                        k + 2 <= nz - 1);
            dr += m * a.rdz; dt += m * tf * a.rdz;
        }
        const size_t id = ic(a.D, i, j, k);
        put_field<T>(a.D, a.out, 0, i, j, k, a.un[0][id] - a.cdt * dr);
        put_field<T>(a.D, a.out, 1, i, j, k, a.un[1][id] - a.cdt * dt);
    }
    // ---- x-face instance (rho u at face i)
    {
        T m, f, du = 0;
        m = T(0.5) * (c.RU(xm1, j, k) + c.RU(i, j, k));
        f = upw<T>(m, c.UU(xm2, j, k), c.UU(xm1, j, k), c.UU(i, j, k), c.UU(xp1, j, k), true, true);
        du -= m * f * a.rdx;
        m = T(0.5) * (c.RU(i, j, k) + c.RU(xp1, j, k));
        f = upw<T>(m, c.UU(xm1, j, k), c.UU(i, j, k), c.UU(xp1, j, k), c.UU(xp2, j, k), true, true);
        du += m * f * a.rdx;
        m = T(0.5) * (c.RV(xm1, j, k) + c.RV(i, j, k));
        f = upw<T>(m, c.UU(i, ym2, k), c.UU(i, ym1, k), c.UU(i, j, k), c.UU(i, yp1, k), true, true);
        du -= m * f * a.rdy;
        m = T(0.5) * (c.RV(xm1, yp1, k) + c.RV(i, yp1, k));
        f = upw<T>(m, c.UU(i, ym1, k), c.UU(i, j, k), c.UU(i, yp1, k), c.UU(i, yp2, k), true, true);
        du += m * f * a.rdy;
        m = T(0.5) * (c.RW(xm1, j, k) + c.RW(i, j, k));
        f = upw<T>(m, c.UU(i, j, k - 2), c.UU(i, j, k - 1), c.UU(i, j, k), c.UU(i, j, k + 1), true,
                   k + 1 <= nz - 1);
        du -= m * f * a.rdz;
        if (!top) {
            m = T(0.5) * (c.RW(xm1, j, k + 1) + c.RW(i, j, k + 1));
            f = upw<T>(m, c.UU(i, j, k - 1), c.UU(i, j, k), c.UU(i, j, k + 1), c.UU(i, j, k + 2), true,
                       k + 2 <= nz - 1);
            du += m * f * a.rdz;
        }
        put_field<T>(a.D, a.out, 2, i, j, k, a.un[2][iu(a.D, i, j, k)] - a.cdt * du);
    }
    // ---- y-face instance (rho v at face j)
    {
        T m, f, dv = 0;
        m = T(0.5) * (c.RU(i, ym1, k) + c.RU(i, j, k));
        f = upw<T>(m, c.VV(xm2, j, k), c.VV(xm1, j, k), c.VV(i, j, k), c.VV(xp1, j, k), true, true);
        dv -= m * f * a.rdx;
        m = T(0.5) * (c.RU(xp1, ym1, k) + c.RU(xp1, j, k));
        f = upw<T>(m, c.VV(xm1, j, k), c.VV(i, j, k), c.VV(xp1, j, k), c.VV(xp2, j, k), true, true);
        dv += m * f * a.rdx;
        m = T(0.5) * (c.RV(i, ym1, k) + c.RV(i, j, k));
        f = upw<T>(m, c.VV(i, ym2, k), c.VV(i, ym1, k), c.VV(i, j, k), c.VV(i, yp1, k), true, true);
        dv -= m * f * a.rdy;
        m = T(0.5) * (c.RV(i, j, k) + c.RV(i, yp1, k));
        f = upw<T>(m, c.VV(i, ym1, k), c.VV(i, j, k), c.VV(i, yp1, k), c.VV(i, yp2, k), true, true);
        dv += m * f * a.rdy;
        m = T(0.5) * (c.RW(i, ym1, k) + c.RW(i, j, k));
        f = upw<T>(m, c.VV(i, j, k - 2), c.VV(i, j, k - 1), c.VV(i, j, k), c.VV(i, j, k + 1), true,
                   k + 1 <= nz - 1);
        dv -= m * f * a.rdz;
        if (!top) {
            m = T(0.5) * (c.RW(i, ym1, k + 1) + c.RW(i, j, k + 1));
            f = upw<T>(m, c.VV(i, j, k - 1), c.VV(i, j, k), c.VV(i, j, k + 1), c.VV(i, j, k + 2), true,
                       k + 2 <= nz - 1);
            dv += m * f * a.rdz;
        }
        put_field<T>(a.D, a.out, 3, i, j, k, a.un[3][iv(a.D, i, j, k)] - a.cdt * dv);
    }
    // ---- z-face instance (rho w at face k; k >= 1 in the bulk range)
    {
        T m, f, dw = 0;
        m = T(0.5) * (c.RU(i, j, k - 1) + c.RU(i, j, k));
        f = upw<T>(m, c.WW(xm2, j, k), c.WW(xm1, j, k), c.WW(i, j, k), c.WW(xp1, j, k), true, true);
        dw -= m * f * a.rdx;
        m = T(0.5) * (c.RU(xp1, j, k - 1) + c.RU(xp1, j, k));
        f = upw<T>(m, c.WW(xm1, j, k), c.WW(i, j, k), c.WW(xp1, j, k), c.WW(xp2, j, k), true, true);
        dw += m * f * a.rdx;
        m = T(0.5) * (c.RV(i, j, k - 1) + c.RV(i, j, k));
        f = upw<T>(m, c.WW(i, ym2, k), c.WW(i, ym1, k), c.WW(i, j, k), c.WW(i, yp1, k), true, true);
        dw -= m * f * a.rdy;
        m = T(0.5) * (c.RV(i, yp1, k - 1) + c.RV(i, yp1, k));
        f = upw<T>(m, c.WW(i, ym1, k), c.WW(i, j, k), c.WW(i, yp1, k), c.WW(i, yp2, k), true, true);
        dw += m * f * a.rdy;
        if (k != 1) {
            m = T(0.5) * (c.RW(i, j, k - 1) + c.RW(i, j, k));
            f = upw<T>(m, c.WW(i, j, k - 2), c.WW(i, j, k - 1), c.WW(i, j, k), c.WW(i, j, k + 1),
                       k - 2 >= 1, k + 1 <= nz - 1);
            dw -= m * f * a.rdz;
        }
        if (k != nz - 1) {
            m = T(0.5) * (c.RW(i, j, k) + c.RW(i, j, k + 1));
            f = upw<T>(m, c.WW(i, j, k - 1), c.WW(i, j, k), c.WW(i, j, k + 1), c.WW(i, j, k + 2),
                       k - 1 >= 1, k + 2 <= nz - 1);
            dw += m * f * a.rdz;
        }
        put_field<T>(a.D, a.out, 4, i, j, k, a.un[4][ic(a.D, i, j, k)] - a.cdt * dw);
    }
}

template <typename T>
__global__ void __launch_bounds__(512) k_bulk(BulkArgs<T> a) {
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const ebs_tile tl = a.tiles[t];
        const int i = tl.x0 + (int)threadIdx.x;
        const int j = tl.y0 + (int)threadIdx.y;
        if ((int)threadIdx.x >= tl.ex || (int)threadIdx.y >= tl.ey) continue;
        const int c = j * a.D.nx + i;
        const int gb = a.g0[c], ge = a.g1[c];
        for (int k = tl.z0; k < tl.z0 + tl.ez; ++k) {
            if (k >= ge) {
                bulk_update<T>(a, i, j, k);
            } else if (k < gb) {
                for (int f = 0; f < 5; ++f) put_field<T>(a.D, a.out, f, i, j, k, T(0));
            }
        }
    }
}

// --------------------------------------------------------------- general
template <typename T>
struct GenArgs {
    Dims D;
    GeoView v;
    const T* un[5];
    const T* cur[5];
    T* out[5];
    double* uhat;  // [5][G]
    double cdt;
    double del[3];
    int eb_mode;
};

template <typename T>
struct Gen {
    const GenArgs<T>& a;
    __device__ explicit Gen(const GenArgs<T>& a_) : a(a_) {}

    // 0: not fluid, 1: fluid; alpha in *al
    __device__ bool fluid(int inst, int i, int j, int k, double* al = nullptr) const {
        if (!cv_plane(a.v, inst, k)) return false;
        i = wrapi(i, a.D.nx);
        j = wrapi(j, a.D.ny);
        const int g = gidx(a.v, i, j, k);
        if (g == -2) return false;
        if (g == -1) { if (al) *al = 1.0; return true; }
        if (a.v.type[(size_t)inst * a.v.G + g] == 0) return false;
        if (al) *al = gq(a.v, inst, GQ_ALPHA, g);
        return true;
    }
    // lower-face fraction of CV (i,j,k) in direction d; plane nz is the top face
    __device__ double beta(int inst, int d, int i, int j, int k) const {
        if (k == a.D.nz) return d == 2 ? 1.0 : 0.0;
        if (!cv_plane(a.v, inst, k)) return 0.0;
        i = wrapi(i, a.D.nx);
        j = wrapi(j, a.D.ny);
        const int g = gidx(a.v, i, j, k);
        if (g == -2) return 0.0;
        if (g == -1) return 1.0;
        return gq(a.v, inst, GQ_BX + d, g);
    }
    __device__ void gam(int inst, int d, int i, int j, int k, double& g1, double& g2) const {
        g1 = g2 = 0.0;
        if (k >= a.D.nz || !cv_plane(a.v, inst, k)) return;
        i = wrapi(i, a.D.nx);
        j = wrapi(j, a.D.ny);
        const int g = gidx(a.v, i, j, k);
        if (g < 0) return;
        g1 = gq(a.v, inst, GQ_FX1 + 2 * d, g);
        g2 = gq(a.v, inst, GQ_FX1 + 2 * d + 1, g);
    }
    // state value, zero where the CV is not fluid
    __device__ double sv(const T* const* U, int f, int i, int j, int k) const {
        const int inst = f < 2 ? 0 : f - 1;
        if (!fluid(inst, i, j, k)) return 0.0;
        return (double)U[f][fidx(a.D, f, wrapi(i, a.D.nx), wrapi(j, a.D.ny), k)];
    }
    // advected quantity of field f (1: theta, 2..4: velocity) at a CV of its instance
    __device__ double phi(int f, int i, int j, int k) const {
        const int inst = f < 2 ? 0 : f - 1;
        if (!fluid(inst, i, j, k)) return 0.0;
        const int ii = wrapi(i, a.D.nx), jj = wrapi(j, a.D.ny);
        if (f == 1) return (double)a.cur[1][ic(a.D, ii, jj, k)] / (double)a.cur[0][ic(a.D, ii, jj, k)];
        int i0 = ii, j0 = jj, k0 = k;
        if (f == 2) i0 = wrapi(ii - 1, a.D.nx);
        if (f == 3) j0 = wrapi(jj - 1, a.D.ny);
        if (f == 4) k0 = k - 1;
        double s = 0.0;
        int cnt = 0;
        if (fluid(0, i0, j0, k0)) { s += (double)a.cur[0][ic(a.D, i0, j0, k0)]; ++cnt; }
        if (fluid(0, ii, jj, k)) { s += (double)a.cur[0][ic(a.D, ii, jj, k)]; ++cnt; }
        if (cnt == 0) return 0.0;
        return (double)a.cur[f][fidx(a.D, f, ii, jj, k)] / (s / cnt);
    }
    __device__ double mass(int inst, int d, int i, int j, int k) const {
        const int mf = 2 + d;
        if (inst == 0) return sv(a.cur, mf, i, j, k);
        int i0 = i, j0 = j, k0 = k;
        if (inst == 1) i0 = i - 1;
        if (inst == 2) j0 = j - 1;
        if (inst == 3) k0 = k - 1;
        return 0.5 * (sv(a.cur, mf, i0, j0, k0) + sv(a.cur, mf, i, j, k));
    }
    // provisional flux on the lower d-face of CV (i,j,k)
    __device__ double fhat(int f, int d, int i, int j, int k) const {
        const int inst = f < 2 ? 0 : f - 1;
        if (d == 2) {
            if (inst != 3 && (k == 0 || k == a.D.nz)) return 0.0;
            if (inst == 3 && (k == 1 || k == a.D.nz)) return 0.0;
        }
        const double m = mass(inst, d, i, j, k);
        if (f == 0) return m;
        const int o0 = d == 0, o1 = d == 1, o2 = d == 2;
        const double pLL = phi(f, i - 2 * o0, j - 2 * o1, k - 2 * o2);
        const double pL = phi(f, i - o0, j - o1, k - o2);
        const double pR = phi(f, i, j, k);
        const double pRR = phi(f, i + o0, j + o1, k + o2);
        const bool okLL = fluid(inst, i - 2 * o0, j - 2 * o1, k - 2 * o2);
        const bool okRR = fluid(inst, i + o0, j + o1, k + o2);
        return m * upw<double>(m, pLL, pL, pR, pRR, okLL, okRR);
    }
    // flux used in the divergence on the lower d-face, moved to the cut-face centroid
    __device__ double face(int f, int d, int i, int j, int k) const {
        const int inst = f < 2 ? 0 : f - 1;
        const double b = beta(inst, d, i, j, k);
        if (!(b > 0.0)) return 0.0;
        const double F0 = fhat(f, d, i, j, k);
        if (!(b < 1.0)) return F0;
        double g1, g2;
        gam(inst, d, i, j, k, g1, g2);
        const int s1 = g1 > 0.0 ? 1 : (g1 < 0.0 ? -1 : 0);
        const int s2 = g2 > 0.0 ? 1 : (g2 < 0.0 ? -1 : 0);
        if (s1 == 0 && s2 == 0) return F0;
        int e1[3] = {0, 0, 0}, e2[3] = {0, 0, 0};
        const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
        e1[t1] = s1;
        e2[t2] = s2;
        const int nb[3][3] = {{i + e1[0], j + e1[1], k + e1[2]},
                              {i + e2[0], j + e2[1], k + e2[2]},
                              {i + e1[0] + e2[0], j + e1[1] + e2[1], k + e1[2] + e2[2]}};
        const bool use[3] = {s1 != 0, s2 != 0, s1 != 0 && s2 != 0};
        for (int q = 0; q < 3; ++q) {
            if (!use[q]) continue;
            if (nb[q][2] != k && !cv_plane(a.v, inst, nb[q][2])) return F0;
            if (!(beta(inst, d, nb[q][0], nb[q][1], nb[q][2]) > 0.0)) return F0;
        }
        const double w1 = fabs(g1), w2 = fabs(g2);
        double F = (1.0 - w1) * (1.0 - w2) * F0;
        if (use[0]) F += w1 * (1.0 - w2) * fhat(f, d, nb[0][0], nb[0][1], nb[0][2]);
        if (use[1]) F += (1.0 - w1) * w2 * fhat(f, d, nb[1][0], nb[1][1], nb[1][2]);
        if (use[2]) F += w1 * w2 * fhat(f, d, nb[2][0], nb[2][1], nb[2][2]);
        return F;
    }
    // provisional value of field f at CV (i,j,k) (fluid, alpha al)
    __device__ double update(int f, int i, int j, int k, double al, int g) const {
        const int inst = f < 2 ? 0 : f - 1;
        double br = 0.0;
        for (int d = 0; d < 3; ++d) {
            const int ip = i + (d == 0), jp = j + (d == 1), kp = k + (d == 2);
            const double blo = beta(inst, d, i, j, k);
            const double bhi = beta(inst, d, ip, jp, kp);
            const double Flo = face(f, d, i, j, k);
            const double Fhi = face(f, d, ip, jp, kp);
            br += (bhi * Fhi - blo * Flo) / a.del[d];
            if (a.eb_mode == 1 && g >= 0) {
                double s = 0.0;
                int cnt = 0;
                if (blo > 0.0) { s += fhat(f, d, i, j, k); ++cnt; }
                if (bhi > 0.0) { s += fhat(f, d, ip, jp, kp); ++cnt; }
                const double fb = cnt ? s / cnt : 0.0;
                br -= gq(a.v, inst, GQ_AX + d, g) * fb / a.del[d];
            }
        }
        return sv(a.un, f, i, j, k) - a.cdt * br / al;
    }
};

template <typename T>
__global__ void __launch_bounds__(256) k_general(GenArgs<T> a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= a.v.G) return;
    const Gen<T> G(a);
    const int c = a.v.gcol[g];
    const int i = c % a.D.nx, j = c / a.D.nx;
    const int k = a.v.g0[c] + (g - a.v.goff[c]);
    for (int f = 0; f < 5; ++f) {
        const int inst = f < 2 ? 0 : f - 1;
        double al = 0.0;
        double val = 0.0;
        if (G.fluid(inst, i, j, k, &al)) val = G.update(f, i, j, k, al, g);
        a.uhat[(size_t)f * a.v.G + g] = val;
        put_field<T>(a.D, a.out, f, i, j, k, (T)val);
    }
}

}  // namespace

// ------------------------------------------------------------- host side
ebs_status build_tiles(ebs_ctx* cx) {
    cx->h_tiles.clear();
    const int TX = cx->tile_x, TY = cx->tile_y, TZ = cx->tile_z;
    for (const ebs_box& b : cx->boxes) {
        for (int z = b.lo[2]; z < b.hi[2]; z += TZ)
            for (int y = b.lo[1]; y < b.hi[1]; y += TY)
                for (int x = b.lo[0]; x < b.hi[0]; x += TX) {
                    ebs_tile t;
                    t.x0 = x; t.y0 = y; t.z0 = z;
                    t.ex = (int16_t)std::min(TX, b.hi[0] - x);
                    t.ey = (int16_t)std::min(TY, b.hi[1] - y);
                    t.ez = (int16_t)std::min(TZ, b.hi[2] - z);
                    t.flags = 0;
                    cx->h_tiles.push_back(t);
                }
    }
    cx->ntiles = (int32_t)cx->h_tiles.size();
    if (cx->d_tiles) (void)hipFree(cx->d_tiles);
    cx->d_tiles = nullptr;
    if (hipMalloc(&cx->d_tiles, sizeof(ebs_tile) * std::max(1, cx->ntiles)) != hipSuccess) {
        cx->err = "tile list allocation failed";
        return EBS_E_OOM;
    }
    EBS_HIP(cx, hipMemcpy(cx->d_tiles, cx->h_tiles.data(), sizeof(ebs_tile) * cx->ntiles,
                          hipMemcpyHostToDevice));
    // algorithmic bytes of the regular-region kernel: cells at or above g1
    if (!cx->h_g1.empty()) {
        double cells = 0;
        for (int c = 0; c < cx->ncol; ++c) cells += (double)(cx->nz - cx->h_g1[c]);
        const double es = cx->g.precision == EBS_F32_BULK ? 4.0 : 8.0;
        cx->alg_bytes[0] = cells * 5 * es * 2;  // read Un (= Ucur), write
        cx->alg_bytes[1] = cells * 5 * es * 3;  // read Un and Ucur, write
    }
    return EBS_OK;
}

template <typename T>
static ebs_status advance_t(ebs_ctx* cx, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uh,
                            double cdt) {
    const void* const un[5] = {Un->rho, Un->rhotheta, Un->rhou, Un->rhov, Un->rhow};
    const void* const cu[5] = {Ucur->rho, Ucur->rhotheta, Ucur->rhou, Ucur->rhov, Ucur->rhow};
    void* const ou[5] = {Uh->rho, Uh->rhotheta, Uh->rhou, Uh->rhov, Uh->rhow};
    Dims D{cx->nx, cx->ny, cx->nz};
    {
        BulkArgs<T> a;
        a.D = D;
        for (int f = 0; f < 5; ++f) {
            a.un[f] = (const T*)un[f];
            a.cur[f] = (const T*)cu[f];
            a.out[f] = (T*)ou[f];
        }
        a.cdt = (T)cdt;
        a.rdx = (T)(1.0 / cx->g.dx[0]);
        a.rdy = (T)(1.0 / cx->g.dx[1]);
        a.rdz = (T)(1.0 / cx->g.dx[2]);
        a.g0 = cx->d_g0;
        a.g1 = cx->d_g1;
        a.tiles = cx->d_tiles;
        a.ntiles = cx->ntiles;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (cx->timing) {
            if (cx->ev_used + 2 > cx->ev_pool.size()) {
                for (int q = 0; q < 64; ++q) {
                    hipEvent_t e;
                    EBS_HIP(cx, hipEventCreate(&e));
                    cx->ev_pool.push_back(e);
                }
            }
            e0 = cx->ev_pool[cx->ev_used++];
            e1 = cx->ev_pool[cx->ev_used++];
            EBS_HIP(cx, hipEventRecord(e0, cx->stream));
        }
        const int blocks = std::min(cx->ntiles, 256 * 16);
        if (blocks > 0) {
            hipLaunchKernelGGL(k_bulk<T>, dim3(blocks), dim3(cx->tile_x, cx->tile_y), 0, cx->stream, a);
            EBS_HIP(cx, hipGetLastError());
        }
        if (cx->timing) EBS_HIP(cx, hipEventRecord(e1, cx->stream));
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
        a.cdt = cdt;
        for (int d = 0; d < 3; ++d) a.del[d] = cx->g.dx[d];
        a.eb_mode = cx->g.eb_flux;
        hipLaunchKernelGGL(k_general<T>, dim3((cx->G + 255) / 256), dim3(256), 0, cx->stream, a);
        EBS_HIP(cx, hipGetLastError());
    }
    return EBS_OK;
}

ebs_status launch_advance(ebs_ctx* cx, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uhat,
                          double cdt) {
    if (cx->g.precision == EBS_F32_BULK) return advance_t<float>(cx, Un, Ucur, Uhat, cdt);
    return advance_t<double>(cx, Un, Ucur, Uhat, cdt);
}

}  // namespace ebs
