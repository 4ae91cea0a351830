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
//   * the k_gen_* passes handle the general range of each column (the cut band and a
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
#include <vector>

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

// field pointer by runtime index without indexing the kernel-argument array
// (dynamic indexing would place the argument struct in scratch memory)
template <typename P>
__device__ inline P pick5(const P (&p)[5], int f) {
    return f == 0 ? p[0] : f == 1 ? p[1] : f == 2 ? p[2] : f == 3 ? p[3] : p[4];
}

// write helper covering the periodic repeats and the top wall plane
template <typename T>
__device__ inline void put_field(const Dims& D, T* const (&out)[5], int f, int i, int j, int k, T v) {
    pick5(out, f)[fidx(D, f, i, j, k)] = v;
    if (f == 2 && i == 0) out[2][iu(D, D.nx, j, k)] = v;
    if (f == 3 && j == 0) out[3][iv(D, i, D.ny, k)] = v;
    if (f == 4 && k == D.nz - 1) out[4][ic(D, i, j, D.nz)] = T(0);
}

// ------------------------------------------------------------------ bulk
//
// 2.5-D z-march.  A block owns an xy tile of TX x TY columns and walks up the
// tile's z-range.  Every plane of the five fields is read from HBM exactly once
// per block, over the tile plus a halo (3 cells on the low sides, 2 on the high
// sides), into LDS rings; the advected quantities (theta, u, v, w) are then
// computed once per point from LDS.  Rings: rho 2 planes, momenta 4 planes
// (k-1..k+2), advected quantities 3 planes (k..k+2); the own column's planes
// k-1 and k-2 of the advected quantities stay in registers.  Only U^n and the
// outputs go to HBM directly.  Consecutive blocks are spread so that each XCD
// receives a contiguous run of neighbouring tiles (shared halos stay in its
// L2).  Stencil points beyond the top and bottom walls are flagged and never
// loaded.
template <typename T>
struct BulkArgs {
    Dims D;
    const T* __restrict__ un[5];
    const T* __restrict__ cur[5];
    T* out[5];
    T cdt;
    T rdx, rdy, rdz;
    const int32_t* __restrict__ g0;
    const int32_t* __restrict__ g1;
    const ebs_tile* __restrict__ tiles;
    int32_t ntiles;
    int32_t per_xcd;  // tiles per XCD chunk
};

template <typename T>
__device__ inline T qdiv(T a, T b) {
    return a / b;
}
template <>
__device__ inline float qdiv<float>(float a, float b) {
    return a * __builtin_amdgcn_rcpf(b);
}

constexpr int HALO_PTS = 4;  // region points per thread: (TX+5)(TY+5) <= 4 TX TY for TX*TY >= 64
constexpr int NXCD = 8;

// LDS arrays, each WS entries: rho[2], rhou[4], rhov[4], rhow[4], prim[4 quantities][3]
enum : int { L_RHO = 0, L_RU = 2, L_RV = 6, L_RW = 10, L_PRIM = 14, L_COUNT = 26 };

template <typename T>
__device__ inline void prims_direct(const BulkArgs<T>& a, uint32_t c, uint32_t u, int dxm, int dym, int p,
                                    uint32_t pc, uint32_t pu, uint32_t pv, T* q) {
    if (p < 0 || p >= a.D.nz) {  // beyond the walls
        q[0] = q[1] = q[2] = q[3] = T(0);
        return;
    }
    const uint32_t oc = (uint32_t)p * pc + c;
    const T r = a.cur[0][oc];
    q[0] = qdiv<T>(a.cur[1][oc], r);
    q[1] = qdiv<T>(T(2) * a.cur[2][(uint32_t)p * pu + u], a.cur[0][oc + dxm] + r);
    q[2] = qdiv<T>(T(2) * a.cur[3][(uint32_t)p * pv + c], a.cur[0][oc + dym] + r);
    q[3] = p == 0 ? T(0) : qdiv<T>(T(2) * a.cur[4][oc], a.cur[0][oc - pc] + r);  // no w CV at k = 0
}

// six times the upwind face value (the 1/6 is applied once per CV): branch-free
// third-order upwind, second-order centred when the stencil end is unavailable
template <typename T>
__device__ __forceinline__ T upw6(T m, T pLL, T pL, T pR, T pRR, bool okLL, bool okRR) {
    const bool up = m >= T(0);
    const T a = up ? pL : pR, b = up ? pR : pL, e = up ? pLL : pRR;
    const bool ok = up ? okLL : okRR;
    return ok ? (T(5) * a + T(2) * b - e) : T(3) * (a + b);
}

// element access with a 32-bit byte offset (every field is below 4 GiB; the
// context checks it), so the address is a scalar base plus a vector offset
template <typename T>
__device__ __forceinline__ T ld(const T* __restrict__ base, uint32_t off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(off * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st(T* base, uint32_t off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(off * (uint32_t)sizeof(T))) = v;
}

template <typename T, int TX, int TY>
__global__ void __launch_bounds__(TX * TY) k_bulk(BulkArgs<T> a) {
    constexpr int WX = TX + 5, WS = WX * (TY + 5), NTHR = TX * TY;
    constexpr int NPTS = (WS + NTHR - 1) / NTHR;
    static_assert(NPTS <= HALO_PTS, "halo points per thread");
    extern __shared__ unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int nx = a.D.nx, ny = a.D.ny, nz = a.D.nz;
    const uint32_t pc = (uint32_t)nx * ny, pu = (uint32_t)(nx + 1) * ny, pv = (uint32_t)nx * (ny + 1);
    const int t = (blockIdx.x % NXCD) * a.per_xcd + blockIdx.x / NXCD;
    if (t >= a.ntiles) return;
    const ebs_tile tl = a.tiles[t];
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = ty * TX + tx;
    const bool act = tx < tl.ex && ty < tl.ey;
    const int i = tl.x0 + (act ? tx : 0), j = tl.y0 + (act ? ty : 0);
    const int z1 = tl.z0 + tl.ez;
    int ge = nz;
    if (act) {
        const int c = j * nx + i;
        const int gb = a.g0[c];
        ge = a.g1[c];
        for (int k = tl.z0; k < min(gb, z1); ++k)
            for (int f = 0; f < 5; ++f) put_field<T>(a.D, a.out, f, i, j, k, T(0));
    }
    const int k0 = tl.z0 + tl.flags;  // first plane with regular-region work (block uniform)
    if (k0 >= z1) return;
    uint32_t rc[NPTS], ru[NPTS];
#pragma unroll
    for (int q = 0; q < NPTS; ++q) {
        const int r = tid + q * NTHR;
        const int x = wrapi(tl.x0 - 3 + r % WX, nx), y = wrapi(tl.y0 - 3 + r / WX, ny);
        rc[q] = (uint32_t)(y * nx + x);
        ru[q] = (uint32_t)(y * (nx + 1) + x);
    }
    // Raw values of the next plane to enter the rings are loaded into registers
    // one z-iteration ahead (fetch) and written to LDS at the top of the next
    // iteration (commit), so the global-load latency overlaps a whole plane of
    // arithmetic.  rth keeps rho*theta of the committed plane for make_prims.
    T pfA[NPTS][5], pfB[NPTS][5], rth[NPTS];
    auto fetch = [&](int p, T (&pf)[NPTS][5]) {
        const bool in = p >= 0 && p < nz;  // block uniform
        const uint32_t oc0 = (uint32_t)p * pc, ou0 = (uint32_t)p * pu;
#pragma unroll
        for (int q = 0; q < NPTS; ++q) {
            const int r = tid + q * NTHR;
            if (q == NPTS - 1 && r >= WS) break;
            if (in) {
                pf[q][0] = ld(a.cur[0], oc0 + rc[q]);
                pf[q][1] = ld(a.cur[1], oc0 + rc[q]);
                pf[q][2] = ld(a.cur[2], ou0 + ru[q]);
                pf[q][3] = ld(a.cur[3], (uint32_t)p * pv + rc[q]);
                pf[q][4] = ld(a.cur[4], oc0 + rc[q]);
            } else {
#pragma unroll
                for (int f = 0; f < 5; ++f) pf[q][f] = T(0);
            }
        }
    };
    auto commit = [&](int p, const T (&pf)[NPTS][5]) {
        T* RHO = sm + (L_RHO + (p & 1)) * WS;
        T* RU = sm + (L_RU + (p & 3)) * WS;
        T* RV = sm + (L_RV + (p & 3)) * WS;
        T* RW = sm + (L_RW + (p & 3)) * WS;
#pragma unroll
        for (int q = 0; q < NPTS; ++q) {
            const int r = tid + q * NTHR;
            if (q == NPTS - 1 && r >= WS) break;
            RHO[r] = pf[q][0];
            rth[q] = pf[q][1];
            RU[r] = pf[q][2];
            RV[r] = pf[q][3];
            RW[r] = pf[q][4];
        }
    };
    auto make_prims = [&](int p) {
        const T* RHO = sm + (L_RHO + (p & 1)) * WS;
        const T* RHOm = sm + (L_RHO + ((p + 1) & 1)) * WS;
        const T* RU = sm + (L_RU + (p & 3)) * WS;
        const T* RV = sm + (L_RV + (p & 3)) * WS;
        const T* RW = sm + (L_RW + (p & 3)) * WS;
        T* P = sm + (L_PRIM + p % 3) * WS;
        const bool in = p >= 0 && p < nz;
#pragma unroll
        for (int q = 0; q < NPTS; ++q) {
            const int r = tid + q * NTHR;
            if (q == NPTS - 1 && r >= WS) break;
            if (r < WX || r % WX == 0) continue;
            T th = T(0), u = T(0), v = T(0), w = T(0);
            if (in) {
                const T rr = RHO[r];
                th = qdiv<T>(rth[q], rr);
                u = qdiv<T>(T(2) * RU[r], RHO[r - 1] + rr);
                v = qdiv<T>(T(2) * RV[r], RHO[r - WX] + rr);
                w = qdiv<T>(T(2) * RW[r], RHOm[r] + rr);
            }
            P[0 * 3 * WS + r] = th;
            P[1 * 3 * WS + r] = u;
            P[2 * 3 * WS + r] = v;
            P[3 * 3 * WS + r] = w;
        }
    };
    const int me = (ty + 3) * WX + (tx + 3);
    const int dxm = (i == 0) ? nx - 1 : -1;
    const int dym = (j == 0) ? ny - 1 : -1;
    const uint32_t c0 = (uint32_t)(j * nx + i), u0 = (uint32_t)(j * (nx + 1) + i);
    T m2[4], m1[4];
    prims_direct<T>(a, c0, u0, dxm, dym * nx, k0 - 2, pc, pu, pv, m2);
    prims_direct<T>(a, c0, u0, dxm, dym * nx, k0 - 1, pc, pu, pv, m1);
    // Raw planes run two z-iterations ahead in two register sets (pfA, pfB,
    // alternating), the own-cell Un values likewise (unA, unB).
    fetch(k0 - 1, pfA);
    commit(k0 - 1, pfA);
    fetch(k0, pfA);
    commit(k0, pfA);
    fetch(k0 + 1, pfA);
    __syncthreads();
    make_prims(k0);
    __syncthreads();  // the density slot of plane k0 - 1 is reused by plane k0 + 1
    commit(k0 + 1, pfA);
    fetch(k0 + 2, pfA);
    fetch(k0 + 3, pfB);
    __syncthreads();
    make_prims(k0 + 1);
    __syncthreads();  // the density slot of plane k0 is reused by plane k0 + 2
    const uint32_t ov0 = (uint32_t)(j * nx + i);
    auto fetch_un = [&](int kk, T (&dst)[5]) {
        if (act && kk < z1 && kk >= ge) {
            dst[0] = ld(a.un[0], (uint32_t)kk * pc + c0);
            dst[1] = ld(a.un[1], (uint32_t)kk * pc + c0);
            dst[2] = ld(a.un[2], (uint32_t)kk * pu + u0);
            dst[3] = ld(a.un[3], (uint32_t)kk * pv + ov0);
            dst[4] = ld(a.un[4], (uint32_t)kk * pc + c0);
        } else {
#pragma unroll
            for (int f = 0; f < 5; ++f) dst[f] = T(0);
        }
    };
    T unA[5], unB[5];
    T fzc[4] = {T(0), T(0), T(0), T(0)};  // upper z-face flux terms of the last plane
    fetch_un(k0, unA);
    fetch_un(k0 + 1, unB);
    const T sixth = T(1) / T(6);
    // one z-iteration: plane k is updated; rp holds raw plane k + 2 on entry and
    // plane k + 4 on exit, uc the Un values of plane k on entry and k + 2 on exit
    auto step = [&](int k, T (&rp)[NPTS][5], T (&uc)[5]) __attribute__((always_inline)) {
        commit(k + 2, rp);
        fetch(k + 4, rp);
        __syncthreads();
        make_prims(k + 2);
        __syncthreads();
        const int s0 = k % 3, s1 = (k + 1) % 3, s2 = (k + 2) % 3;
        const T* P0 = sm + (L_PRIM + s0) * WS + me;  // quantity q at + q * 3 * WS
        const T* P1 = sm + (L_PRIM + s1) * WS + me;
        const T* P2 = sm + (L_PRIM + s2) * WS + me;
        const T* TH = P0;
        const T* UU = P0 + 3 * WS;
        const T* VV = P0 + 6 * WS;
        const T* WW = P0 + 9 * WS;
        const T* RUk = sm + (L_RU + (k & 3)) * WS + me;
        const T* RVk = sm + (L_RV + (k & 3)) * WS + me;
        const T* RUm = sm + (L_RU + ((k + 3) & 3)) * WS + me;  // plane k-1
        const T* RVm = sm + (L_RV + ((k + 3) & 3)) * WS + me;
        const T* RWk = sm + (L_RW + (k & 3)) * WS + me;
        const T* RWp = sm + (L_RW + ((k + 1) & 3)) * WS + me;
        const T* RWm = sm + (L_RW + ((k + 3) & 3)) * WS + me;
        if (act && k >= ge) {
            const bool top = (k + 1 == nz);
            const bool okR1 = k + 1 <= nz - 1, okR2 = k + 2 <= nz - 1;
            // far upwind ends of the z stencils of the lower / upper faces inside
            // the domain (cell-centred and x-, y-face CVs; plane 0 is the bottom)
            const bool okL1 = k - 2 >= 0, okL0 = k - 1 >= 0;
            T zc[4][5];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                zc[q][0] = m2[q];
                zc[q][1] = m1[q];
                zc[q][2] = P0[q * 3 * WS];
                zc[q][3] = P1[q * 3 * WS];
                zc[q][4] = P2[q * 3 * WS];
            }
            const uint32_t oc = (uint32_t)k * pc + c0;
            const uint32_t ou = (uint32_t)k * pu + u0;
            const uint32_t ov = (uint32_t)k * pv + c0;
            const T ru_i = RUk[0], ru_ip = RUk[1], ru_im = RUk[-1];
            const T rv_j = RVk[0], rv_jp = RVk[WX], rv_jm = RVk[-WX];
            const T rw_k = RWk[0], rw_kp = top ? T(0) : RWp[0];
            const T h = T(0.5);
            // lower z-face flux terms: carried from the upper faces of plane k - 1
            // when this thread updated it (same values, same arithmetic)
            T zl[4];
            if (k > k0 && k - 1 >= ge) {
#pragma unroll
                for (int q = 0; q < 4; ++q) zl[q] = fzc[q];
            } else {
                zl[0] = rw_k * upw6<T>(rw_k, zc[0][0], zc[0][1], zc[0][2], zc[0][3], okL1, okR1);
                const T m1l = h * (RWk[-1] + rw_k), m2l = h * (RWk[-WX] + rw_k);
                const T m3l = (k != 1) ? h * (RWm[0] + rw_k) : T(0);
                zl[1] = m1l * upw6<T>(m1l, zc[1][0], zc[1][1], zc[1][2], zc[1][3], okL1, okR1);
                zl[2] = m2l * upw6<T>(m2l, zc[2][0], zc[2][1], zc[2][2], zc[2][3], okL1, okR1);
                zl[3] = m3l * upw6<T>(m3l, zc[3][0], zc[3][1], zc[3][2], zc[3][3], k - 2 >= 1, okR1);
            }
            // ---- cell-centred instance
            {
                const T ex = ru_ip - ru_i, ey = rv_jp - rv_j, ez = rw_kp - rw_k;
                const T fx = ru_ip * upw6<T>(ru_ip, TH[-1], TH[0], TH[1], TH[2], true, true) -
                             ru_i * upw6<T>(ru_i, TH[-2], TH[-1], TH[0], TH[1], true, true);
                const T fy = rv_jp * upw6<T>(rv_jp, TH[-WX], TH[0], TH[WX], TH[2 * WX], true, true) -
                             rv_j * upw6<T>(rv_j, TH[-2 * WX], TH[-WX], TH[0], TH[WX], true, true);
                fzc[0] = rw_kp * upw6<T>(rw_kp, zc[0][1], zc[0][2], zc[0][3], zc[0][4], okL0, okR2);
                const T fz = fzc[0] - zl[0];
                const T dr = ex * a.rdx + ey * a.rdy + ez * a.rdz;
                const T dt = (fx * a.rdx + fy * a.rdy + fz * a.rdz) * sixth;
                st(a.out[0], oc, uc[0] - a.cdt * dr);
                st(a.out[1], oc, uc[1] - a.cdt * dt);
            }
            // ---- x-face instance
            {
                const T mxl = h * (ru_im + ru_i), mxh = h * (ru_i + ru_ip);
                const T myl = h * (RVk[-1] + rv_j), myh = h * (RVk[WX - 1] + rv_jp);
                const T mzh = top ? T(0) : h * (RWp[-1] + rw_kp);
                const T fx = mxh * upw6<T>(mxh, UU[-1], UU[0], UU[1], UU[2], true, true) -
                             mxl * upw6<T>(mxl, UU[-2], UU[-1], UU[0], UU[1], true, true);
                const T fy = myh * upw6<T>(myh, UU[-WX], UU[0], UU[WX], UU[2 * WX], true, true) -
                             myl * upw6<T>(myl, UU[-2 * WX], UU[-WX], UU[0], UU[WX], true, true);
                fzc[1] = mzh * upw6<T>(mzh, zc[1][1], zc[1][2], zc[1][3], zc[1][4], okL0, okR2);
                const T fz = fzc[1] - zl[1];
                const T val = uc[2] - a.cdt * (fx * a.rdx + fy * a.rdy + fz * a.rdz) * sixth;
                st(a.out[2], ou, val);
                if (i == 0) st(a.out[2], ou + nx, val);
            }
            // ---- y-face instance
            {
                const T mxl = h * (RUk[-WX] + ru_i), mxh = h * (RUk[1 - WX] + ru_ip);
                const T myl = h * (rv_jm + rv_j), myh = h * (rv_j + rv_jp);
                const T mzh = top ? T(0) : h * (RWp[-WX] + rw_kp);
                const T fx = mxh * upw6<T>(mxh, VV[-1], VV[0], VV[1], VV[2], true, true) -
                             mxl * upw6<T>(mxl, VV[-2], VV[-1], VV[0], VV[1], true, true);
                const T fy = myh * upw6<T>(myh, VV[-WX], VV[0], VV[WX], VV[2 * WX], true, true) -
                             myl * upw6<T>(myl, VV[-2 * WX], VV[-WX], VV[0], VV[WX], true, true);
                fzc[2] = mzh * upw6<T>(mzh, zc[2][1], zc[2][2], zc[2][3], zc[2][4], okL0, okR2);
                const T fz = fzc[2] - zl[2];
                const T val = uc[3] - a.cdt * (fx * a.rdx + fy * a.rdy + fz * a.rdz) * sixth;
                st(a.out[3], ov, val);
                if (j == 0) st(a.out[3], ov + (uint32_t)ny * nx, val);
            }
            // ---- z-face instance (k >= 1 in the regular range); zero flux
            // through the mid planes of the bottom and top cell layers
            {
                const T mxl = h * (RUm[0] + ru_i), mxh = h * (RUm[1] + ru_ip);
                const T myl = h * (RVm[0] + rv_j), myh = h * (RVm[WX] + rv_jp);
                // (at k = 0 there is no z-face CV: its "upper face" term is the
                // zero flux of the lower face of the CV at k = 1, carried up)
                const T mzh = (k != nz - 1 && k != 0) ? h * (rw_k + rw_kp) : T(0);
                const T fx = mxh * upw6<T>(mxh, WW[-1], WW[0], WW[1], WW[2], true, true) -
                             mxl * upw6<T>(mxl, WW[-2], WW[-1], WW[0], WW[1], true, true);
                const T fy = myh * upw6<T>(myh, WW[-WX], WW[0], WW[WX], WW[2 * WX], true, true) -
                             myl * upw6<T>(myl, WW[-2 * WX], WW[-WX], WW[0], WW[WX], true, true);
                fzc[3] = mzh * upw6<T>(mzh, zc[3][1], zc[3][2], zc[3][3], zc[3][4], k - 1 >= 1, okR2);
                const T fz = fzc[3] - zl[3];
                // plane 0 holds the bottom wall face, not a CV
                st(a.out[4], oc, k == 0 ? T(0) : uc[4] - a.cdt * (fx * a.rdx + fy * a.rdy + fz * a.rdz) * sixth);
                if (k == nz - 1) st(a.out[4], oc + pc, T(0));
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            m2[q] = m1[q];
            m1[q] = P0[q * 3 * WS];
        }
        fetch_un(k + 2, uc);
        __syncthreads();
    };
    for (int k = k0; k < z1; k += 2) {
        step(k, pfA, unA);
        if (k + 1 < z1) step(k + 1, pfB, unB);
    }
}

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
        constexpr int s = F < 2 ? 0 : F - 1;
        if (P.k == a.D.nz) return 0.0;  // top wall: zero flux
        if (!(P.ff & ff_pos(s, D))) return 0.0;
        const double F0 = fhat_any<F, D>(P);
        if (P.ff & ff_full(s, D)) return F0;
        const uint32_t part = (P.ff & 0xFFFu) & ~(P.ff >> 16);
        const CutRec& r = a.crec[a.cbase[P.g] + __popc(part & (ff_pos(s, D) - 1u))];
        const double* fhd = a.fh + ((size_t)F * 3 + D) * a.v.Ge;
        double Fv = r.c[0] * F0;
        if (r.n[0] >= 0) Fv += r.c[1] * fhd[r.n[0]];
        if (r.n[1] >= 0) Fv += r.c[2] * fhd[r.n[1]];
        if (r.n[2] >= 0) Fv += r.c[3] * fhd[r.n[2]];
        return r.b * Fv;
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
    // divergence term of field F at the CV P (upper neighbours Ux, Uy, Uz)
    template <int F, int D>
    __device__ __forceinline__ double div_dir(const Pt& P, const Pt& U, int g) const {
        constexpr int s = F < 2 ? 0 : F - 1;
        const double rd = a.rdel[D];
        double br = (bface<F, D>(U) - bface<F, D>(P)) * rd;
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
        double val = 0.0;
        if ((P.fl >> s) & 1) {
            const double al = geo(s, GQ_ALPHA, g);
            double br = div_dir<F, 0>(P, Ux, g);
            br += div_dir<F, 1>(P, Uy, g);
            br += div_dir<F, 2>(P, Uz, g);
            val = st(a.un, F, P.i, P.j, P.k) - a.cdt * br / al;
        }
        a.uhat[(size_t)F * a.v.G + g] = val;
        put_field<T>(a.D, a.out, F, P.i, P.j, P.k, (T)val);
    }
    template <int D>
    __device__ __forceinline__ void fhat_dir(const Pt& P, const Pt& Lx, const Pt& Ly, const Pt& Lz,
                                             const int4& ci, int g) const {
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
        a.fh[(0 * 3 + D) * G + g] = (ff & ff_pos(0, D)) ? fhat<0, D>(LL, L, P, RR, P) : 0.0;
        a.fh[(1 * 3 + D) * G + g] = (ff & ff_pos(0, D)) ? fhat<1, D>(LL, L, P, RR, P) : 0.0;
        a.fh[(2 * 3 + D) * G + g] = (ff & ff_pos(1, D)) ? fhat<2, D>(LL, L, P, RR, Lx) : 0.0;
        a.fh[(3 * 3 + D) * G + g] = (ff & ff_pos(2, D)) ? fhat<3, D>(LL, L, P, RR, Ly) : 0.0;
        a.fh[(4 * 3 + D) * G + g] = (ff & ff_pos(3, D)) ? fhat<4, D>(LL, L, P, RR, Lz) : 0.0;
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
    G.template fhat_dir<0>(P, Lx, Ly, Lz, ci, g);
    G.template fhat_dir<1>(P, Lx, Ly, Lz, ci, g);
    G.template fhat_dir<2>(P, Lx, Ly, Lz, ci, g);
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
    if (hipMalloc(&cx->d_crec, sizeof(CutRec) * std::max<int64_t>(tot, 1)) != hipSuccess) {
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

size_t bulk_lds_bytes(int tx, int ty, int precision) {
    return (precision == EBS_F32_BULK ? 4 : 8) * (size_t)L_COUNT * (tx + 5) * (ty + 5);
}

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
                    // first plane at or above the general range of every column
                    int kmin = cx->nz;
                    for (int yy = y; yy < y + t.ey; ++yy)
                        for (int xx = x; xx < x + t.ex; ++xx)
                            kmin = std::min(kmin, cx->h_g1.empty() ? 0 : cx->h_g1[yy * cx->nx + xx]);
                    t.flags = (int16_t)std::min<int>(std::max(kmin - z, 0), t.ez);
                    cx->h_tiles.push_back(t);
                }
    }
    // Order: z band, then Morton order of the tile origin in 16-cell units.  The
    // launch hands each XCD a contiguous run of this list, so the blocks resident
    // on one XCD cover a compact patch at similar heights and share their halo
    // cache lines in that XCD's L2.
    auto morton = [](uint32_t x, uint32_t y) {
        uint64_t m = 0;
        for (int b = 0; b < 16; ++b) m |= (uint64_t)((x >> b) & 1) << (2 * b) | (uint64_t)((y >> b) & 1) << (2 * b + 1);
        return m;
    };
    std::stable_sort(cx->h_tiles.begin(), cx->h_tiles.end(), [&](const ebs_tile& p, const ebs_tile& q) {
        const int bp = p.z0 / TZ, bq = q.z0 / TZ;
        if (bp != bq) return bp < bq;
        return morton(p.x0 >> 4, p.y0 >> 4) < morton(q.x0 >> 4, q.y0 >> 4);
    });
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
                            double cdt, bool defer_join) {
    // The regular-region kernel and the general-range passes write disjoint
    // cells and read U_cur (never an output), so the former runs on the side
    // stream, forked from and joined back into the context stream.
    const bool fork = cx->side && cx->ntiles > 0 && cx->G > 0;
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
            EBS_HIP(cx, hipEventRecord(e0, bs));
        }
        const size_t lds = bulk_lds_bytes(cx->tile_x, cx->tile_y, cx->g.precision);
        a.per_xcd = (cx->ntiles + NXCD - 1) / NXCD;
        if (cx->ntiles > 0) {
            const dim3 grid(a.per_xcd * NXCD), blk(cx->tile_x, cx->tile_y);
#define EBS_BULK_CASE(X, Y)                                                                   \
    if (cx->tile_x == X && cx->tile_y == Y) {                                                 \
        hipLaunchKernelGGL((k_bulk<T, X, Y>), grid, blk, lds, bs, a);                         \
    } else
            EBS_BULK_CASE(16, 4) EBS_BULK_CASE(16, 8) EBS_BULK_CASE(16, 16) EBS_BULK_CASE(32, 4)
            EBS_BULK_CASE(32, 8) EBS_BULK_CASE(64, 2) EBS_BULK_CASE(64, 4) {
                cx->err = "tile shape without a compiled kernel";
                return EBS_E_UNSUPPORTED;
            }
#undef EBS_BULK_CASE
            EBS_HIP(cx, hipGetLastError());
        }
        if (cx->timing) EBS_HIP(cx, hipEventRecord(e1, bs));
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
        a.cdt = cdt;
        for (int d = 0; d < 3; ++d) a.rdel[d] = 1.0 / cx->g.dx[d];
        a.eb_mode = cx->g.eb_flux;
        const dim3 grid((cx->G + 255) / 256), gride((cx->Ge + 255) / 256), blk(256);
        // the first two passes only read the input state; the update writes
        // the output (which may alias U^n, never U_cur)
        hipLaunchKernelGGL(k_gen_prims<T>, grid, blk, 0, cx->stream, a);
        hipLaunchKernelGGL(k_gen_fhat<T>, gride, blk, 0, cx->stream, a);
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
