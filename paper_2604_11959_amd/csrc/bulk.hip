// Regular-region stage kernel: the explicit update of the four instances
// (Eqs. update-cc / update-fc of Section 3.1 with the advective flux of
// Section 4.1; Algorithm 1 steps 1-3) on every cell at or above its column's
// general range.  Every CV and every stencil member there is a full cell, so
// the update needs no geometry: face fractions are one, no flux is moved to a
// centroid, and the only special cases are the top and bottom walls.  It runs
// over a tile list derived from the box list, in the state precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ebs_internal.h"
#include "stage_common.h"

namespace ebs {
namespace {

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
//
// With the momentum sources (SRC), the perturbation pressure of every plane
// is evaluated once per point from the raw rho theta of the region loads, for
// the own cells and the -x column and -y row next to the tile, into a
// two-plane LDS ring; the own column's p' and rho of the plane below stay in
// registers.
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
    // sources: per-level table [5][nz] (p0, rho theta0 high and low part,
    // 1 / rho theta0, rho0), gravity, gamma
    const T* __restrict__ sref;
    T sg, sgam;
    T bc[8];  // FP32: binomial coefficients C(gamma, n), n = 1..8
};

__device__ __forceinline__ float log1p_t(float x) { return log1pf(x); }
__device__ __forceinline__ double log1p_t(double x) { return log1p(x); }
__device__ __forceinline__ float expm1_t(float x) { return expm1f(x); }
__device__ __forceinline__ double expm1_t(double x) { return expm1(x); }

// perturbation pressure of a cell of level k from its rho theta:
// p - p0 = p0 ((rho theta / rho theta0)^gamma - 1), evaluated from the
// relative departure (rho theta - rho theta0) / rho theta0 so that the small
// difference keeps the state precision's relative accuracy (FP32: rho theta0
// as a float pair, so the departure is exact up to one rounding)
//
// FP32: (1 + x)^gamma - 1 from the binomial series sum_{n=1..8} C(gamma, n) x^n
// for |x| < 1/8 (truncation below 1e-9 relative; coefficients in bc[]).
// Beyond, 1 + x is first divided by a tabulated R = 2^(m/8) close to it (m
// from the hardware base-2 logarithm, which only has to pick the entry):
// y = x R' + (R' - 1) with R' = 1/R is exact up to one rounding and below
// 2^(1/16) - 1 in magnitude, so the same series gives (1 + y)^gamma - 1, and
// (1 + x)^gamma - 1 = c (1 + y)^gamma - 1 = c s + (c - 1) with c = R^gamma
// (table entries {R', R' - 1, c, c - 1} for m = -32..32, formed in FP64 from
// the FP32 value of R').  No library call and no extra registers on the
// common path (expm1f / log1pf made the kernel spill or, out of line, cost a
// call frame), and no subtraction of two values near 1 (the hardware base-2
// exponential and logarithm of the whole power would put an error of about
// 1.5e-7 p0 on p', several times its own rounding).  FP64: log1p and expm1.
constexpr int PP_DEG = 8;
constexpr int PP_TAB = 32;  // table entries m = -PP_TAB .. PP_TAB, after the 5 nz level values
template <typename T>
__device__ __forceinline__ T pow_series(const T* bc, T x) {
    T e = bc[PP_DEG - 1];
#pragma unroll
    for (int n = PP_DEG - 2; n >= 0; --n) e = e * x + bc[n];
    return e * x;
}
template <typename T>
__device__ __forceinline__ T pprime(const T* __restrict__ sref, int nz, T gam, const T* bc, T rt, int k) {
    if constexpr (sizeof(T) == 8) {
        const T x = (rt - sref[nz + k]) / sref[nz + k];
        return sref[k] * expm1_t(gam * log1p_t(x));
    } else {
        const float x = ((rt - sref[nz + k]) - sref[2 * nz + k]) * sref[3 * nz + k];
        float e;
        if (fabsf(x) < 0.125f) {
            e = pow_series<float>(bc, x);
        } else {
            const int m = (int)rintf(8.0f * __builtin_amdgcn_logf(1.0f + x));
            const float* t = sref + 5 * nz + 4 * (min(max(m, -PP_TAB), PP_TAB) + PP_TAB);
            const float y = fmaf(x, t[0], t[1]);
            e = fmaf(t[2], pow_series<float>(bc, y), t[3]);
        }
        return sref[k] * e;
    }
}

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

// the same for z-faces, whose wall flags are uniform over the block: the
// common case (both stencil ends inside the domain) takes a branch-free path
template <typename T>
__device__ __forceinline__ T upw6z(T m, T pLL, T pL, T pR, T pRR, bool okLL, bool okRR) {
    if (okLL && okRR) return upw6<T>(m, pLL, pL, pR, pRR, true, true);
    return upw6<T>(m, pLL, pL, pR, pRR, okLL, okRR);
}

// element access with a 32-bit byte offset (every field is below 4 GiB; the
// context checks it), so the address is a scalar base plus a vector offset
template <typename T>
__device__ __forceinline__ T ld(const T* __restrict__ base, uint32_t off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(off * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ void st(T* base, uint32_t off, T v) {
    // written once per stage and not read again by this launch: streaming store
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + (uint32_t)(off * (uint32_t)sizeof(T))));
}
// own-cell U^n values, read once per launch: streaming load
template <typename T>
__device__ __forceinline__ T ld_once(const T* __restrict__ base, uint32_t off) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(off * (uint32_t)sizeof(T))));
}

// One tile of the regular-region update (the whole 2.5-D march of a block).
// SAME: U^n and U_cur are the same state (the first stage), so the own-cell
// values of U^n are taken from the region loads instead of being read again.
template <typename T, int TX, int TY, bool SAME, bool SRC>
__device__ __forceinline__ void bulk_tile(const BulkArgs<T>& a, int t, T* sm) {
    constexpr int WX = TX + 5, WS = WX * (TY + 5), NTHR = TX * TY, NH = WS - NTHR;
    constexpr int PW = TX + 1, PS = PW * (TY + 1);  // pressure plane: own cells, -x column, -y row
    constexpr int NPTS = 1 + (NH + NTHR - 1) / NTHR;
    static_assert(NPTS <= HALO_PTS, "halo points per thread");
    const int nx = a.D.nx, ny = a.D.ny, nz = a.D.nz;
    const uint32_t pc = (uint32_t)nx * ny, pu = (uint32_t)(nx + 1) * ny, pv = (uint32_t)nx * (ny + 1);
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
    // Region points of this thread (row-major index into the (TX+5) x (TY+5)
    // region): point 0 is its own column's cell; points q >= 1 are the halo
    // points numbered tid + (q - 1) NTHR (rows 0-2, then the 3 + 2 side points
    // of each interior row, then the last two rows); lr = -1 past the last.
    const int me = (ty + 3) * WX + (tx + 3);
    int lr[NPTS], lp[NPTS];
    uint32_t rc[NPTS], ru[NPTS];
#pragma unroll
    for (int q = 0; q < NPTS; ++q) {
        int r = me;
        if (q > 0) {
            int h = tid + (q - 1) * NTHR;
            if (h >= NH) {
                r = -1;
            } else if (h < 3 * WX) {
                r = h;
            } else if ((h -= 3 * WX) < 5 * TY) {
                const int c = h % 5;
                r = (3 + h / 5) * WX + (c < 3 ? c : TX + c);
            } else {
                r = (TY + 3) * WX + (h - 5 * TY);
            }
        }
        lr[q] = r;
        if (SRC) {
            const int rx = r % WX, ry = r / WX;
            const bool win = r >= 0 && rx >= 2 && rx <= TX + 2 && ry >= 2 && ry <= TY + 2 && (rx > 2 || ry > 2);
            lp[q] = win ? (ry - 2) * PW + (rx - 2) : -1;
        }
        const int rr = max(r, 0);
        const int x = wrapi(tl.x0 - 3 + rr % WX, nx), y = wrapi(tl.y0 - 3 + rr / WX, ny);
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
            if (q > 0 && lr[q] < 0) break;
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
            const int r = lr[q];
            if (q > 0 && r < 0) break;
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
            const int r = lr[q];
            if (q > 0 && r < 0) break;
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
    // SRC: p' of plane p at this thread's points in the pressure window, from
    // the raw rho theta of the last commit (rth); returns the own cell's value
    T* const PPB = sm + L_COUNT * WS;
    auto write_pp = [&](int p) -> T {
        T own = T(0);
        if (p < 0 || p >= nz) return own;  // block uniform
        T* PP = PPB + (p & 1) * PS;
#pragma unroll
        for (int q = 0; q < NPTS; ++q) {
            if (q > 0 && lr[q] < 0) break;
            if (lp[q] < 0) continue;
            const T v = pprime<T>(a.sref, nz, a.sgam, a.bc, rth[q], p);
            PP[lp[q]] = v;
            if (q == 0) own = v;
        }
        return own;
    };
    auto own_rho = [&](int p) -> T { return sm[(L_RHO + (p & 1)) * WS + me]; };
    const int dxm = (i == 0) ? nx - 1 : -1;
    const int dym = (j == 0) ? ny - 1 : -1;
    const uint32_t c0 = (uint32_t)(j * nx + i), u0 = (uint32_t)(j * (nx + 1) + i);
    T m2[4], m1[4];
    prims_direct<T>(a, c0, u0, dxm, dym * nx, k0 - 2, pc, pu, pv, m2);
    prims_direct<T>(a, c0, u0, dxm, dym * nx, k0 - 1, pc, pu, pv, m1);
    // Raw planes run two z-iterations ahead in two register sets (pfA, pfB,
    // alternating), the own-cell Un values likewise (unA, unB).  With SAME,
    // unA / unB keep rho and rho theta of the own cell from the region loads
    // (point 0) and the momenta are read from the LDS rings.
    T unA[5], unB[5];
    // SRC: own p' of planes k - 1, k, k + 1 and own rho of planes k - 1, k
    T ppm = T(0), pc0 = T(0), pc1 = T(0), rkm = T(0), rk = T(0);
    fetch(k0 - 1, pfA);
    commit(k0 - 1, pfA);
    if (SRC) {
        ppm = (k0 >= 1) ? pprime<T>(a.sref, nz, a.sgam, a.bc, rth[0], k0 - 1) : T(0);
        rkm = own_rho(k0 - 1);
    }
    fetch(k0, pfA);
    if (SAME) unA[0] = pfA[0][0], unA[1] = pfA[0][1];
    commit(k0, pfA);
    fetch(k0 + 1, pfA);
    __syncthreads();
    make_prims(k0);
    __syncthreads();  // the density slot of plane k0 - 1 is reused by plane k0 + 1
    if (SAME) unB[0] = pfA[0][0], unB[1] = pfA[0][1];
    if (SRC) pc0 = write_pp(k0);
    commit(k0 + 1, pfA);
    fetch(k0 + 2, pfA);
    fetch(k0 + 3, pfB);
    __syncthreads();
    make_prims(k0 + 1);
    __syncthreads();  // the density slot of plane k0 is reused by plane k0 + 2
    const uint32_t ov0 = (uint32_t)(j * nx + i);
    auto fetch_un = [&](int kk, T (&dst)[5]) {
        if (act && kk < z1 && kk >= ge) {
            dst[0] = ld_once(a.un[0], (uint32_t)kk * pc + c0);
            dst[1] = ld_once(a.un[1], (uint32_t)kk * pc + c0);
            dst[2] = ld_once(a.un[2], (uint32_t)kk * pu + u0);
            dst[3] = ld_once(a.un[3], (uint32_t)kk * pv + ov0);
            dst[4] = ld_once(a.un[4], (uint32_t)kk * pc + c0);
        } else {
#pragma unroll
            for (int f = 0; f < 5; ++f) dst[f] = T(0);
        }
    };
    T fzc[4] = {T(0), T(0), T(0), T(0)};  // upper z-face flux terms of the last plane
    // (with the sources, whose extra registers would not fit beside two
    // planes of U^n, U^n is loaded at the top of its own z-iteration)
    if (!SAME && !SRC) {
        fetch_un(k0, unA);
        fetch_un(k0 + 1, unB);
    }
    const T sixth = T(1) / T(6);
    // one z-iteration: plane k is updated; rp holds raw plane k + 2 on entry and
    // plane k + 4 on exit, uc the Un values of plane k on entry and k + 2 on exit
    auto step = [&](int k, T (&rp)[NPTS][5], T (&uc)[5]) __attribute__((always_inline)) {
        T nr0 = T(0), nr1 = T(0);  // SAME: rho, rho theta of the own cell of plane k + 2
        if (SAME) nr0 = rp[0][0], nr1 = rp[0][1];
        if (SRC) {
            if (!SAME) fetch_un(k, uc);
            rk = own_rho(k);  // plane k leaves the density ring with this commit
            pc1 = write_pp(k + 1);
        }
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
            // The staggered instances' mass fluxes are the means of two stored
            // momenta; their factor 1/2 is applied once, with the 1/6 of the
            // upwind values (scaling by 1/2 is exact, so every rounding is the
            // same as with the factor inside).
            const T hs = T(0.5) * sixth;
            // lower z-face flux terms: carried from the upper faces of plane k - 1
            // when this thread updated it (same values, same arithmetic)
            T zl[4];
            if (k > k0 && k - 1 >= ge) {
#pragma unroll
                for (int q = 0; q < 4; ++q) zl[q] = fzc[q];
            } else {
                zl[0] = rw_k * upw6z<T>(rw_k, zc[0][0], zc[0][1], zc[0][2], zc[0][3], okL1, okR1);
                const T m1l = RWk[-1] + rw_k, m2l = RWk[-WX] + rw_k;
                const T m3l = (k != 1) ? RWm[0] + rw_k : T(0);
                zl[1] = m1l * upw6z<T>(m1l, zc[1][0], zc[1][1], zc[1][2], zc[1][3], okL1, okR1);
                zl[2] = m2l * upw6z<T>(m2l, zc[2][0], zc[2][1], zc[2][2], zc[2][3], okL1, okR1);
                zl[3] = m3l * upw6z<T>(m3l, zc[3][0], zc[3][1], zc[3][2], zc[3][3], k - 2 >= 1, okR1);
            }
            // sources of the three momentum CVs of this cell (p' of the own
            // cell and of its -x, -y, -z neighbours, all fluid here), each
            // evaluated next to its use
            const T* PPk = PPB + (k & 1) * PS + (ty + 1) * PW + (tx + 1);
            // ---- cell-centred instance
            {
                const T ex = ru_ip - ru_i, ey = rv_jp - rv_j, ez = rw_kp - rw_k;
                const T fx = ru_ip * upw6<T>(ru_ip, TH[-1], TH[0], TH[1], TH[2], true, true) -
                             ru_i * upw6<T>(ru_i, TH[-2], TH[-1], TH[0], TH[1], true, true);
                const T fy = rv_jp * upw6<T>(rv_jp, TH[-WX], TH[0], TH[WX], TH[2 * WX], true, true) -
                             rv_j * upw6<T>(rv_j, TH[-2 * WX], TH[-WX], TH[0], TH[WX], true, true);
                fzc[0] = rw_kp * upw6z<T>(rw_kp, zc[0][1], zc[0][2], zc[0][3], zc[0][4], okL0, okR2);
                const T fz = fzc[0] - zl[0];
                const T dr = ex * a.rdx + ey * a.rdy + ez * a.rdz;
                const T dt = (fx * a.rdx + fy * a.rdy + fz * a.rdz) * sixth;
                st(a.out[0], oc, uc[0] - a.cdt * dr);
                st(a.out[1], oc, uc[1] - a.cdt * dt);
            }
            // ---- x-face instance
            {
                const T mxl = ru_im + ru_i, mxh = ru_i + ru_ip;
                const T myl = RVk[-1] + rv_j, myh = RVk[WX - 1] + rv_jp;
                const T mzh = top ? T(0) : RWp[-1] + rw_kp;
                const T fx = mxh * upw6<T>(mxh, UU[-1], UU[0], UU[1], UU[2], true, true) -
                             mxl * upw6<T>(mxl, UU[-2], UU[-1], UU[0], UU[1], true, true);
                const T fy = myh * upw6<T>(myh, UU[-WX], UU[0], UU[WX], UU[2 * WX], true, true) -
                             myl * upw6<T>(myl, UU[-2 * WX], UU[-WX], UU[0], UU[WX], true, true);
                fzc[1] = mzh * upw6z<T>(mzh, zc[1][1], zc[1][2], zc[1][3], zc[1][4], okL0, okR2);
                const T fz = fzc[1] - zl[1];
                T val = (SAME ? ru_i : uc[2]) - a.cdt * (fx * a.rdx + fy * a.rdy + fz * a.rdz) * hs;
                if (SRC) val += a.cdt * (-(pc0 - PPk[-1]) * a.rdx);
                st(a.out[2], ou, val);
                if (i == 0) st(a.out[2], ou + nx, val);
            }
            // ---- y-face instance
            {
                const T mxl = RUk[-WX] + ru_i, mxh = RUk[1 - WX] + ru_ip;
                const T myl = rv_jm + rv_j, myh = rv_j + rv_jp;
                const T mzh = top ? T(0) : RWp[-WX] + rw_kp;
                const T fx = mxh * upw6<T>(mxh, VV[-1], VV[0], VV[1], VV[2], true, true) -
                             mxl * upw6<T>(mxl, VV[-2], VV[-1], VV[0], VV[1], true, true);
                const T fy = myh * upw6<T>(myh, VV[-WX], VV[0], VV[WX], VV[2 * WX], true, true) -
                             myl * upw6<T>(myl, VV[-2 * WX], VV[-WX], VV[0], VV[WX], true, true);
                fzc[2] = mzh * upw6z<T>(mzh, zc[2][1], zc[2][2], zc[2][3], zc[2][4], okL0, okR2);
                const T fz = fzc[2] - zl[2];
                T val = (SAME ? rv_j : uc[3]) - a.cdt * (fx * a.rdx + fy * a.rdy + fz * a.rdz) * hs;
                if (SRC) val += a.cdt * (-(pc0 - PPk[-PW]) * a.rdy);
                st(a.out[3], ov, val);
                if (j == 0) st(a.out[3], ov + (uint32_t)ny * nx, val);
            }
            // ---- z-face instance (k >= 1 in the regular range); zero flux
            // through the mid planes of the bottom and top cell layers
            {
                const T mxl = RUm[0] + ru_i, mxh = RUm[1] + ru_ip;
                const T myl = RVm[0] + rv_j, myh = RVm[WX] + rv_jp;
                // (at k = 0 there is no z-face CV: its "upper face" term is the
                // zero flux of the lower face of the CV at k = 1, carried up)
                const T mzh = (k != nz - 1 && k != 0) ? rw_k + rw_kp : T(0);
                const T fx = mxh * upw6<T>(mxh, WW[-1], WW[0], WW[1], WW[2], true, true) -
                             mxl * upw6<T>(mxl, WW[-2], WW[-1], WW[0], WW[1], true, true);
                const T fy = myh * upw6<T>(myh, WW[-WX], WW[0], WW[WX], WW[2 * WX], true, true) -
                             myl * upw6<T>(myl, WW[-2 * WX], WW[-WX], WW[0], WW[WX], true, true);
                fzc[3] = mzh * upw6z<T>(mzh, zc[3][1], zc[3][2], zc[3][3], zc[3][4], k - 1 >= 1, okR2);
                const T fz = fzc[3] - zl[3];
                // plane 0 holds the bottom wall face, not a CV
                T val = (SAME ? rw_k : uc[4]) - a.cdt * (fx * a.rdx + fy * a.rdy + fz * a.rdz) * hs;
                if (SRC && k >= 1)
                    val += a.cdt * (-(pc0 - ppm) * a.rdz -
                                    a.sg * T(0.5) * ((rk - a.sref[4 * nz + k]) + (rkm - a.sref[4 * nz + k - 1])));
                st(a.out[4], oc, k == 0 ? T(0) : val);
                if (k == nz - 1) st(a.out[4], oc + pc, T(0));
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            m2[q] = m1[q];
            m1[q] = P0[q * 3 * WS];
        }
        if (SAME) {
            uc[0] = nr0;
            uc[1] = nr1;
        } else if (!SRC) {
            fetch_un(k + 2, uc);
        }
        if (SRC) {
            ppm = pc0;
            pc0 = pc1;
            rkm = rk;
        }
        __syncthreads();
    };
    for (int k = k0; k < z1; k += 2) {
        step(k, pfA, unA);
        if (k + 1 < z1) step(k + 1, pfB, unB);
    }
}

// Block b runs on XCD b % NXCD and takes that XCD's contiguous chunk of the
// tile list (per_xcd tiles), one tile per iteration with a stride of the
// number of blocks per XCD: a single iteration when the grid covers every
// tile, several in the persistent schedule (a grid of as many blocks as the
// GPU holds at once), where a static stride keeps the tiles that run
// together on one XCD neighbours in the list.
template <typename T, int TX, int TY, bool SAME, bool SRC, bool PERSIST>
__global__ void __launch_bounds__(TX * TY) k_bulk(BulkArgs<T> a) {
    extern __shared__ unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    const int xcd = blockIdx.x % NXCD, slot = blockIdx.x / NXCD;
    if (!PERSIST) {  // one tile per block (kept free of the loop: no extra live registers)
        bulk_tile<T, TX, TY, SAME, SRC>(a, xcd * a.per_xcd + slot, sm);
        return;
    }
    const int nslot = gridDim.x / NXCD;
    for (int s = slot; s < a.per_xcd; s += nslot) {
        bulk_tile<T, TX, TY, SAME, SRC>(a, xcd * a.per_xcd + s, sm);
        if (s + nslot < a.per_xcd) __syncthreads();  // the next tile reuses the LDS rings
    }
}

template <typename T>
ebs_status launch_bulk_t(ebs_ctx* cx, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uh, double cdt,
                         hipStream_t bs) {
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
        const bool src = cx->src_on;
        const size_t lds = bulk_lds_bytes(cx->tile_x, cx->tile_y, cx->g.precision, src);
        a.sref = nullptr;
        a.sg = a.sgam = T(0);
        if (src) {
            a.sref = cx->g.precision == EBS_F32_BULK ? (const T*)(const void*)cx->d_srcf
                                                     : (const T*)(const void*)cx->d_srcd;
            a.sg = (T)cx->src.g;
            a.sgam = (T)cx->src.gamma;
            double cn = 1.0;
            for (int q = 0; q < 8; ++q) {  // C(gamma, q + 1)
                cn *= (cx->src.gamma - q) / (q + 1);
                a.bc[q] = (T)cn;
            }
        }
        a.per_xcd = (cx->ntiles + NXCD - 1) / NXCD;
        bool same = true;
        for (int f = 0; f < 5; ++f) same = same && un[f] == cu[f];
        if (cx->ntiles > 0) {
            const dim3 blk(cx->tile_x, cx->tile_y);
            // blocks per XCD: every tile of the chunk, or (persistent) as many
            // as the XCD holds at once, resident blocks per CU times its CUs
            auto blocks_per_xcd = [&](const void* kf) -> int {
                if (!cx->persistent) return a.per_xcd;
                int per_cu = 0, dev = 0, ncu = 0;
                if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kf, blk.x * blk.y, lds) != hipSuccess ||
                    hipGetDevice(&dev) != hipSuccess ||
                    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                    per_cu <= 0 || ncu <= 0)
                    return a.per_xcd;
                return std::max(1, std::min(a.per_xcd, per_cu * ncu / NXCD));
            };
#define EBS_BULK_CASE(X, Y)                                                                   \
    if (cx->tile_x == X && cx->tile_y == Y) {                                                 \
        auto kf = cx->persistent                                                              \
            ? (src ? (same ? k_bulk<T, X, Y, true, true, true> : k_bulk<T, X, Y, false, true, true>)        \
                   : (same ? k_bulk<T, X, Y, true, false, true> : k_bulk<T, X, Y, false, false, true>))    \
            : (src ? (same ? k_bulk<T, X, Y, true, true, false> : k_bulk<T, X, Y, false, true, false>)      \
                   : (same ? k_bulk<T, X, Y, true, false, false> : k_bulk<T, X, Y, false, false, false>)); \
        if (lds > 64 * 1024)                                                                  \
            EBS_HIP(cx, hipFuncSetAttribute((const void*)kf,                                   \
                                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)); \
        const dim3 grid(blocks_per_xcd((const void*)kf) * NXCD);                              \
        hipLaunchKernelGGL(kf, grid, blk, lds, bs, a);                                        \
    } else
            EBS_BULK_CASE(16, 4) EBS_BULK_CASE(16, 8) EBS_BULK_CASE(16, 16) EBS_BULK_CASE(32, 4)
            EBS_BULK_CASE(32, 8) EBS_BULK_CASE(32, 16) EBS_BULK_CASE(64, 2) EBS_BULK_CASE(64, 4)
            EBS_BULK_CASE(64, 8) EBS_BULK_CASE(64, 16) {
                cx->err = "tile shape without a compiled kernel";
                return EBS_E_UNSUPPORTED;
            }
#undef EBS_BULK_CASE
            EBS_HIP(cx, hipGetLastError());
        }
        if (cx->timing) EBS_HIP(cx, hipEventRecord(e1, bs));
    }
    return EBS_OK;
}

}  // namespace

// ------------------------------------------------------------- host side
size_t bulk_lds_bytes(int tx, int ty, int precision, bool sources) {
    const size_t es = precision == EBS_F32_BULK ? 4 : 8;
    return es * ((size_t)L_COUNT * (tx + 5) * (ty + 5) + (sources ? (size_t)2 * (tx + 1) * (ty + 1) : 0));
}

ebs_status build_tiles(ebs_ctx* cx) {
    cx->h_tiles.clear();
    const int TX = cx->tile_x, TY = cx->tile_y, TZ = cx->tile_z;
    const ebs_box whole = {{0, 0, 0}, {cx->nx, cx->ny, cx->nz}};
    const std::vector<ebs_box> spans(1, whole);
    for (const ebs_box& b : cx->tile_span ? spans : cx->boxes) {
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
    // Order: y slab (one per XCD), z band, then row-major.  The launch hands
    // each XCD a contiguous run of this list, so the blocks resident on one
    // XCD cover whole rows of tiles at similar heights: neighbouring tiles
    // share their halo cache lines in that XCD's L2, and in x (periodic) no
    // halo line is fetched by two XCDs.
    std::stable_sort(cx->h_tiles.begin(), cx->h_tiles.end(), [&](const ebs_tile& p, const ebs_tile& q) {
        const int sp = (int)((int64_t)p.y0 * NXCD / cx->ny), sq = (int)((int64_t)q.y0 * NXCD / cx->ny);
        if (sp != sq) return sp < sq;
        const int bp = p.z0 / TZ, bq = q.z0 / TZ;
        if (bp != bq) return bp < bq;
        if (p.y0 != q.y0) return p.y0 < q.y0;
        return p.x0 < q.x0;
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

ebs_status launch_bulk(ebs_ctx* cx, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uhat, double cdt,
                       hipStream_t stream) {
    if (cx->g.precision == EBS_F32_BULK) return launch_bulk_t<float>(cx, Un, Ucur, Uhat, cdt, stream);
    return launch_bulk_t<double>(cx, Un, Ucur, Uhat, cdt, stream);
}

}  // namespace ebs
