// Weighted state redistribution on the four instances (Section 5.1 of the
// paper; applied after every stage, Algorithm 1 step 4).
//
// Setup (once per geometry): small flags, merge neighbourhoods M (first along
// the EB normal, then the next largest normal component completing a 2x2x1
// block, then the 2x2x2 block, until the neighbourhood volume reaches
// V_target), N = |W|, kappa (Eq. kappa), omega (Eq. omega), neighbourhood
// volume (Eq. nbhd_vol) and centroid.  W is never stored: every kernel that
// needs it gathers over the 26 neighbours and tests their member masks, so no
// atomics are involved and results do not depend on thread order.
//
// Apply (per stage, per field of each instance): Q-hat (Eq. qhat_omega) on
// small CVs, a least-squares gradient of Q-hat with a Barth-Jespersen-style
// limiter, and the final gathered update (Eqs. qrecon, final_update_omega) on
// the CVs the operator can change.  Everything is in double precision and reads
// the double copy of the provisional state kept by the stage kernel.
//
// Readings (the paper is silent or garbled): small <=> 0 < alpha <
// small_vfrac (1 - 1e-12); a tier is accepted once the member volume reaches
// V_target (1 - 1e-12); axes ordered by |n_d| descending with ties (within
// 1e-12 max|n|) to the lower axis, steps along sgn(n_d) (+ for |n_d| within the
// tie tolerance); kappa = min(1, (V_target - V) / sum_{M-} V); N includes the CV's
// own neighbourhood; gradient for small CVs with |M| >= 2 only, unweighted
// least squares anchored at Q-hat_i over the fluid CVs of the 3x3x3 box, a
// direction widened to 5 when the member centroids spread less than half a
// cell along it, zero gradient with < 3 points, too little spread after
// widening, or reciprocal condition number < 1e-10; limiter factor per
// component from the values of the reconstruction at the centroids of M_i.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "ebs_internal.h"
#include "xcd.h"

namespace ebs {
namespace {

__device__ inline int bit_of(int ox, int oy, int oz) { return (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1); }
constexpr int32_t SELF_BIT = 1 << 13;

struct WArgs {
    GeoView v;
    int32_t* mask;
    int8_t* small;
    int8_t* tier;
    double* w;      // [4][WQ_COUNT][G]
    double vfrac;   // small_vfrac
    double dv;
    int32_t* bad;   // counts neighbourhood members above the general range
};

__device__ inline double& wq(const WArgs& a, int inst, int q, int g) {
    return a.w[((size_t)inst * WQ_COUNT + q) * a.v.G + g];
}

// general index of a neighbour CV, -1 if it is a regular CV outside the
// general range, -2 if it is not a fluid CV
__device__ inline int nbr(const GeoView& v, int inst, int i, int j, int k) {
    if (!cv_plane(v, inst, k)) return -2;
    i = wrapi(i, v.nx);
    j = wrapi(j, v.ny);
    const int g = gidx(v, i, j, k);
    if (g == -2) return -2;
    if (g == -1) return -1;
    if (v.type[(size_t)inst * v.G + g] == 0) return -2;
    return g;
}

__device__ inline double alpha_of(const GeoView& v, int inst, int g) {
    return g == -1 ? 1.0 : (g < 0 ? 0.0 : gq(v, inst, GQ_ALPHA, g));
}

__device__ inline void cell_of(const GeoView& v, int g, int& i, int& j, int& k) {
    const int c = v.gcol[g];
    const int4 ci = v.col[c];
    i = c % v.nx;
    j = c / v.nx;
    k = col_g0(ci) + (g - ci.z);
}

__global__ void k_merge(WArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= a.v.G) return;
    const GeoView& v = a.v;
    const size_t o = (size_t)inst * v.G + g;
    a.small[o] = 0;
    a.tier[o] = 0;
    if (v.type[o] == 0) { a.mask[o] = 0; return; }
    const double al = gq(v, inst, GQ_ALPHA, g);
    if (!(al < a.vfrac * (1.0 - TIE))) { a.mask[o] = SELF_BIT; return; }
    a.small[o] = 1;
    int i, j, k;
    cell_of(v, g, i, j, k);
    const double n[3] = {gq(v, inst, GQ_AX, g) * v.dy * v.dz, gq(v, inst, GQ_AY, g) * v.dx * v.dz,
                         gq(v, inst, GQ_AZ, g) * v.dx * v.dy};
    const double mx = fmax(fabs(n[0]), fmax(fabs(n[1]), fabs(n[2])));
    const double tol = TIE * mx;
    int order[3];
    bool used[3] = {false, false, false};
    for (int r = 0; r < 3; ++r) {
        double best = -1.0;
        for (int d = 0; d < 3; ++d)
            if (!used[d]) best = fmax(best, fabs(n[d]));
        for (int d = 0; d < 3; ++d)
            if (!used[d] && fabs(n[d]) >= best - tol) { order[r] = d; used[d] = true; break; }
    }
    int sg[3];
    for (int d = 0; d < 3; ++d) sg[d] = (n[d] < -tol) ? -1 : 1;
    int32_t mask = SELF_BIT;
    const double dv = a.dv;
    const double vt = a.vfrac * dv;
    double vsum = al * dv;
    int tier = 0;
    for (int t = 1; t <= 3; ++t) {
        tier = t;
        for (int p = 0; p <= (t >= 1); ++p)
            for (int q = 0; q <= (t >= 2); ++q)
                for (int e = 0; e <= (t >= 3); ++e) {
                    int off[3] = {0, 0, 0};
                    off[order[0]] += p * sg[order[0]];
                    off[order[1]] += q * sg[order[1]];
                    off[order[2]] += e * sg[order[2]];
                    const int bt = bit_of(off[0], off[1], off[2]);
                    if ((mask >> bt) & 1) continue;
                    const int gn = nbr(v, inst, i + off[0], j + off[1], k + off[2]);
                    if (gn == -2) continue;
                    // members must lie in the general range (its top covers the
                    // footprint of every small CV); checked, not assumed
                    if (gn == -1) atomicAdd(a.bad, 1);
                    mask |= 1 << bt;
                    vsum += alpha_of(v, inst, gn) * dv;
                }
        if (vsum >= vt * (1.0 - TIE)) break;
    }
    a.mask[o] = mask;
    a.tier[o] = (int8_t)tier;
}

__device__ inline int32_t mask_of(const WArgs& a, int inst, int g) {
    return g == -1 ? SELF_BIT : (g < 0 ? 0 : a.mask[(size_t)inst * a.v.G + g]);
}

__global__ void k_count(WArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= a.v.G) return;
    const GeoView& v = a.v;
    if (v.type[(size_t)inst * v.G + g] == 0) { wq(a, inst, WQ_N, g) = 0.0; return; }
    int i, j, k;
    cell_of(v, g, i, j, k);
    int cnt = 0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                const int gr = nbr(v, inst, i - ox, j - oy, k - oz);
                if (gr == -2) continue;
                if ((mask_of(a, inst, gr) >> bit_of(ox, oy, oz)) & 1) ++cnt;
            }
    wq(a, inst, WQ_N, g) = (double)cnt;
}

__global__ void k_kappa(WArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= a.v.G) return;
    const GeoView& v = a.v;
    double kap = 0.0;
    const size_t o = (size_t)inst * v.G + g;
    if (a.small[o]) {
        int i, j, k;
        cell_of(v, g, i, j, k);
        const double dv = a.dv, vt = a.vfrac * dv;
        const double V = gq(v, inst, GQ_ALPHA, g) * dv;
        const int32_t m = a.mask[o];
        double s = 0.0;
        for (int oz = -1; oz <= 1; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    if (ox == 0 && oy == 0 && oz == 0) continue;
                    if (!((m >> bit_of(ox, oy, oz)) & 1)) continue;
                    s += alpha_of(v, inst, nbr(v, inst, i + ox, j + oy, k + oz)) * dv;
                }
        if (V < vt && s > 0.0) kap = fmin(1.0, (vt - V) / s);
    }
    wq(a, inst, WQ_KAPPA, g) = kap;
}

__global__ void k_omega(WArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= a.v.G) return;
    const GeoView& v = a.v;
    if (v.type[(size_t)inst * v.G + g] == 0) { wq(a, inst, WQ_OMEGA, g) = 0.0; return; }
    int i, j, k;
    cell_of(v, g, i, j, k);
    double ks = 0.0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                const int gr = nbr(v, inst, i - ox, j - oy, k - oz);
                if (gr < 0) continue;  // regular CVs outside the range have kappa 0
                if ((a.mask[(size_t)inst * v.G + gr] >> bit_of(ox, oy, oz)) & 1)
                    ks += wq(a, inst, WQ_KAPPA, gr);
            }
    wq(a, inst, WQ_OMEGA, g) = 1.0 - ks / wq(a, inst, WQ_N, g);
}

__global__ void k_vhat(WArgs a) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const int inst = blockIdx.y;
    if (g >= a.v.G) return;
    const GeoView& v = a.v;
    if (v.type[(size_t)inst * v.G + g] == 0) {
        for (int q = WQ_VHAT; q <= WQ_XHZ; ++q) wq(a, inst, q, g) = 0.0;
        return;
    }
    int i, j, k;
    cell_of(v, g, i, j, k);
    const double dv = a.dv;
    const double V = gq(v, inst, GQ_ALPHA, g) * dv;
    const double om = wq(a, inst, WQ_OMEGA, g);
    const double kap = wq(a, inst, WQ_KAPPA, g);
    const int32_t m = a.mask[(size_t)inst * v.G + g];
    double vh = om * V;
    double xs[3];
    for (int d = 0; d < 3; ++d) xs[d] = om * V * gq(v, inst, GQ_VCX + d, g);
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                if (!((m >> bit_of(ox, oy, oz)) & 1)) continue;
                const int gr = nbr(v, inst, i + ox, j + oy, k + oz);
                const double Vr = alpha_of(v, inst, gr) * dv;
                const double Nr = gr >= 0 ? wq(a, inst, WQ_N, gr) : 1.0;
                const int off[3] = {ox, oy, oz};
                vh += kap * Vr / Nr;
                for (int d = 0; d < 3; ++d)
                    xs[d] += kap * Vr / Nr * (off[d] + (gr >= 0 ? gq(v, inst, GQ_VCX + d, gr) : 0.0));
            }
    wq(a, inst, WQ_VHAT, g) = vh / dv;
    for (int d = 0; d < 3; ++d) wq(a, inst, WQ_XHX + d, g) = xs[d] / vh;
}

// ------------------------------------------------------------------ apply
// Each field belongs to one instance: rho and rho theta to the cell-centred
// CVs, rho u / rho v / rho w to the x-, y-, z-face CVs.
__device__ inline int field_inst(int f) { return f < 2 ? 0 : f - 1; }
__device__ inline int inst_f0(int inst) { return inst == 0 ? 0 : inst + 1; }
__device__ inline int inst_nf(int inst) { return inst == 0 ? 2 : 1; }

constexpr uint32_t LSQ_QHAT = 0x80000000u;  // fit point whose Q-hat differs from U-hat
constexpr int LSQ_MAXEV = 8;                // members of a 2x2x2 neighbourhood

struct AArgs {
    GeoView v;
    const int32_t* mask;
    const int8_t* small;
    const double* w;
    const double* uhat;   // [5][G]
    double* qhat;         // [5][G]
    double* sig;          // [5][3][G]
    const int32_t* slist; // [4][G] small CVs with kappa > 0 (per instance)
    const int32_t* alist; // [4][G] CVs the operator may change
    int32_t ns[NINST], na[NINST];
    int32_t sbase[NINST]; // offset of each instance in the concatenated small list
    const int32_t* loff;  // [S+1] least-squares operators (CSR)
    const uint32_t* lidx; // [P]
    const double* lc;     // [3][P]
    int64_t npts;         // P
    const double* lev;    // [S][LSQ_MAXEV][3]
    const int8_t* lnev;   // [S]
    int32_t abase[NINST]; // offset of each instance in the concatenated active list
    const int32_t* woff;  // [A+1] contributors (neighbourhoods containing the CV), CSR
    const int32_t* widx;  // [E] general index of the contributing small CV r
    const double* wgeo;   // [E][4] kappa_r, then (offset + centroid_i - xhat_r) in mesh units
    const double* aself;  // [A][5] omega, N, centroid_i - xhat_i (mesh units; small CVs)
    const int8_t* asmall; // [A] 1 if the CV is small with kappa > 0
    const int32_t* qidx;  // [S][LSQ_MAXEV] Q-hat operator: the CV, then its members
    const double* qw;     // [S][LSQ_MAXEV] weights: omega V, then kappa alpha_r V / N_r
    const double* qden;   // [S] V-hat
    const int8_t* qn;     // [S] entries used
    int limiter;
    double dv;
};

__device__ inline double wv(const AArgs& a, int inst, int q, int g) {
    return a.w[((size_t)inst * WQ_COUNT + q) * a.v.G + g];
}

// Q-hat operator of the small CVs with kappa > 0 (Eq. qhat_omega), built once
// per geometry: Q-hat_i = (omega_i V_i U_i + sum over the members r of
// kappa_i alpha_r V / N_r U_r) / V-hat_i, members in the order of the offsets
// (dz, dy, dx) from -1 to 1.  Every member lies in the general range: its
// margin exceeds the merge radius.
__global__ void __launch_bounds__(128) k_qtab(AArgs a, int32_t* qidx, double* qw, double* qden, int8_t* qn) {
    const int inst = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.ns[inst]) return;
    const int g = a.slist[(size_t)inst * a.v.G + t];
    const size_t e = (size_t)a.sbase[inst] + t;
    const GeoView& v = a.v;
    int i, j, k;
    cell_of(v, g, i, j, k);
    const double V = gq(v, inst, GQ_ALPHA, g) * a.dv;
    const double om = wv(a, inst, WQ_OMEGA, g), kap = wv(a, inst, WQ_KAPPA, g);
    const int32_t m = a.mask[(size_t)inst * v.G + g];
    int32_t* id = qidx + e * LSQ_MAXEV;
    double* w = qw + e * LSQ_MAXEV;
    id[0] = g;
    w[0] = om * V;
    int n = 1;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                if (!((m >> bit_of(ox, oy, oz)) & 1)) continue;
                const int gr = nbr(v, inst, i + ox, j + oy, k + oz);
                if (gr < 0 || n >= LSQ_MAXEV) continue;
                id[n] = gr;
                w[n] = kap * gq(v, inst, GQ_ALPHA, gr) * a.dv / wv(a, inst, WQ_N, gr);
                ++n;
            }
    for (int q = n; q < LSQ_MAXEV; ++q) {
        id[q] = g;
        w[q] = 0.0;
    }
    qn[e] = (int8_t)n;
    qden[e] = wv(a, inst, WQ_VHAT, g) * a.dv;
}

// Q-hat of the small CVs with kappa > 0, from the operator table; all
// instances in one launch (blockIdx.y = instance)
__global__ void __launch_bounds__(128) k_qhat(AArgs a) {
    const int inst = blockIdx.y;
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= a.ns[inst]) return;
    const size_t e = (size_t)a.sbase[inst] + t;
    int32_t id[LSQ_MAXEV];
    double w[LSQ_MAXEV];
#pragma unroll
    for (int q = 0; q < LSQ_MAXEV; ++q) {
        id[q] = a.qidx[e * LSQ_MAXEV + q];
        w[q] = a.qw[e * LSQ_MAXEV + q];
    }
    const int n = a.qn[e];
    const double den = a.qden[e];
    const int f0 = inst_f0(inst), nf = inst_nf(inst);
    for (int f = f0; f < f0 + nf; ++f) {
        const double* U = a.uhat + (size_t)f * a.v.G;
        double s = w[0] * U[id[0]];
#pragma unroll
        for (int q = 1; q < LSQ_MAXEV; ++q)
            if (q < n) s += w[q] * U[id[q]];
        a.qhat[(size_t)f * a.v.G + id[0]] = s / den;
    }
}

__device__ inline double psi(double delta, double qi, double qmin, double qmax) {
    if (delta > 0.0) return fmin(1.0, (qmax - qi) / delta);
    if (delta < 0.0) return fmin(1.0, (qmin - qi) / delta);
    return 1.0;
}

// Limited least-squares gradient of Q-hat, per small CV and field of its
// instance, from the precomputed operator: sigma = sum_s c_s (Q-hat_s - Q-hat_i) with
// c_s = A^-1 e_s, then the Barth-Jespersen-style limiter.  A group of
// GRAD_LANES lanes shares one CV: the lanes split its fit points and combine
// their partial sums and bounds by a butterfly over the group.
constexpr int GRAD_LANES = 8;

// NF fields of one instance (the cell-centred instance carries rho and rho
// theta) share the group's operator loads
template <int NF>
__device__ __forceinline__ void grad_group(const AArgs& a, int inst, int f0, int lane, int t) {
    const bool valid = t < a.ns[inst];
    const GeoView& v = a.v;
    int g = 0, e = 0, p0 = 0, p1 = 0;
    if (valid) {
        g = a.slist[(size_t)inst * v.G + t];
        e = a.sbase[inst] + t;
        p0 = a.loff[e];
        p1 = a.loff[e + 1];
    }
    double qi[NF], s[NF][3], qmin[NF], qmax[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) {
        qi[n] = valid ? a.qhat[(size_t)(f0 + n) * v.G + g] : 0.0;
        s[n][0] = s[n][1] = s[n][2] = 0.0;
        qmin[n] = qmax[n] = qi[n];
    }
    for (int p = p0 + lane; p < p1; p += GRAD_LANES) {
        const uint32_t id = a.lidx[p];
        const double c0 = a.lc[p], c1 = a.lc[a.npts + p], c2 = a.lc[2 * a.npts + p];
#pragma unroll
        for (int n = 0; n < NF; ++n) {
            const size_t fo = (size_t)(f0 + n) * v.G;
            const double qs = (id & LSQ_QHAT) ? a.qhat[fo + (id & ~LSQ_QHAT)] : a.uhat[fo + id];
            const double dq = qs - qi[n];
            s[n][0] += c0 * dq;
            s[n][1] += c1 * dq;
            s[n][2] += c2 * dq;
            qmin[n] = fmin(qmin[n], qs);
            qmax[n] = fmax(qmax[n], qs);
        }
    }
#pragma unroll
    for (int m = GRAD_LANES / 2; m >= 1; m >>= 1)
#pragma unroll
        for (int n = 0; n < NF; ++n) {
            s[n][0] += __shfl_xor(s[n][0], m, GRAD_LANES);
            s[n][1] += __shfl_xor(s[n][1], m, GRAD_LANES);
            s[n][2] += __shfl_xor(s[n][2], m, GRAD_LANES);
            qmin[n] = fmin(qmin[n], __shfl_xor(qmin[n], m, GRAD_LANES));
            qmax[n] = fmax(qmax[n], __shfl_xor(qmax[n], m, GRAD_LANES));
        }
    // limiter: the lanes of the group split the evaluation points (at most
    // LSQ_MAXEV); the factors are combined by a min-butterfly (min is exact,
    // so the result does not depend on the order)
    const bool lim = valid && p1 > p0 && a.limiter != EBS_LIM_NONE;
    double lam[NF][3];
#pragma unroll
    for (int n = 0; n < NF; ++n) lam[n][0] = lam[n][1] = lam[n][2] = 1.0;
    const int nev = lim ? a.lnev[e] : 0;
    for (int q = lane; q < nev; q += GRAD_LANES) {
        const double* ev = a.lev + ((size_t)e * LSQ_MAXEV + q) * 3;
#pragma unroll
        for (int n = 0; n < NF; ++n) {
            if (a.limiter == EBS_LIM_BJ_COMPONENT) {
                for (int d = 0; d < 3; ++d)
                    lam[n][d] = fmin(lam[n][d], psi(s[n][d] * ev[d], qi[n], qmin[n], qmax[n]));
            } else {
                const double l = psi(s[n][0] * ev[0] + s[n][1] * ev[1] + s[n][2] * ev[2], qi[n], qmin[n], qmax[n]);
                for (int d = 0; d < 3; ++d) lam[n][d] = fmin(lam[n][d], l);
            }
        }
    }
#pragma unroll
    for (int m = GRAD_LANES / 2; m >= 1; m >>= 1)
#pragma unroll
        for (int n = 0; n < NF; ++n)
            for (int d = 0; d < 3; ++d) lam[n][d] = fmin(lam[n][d], __shfl_xor(lam[n][d], m, GRAD_LANES));
    if (!valid || lane != 0) return;
    const double del[3] = {v.dx, v.dy, v.dz};
#pragma unroll
    for (int n = 0; n < NF; ++n) {
        if (lim)
            for (int d = 0; d < 3; ++d) s[n][d] *= lam[n][d];
        for (int d = 0; d < 3; ++d) a.sig[((size_t)(f0 + n) * 3 + d) * v.G + g] = s[n][d] / del[d];
    }
}

// one launch for all instances (blockIdx.y = instance)
__global__ void __launch_bounds__(256) k_grad(AArgs a) {
    const int inst = blockIdx.y;
    const int lane = threadIdx.x % GRAD_LANES;
    const int t = xcd_block() * (256 / GRAD_LANES) + threadIdx.x / GRAD_LANES;
    if (inst == 0)
        grad_group<2>(a, 0, 0, lane, t);
    else
        grad_group<1>(a, inst, inst + 1, lane, t);
}

constexpr int FINAL_LANES = 4;

template <typename T>
struct FArgs {
    AArgs a;
    int nx, ny, nz;
    T* out[5];
};

// Final update (Eqs. qrecon, final_update_omega) of the NF fields of one
// instance on the CVs the operator may change, gathered over the precomputed
// list of neighbourhoods containing each CV (W minus itself, fixed order).
template <typename T, int NF>
__device__ __forceinline__ void final_group(const FArgs<T>& F, int inst, int f0, int lane, int t) {
    const AArgs& a = F.a;
    const bool valid = t < a.na[inst];
    const GeoView& v = a.v;
    const int g = valid ? a.alist[(size_t)inst * v.G + t] : 0;
    const int e = valid ? a.abase[inst] + t : 0;
    const double del[3] = {v.dx, v.dy, v.dz};
    double s[NF];
#pragma unroll
    for (int n = 0; n < NF; ++n) s[n] = 0.0;
    const int q1 = valid ? a.woff[e + 1] : 0;
    for (int q = (valid ? a.woff[e] : 0) + lane; q < q1; q += FINAL_LANES) {
        const int gr = a.widx[q];
        const double* w = a.wgeo + (size_t)q * 4;
        const double w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3];
#pragma unroll
        for (int n = 0; n < NF; ++n) {
            const size_t f = f0 + n;
            double qr = a.qhat[f * v.G + gr];
            qr += a.sig[(f * 3 + 0) * v.G + gr] * w1 * del[0];
            qr += a.sig[(f * 3 + 1) * v.G + gr] * w2 * del[1];
            qr += a.sig[(f * 3 + 2) * v.G + gr] * w3 * del[2];
            s[n] += w0 * qr;
        }
    }
#pragma unroll
    for (int m = FINAL_LANES / 2; m >= 1; m >>= 1)
#pragma unroll
        for (int n = 0; n < NF; ++n) s[n] += __shfl_xor(s[n], m, FINAL_LANES);
    if (!valid || lane != 0) return;
    const double* self = a.aself + (size_t)e * 5;
    const double om = self[0], Ni = self[1];
    const bool sm = a.asmall[e];
    // write into the state layout (with the periodic repeat)
    int i, j, k;
    cell_of(v, g, i, j, k);
    const int nx = F.nx, ny = F.ny;
#pragma unroll
    for (int n = 0; n < NF; ++n) {
        const int f = f0 + n;
        double qi;
        if (sm) {
            qi = a.qhat[(size_t)f * v.G + g];
            qi += a.sig[((size_t)f * 3 + 0) * v.G + g] * self[2] * del[0];
            qi += a.sig[((size_t)f * 3 + 1) * v.G + g] * self[3] * del[1];
            qi += a.sig[((size_t)f * 3 + 2) * v.G + g] * self[4] * del[2];
        } else {
            qi = a.uhat[(size_t)f * v.G + g];
        }
        const double val = om * qi + s[n] / Ni;
        size_t idx;
        if (f == 2) idx = ((size_t)k * ny + j) * (nx + 1) + i;
        else if (f == 3) idx = ((size_t)k * (ny + 1) + j) * nx + i;
        else idx = ((size_t)k * ny + j) * nx + i;
        T* o = f == 0 ? F.out[0] : f == 1 ? F.out[1] : f == 2 ? F.out[2] : f == 3 ? F.out[3] : F.out[4];
        o[idx] = (T)val;
        if (f == 2 && i == 0) F.out[2][((size_t)k * ny + j) * (nx + 1) + nx] = (T)val;
        if (f == 3 && j == 0) F.out[3][((size_t)k * (ny + 1) + ny) * nx + i] = (T)val;
    }
}

// FINAL_LANES lanes per CV split its contributors and add their partial sums
// by a butterfly over the group; the fields of one instance share the
// contributor loads (blockIdx.y = instance)
template <typename T>
__global__ void __launch_bounds__(128) k_final(FArgs<T> F) {
    const int inst = blockIdx.y;
    const int lane = threadIdx.x % FINAL_LANES;
    const int t = (xcd_block() * blockDim.x + threadIdx.x) / FINAL_LANES;
    if (inst == 0)
        final_group<T, 2>(F, 0, 0, lane, t);
    else
        final_group<T, 1>(F, inst, inst + 1, lane, t);
}

// Contributor lists of the final update, built once per geometry: for every
// CV the operator may change, the small CVs r whose neighbourhood contains it
// (in the order of the offsets (dz, dy, dx) from -1 to 1), with kappa_r and
// the offset from r's neighbourhood centroid to this CV's centroid.
struct WLArgs {
    GeoView v;
    const int32_t* mask;
    const int8_t* small;
    const double* w;
    const int32_t* alist;  // [4][G]
    int32_t na[NINST], abase[NINST];
    int fill;
    int32_t* cnt;          // count mode: [A]
    const int32_t* off;    // fill mode: [A+1]
    int32_t* idx;
    double* geo4;
    double* self;
    int8_t* smallf;
};

__global__ void __launch_bounds__(128) k_wlist(WLArgs a) {
    const int inst = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.na[inst]) return;
    const GeoView& v = a.v;
    const int g = a.alist[(size_t)inst * v.G + t];
    const int e = a.abase[inst] + t;
    auto W = [&](int q, int gg) { return a.w[((size_t)inst * WQ_COUNT + q) * v.G + gg]; };
    int i, j, k;
    cell_of(v, g, i, j, k);
    const double vc[3] = {gq(v, inst, GQ_VCX, g), gq(v, inst, GQ_VCY, g), gq(v, inst, GQ_VCZ, g)};
    int n = 0;
    int q = a.fill ? a.off[e] : 0;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                const int gr = nbr(v, inst, i - ox, j - oy, k - oz);
                if (gr < 0) continue;
                if (!((a.mask[(size_t)inst * v.G + gr] >> bit_of(ox, oy, oz)) & 1)) continue;
                ++n;
                if (!a.fill) continue;
                const int off[3] = {ox, oy, oz};
                a.idx[q] = gr;
                double* o = a.geo4 + (size_t)q * 4;
                o[0] = W(WQ_KAPPA, gr);
                for (int d = 0; d < 3; ++d) o[1 + d] = off[d] + vc[d] - W(WQ_XHX + d, gr);
                ++q;
            }
    if (!a.fill) {
        a.cnt[e] = n;
        return;
    }
    double* sf = a.self + (size_t)e * 5;
    sf[0] = W(WQ_OMEGA, g);
    sf[1] = W(WQ_N, g);
    for (int d = 0; d < 3; ++d) sf[2 + d] = vc[d] - W(WQ_XHX + d, g);
    a.smallf[e] = (a.small[(size_t)inst * v.G + g] && W(WQ_KAPPA, g) > 0.0) ? 1 : 0;
}

// ------------------------------------------------ least-squares operators
// Built once per geometry for every small CV with kappa > 0: the fit points
// (fluid CVs of the 3x3x3 box, widened to 5 along directions whose centroid
// spread is below half a cell), the normal matrix A = sum e_s e_s^T of the
// centroid offsets e_s (mesh units), its inverse by the adjugate with the
// reciprocal 1-norm condition number test, and c_s = A^-1 e_s.  A zero
// gradient is encoded as an empty point list.  The limiter's evaluation
// offsets (centroids of the members of M_i relative to the neighbourhood
// centroid) are stored beside them.
struct LArgs {
    GeoView v;
    const int32_t* mask;
    const int8_t* small;
    const double* w;
    const int32_t* slist;  // [4][G]
    int32_t ns[NINST], sbase[NINST];
    int fill;              // 0: count points, 1: write them
    int32_t* cnt;          // [S]
    const int32_t* off;    // [S+1]
    uint32_t* idx;
    double* c;             // [3][npts]
    int64_t npts;
    double* ev;
    int8_t* nev;
    int32_t* bad;          // counts fit points above the general range
};

__global__ void __launch_bounds__(64) k_lsq(LArgs a) {
    const int inst = blockIdx.y;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.ns[inst]) return;
    const GeoView& v = a.v;
    const int g = a.slist[(size_t)inst * v.G + t];
    const int e = a.sbase[inst] + t;
    auto W = [&](int q, int gg) { return a.w[((size_t)inst * WQ_COUNT + q) * v.G + gg]; };
    int i, j, k;
    cell_of(v, g, i, j, k);
    const double xh[3] = {W(WQ_XHX, g), W(WQ_XHY, g), W(WQ_XHZ, g)};
    int wd[3] = {1, 1, 1};
    double spread[3];
    int npts = 0;
    for (int pass = 0; pass < 2; ++pass) {
        spread[0] = spread[1] = spread[2] = 0.0;
        npts = 0;
        for (int oz = -wd[2]; oz <= wd[2]; ++oz)
            for (int oy = -wd[1]; oy <= wd[1]; ++oy)
                for (int ox = -wd[0]; ox <= wd[0]; ++ox) {
                    if (ox == 0 && oy == 0 && oz == 0) continue;
                    const int gs = nbr(v, inst, i + ox, j + oy, k + oz);
                    // a fluid CV above the general range would be a missing fit
                    // point: the range's top excludes it, and this checks it
                    if (gs == -1 && !a.fill) atomicAdd(a.bad, 1);
                    if (gs < 0) continue;  // not fluid
                    const int o[3] = {ox, oy, oz};
                    for (int d = 0; d < 3; ++d) spread[d] = fmax(spread[d], fabs(o[d] + W(WQ_XHX + d, gs) - xh[d]));
                    ++npts;
                }
        if (pass == 1) break;
        bool widened = false;
        for (int d = 0; d < 3; ++d)
            if (spread[d] < 0.5 * (1.0 - TIE)) { wd[d] = 2; widened = true; }
        if (!widened) break;
    }
    bool zero = npts < 3;
    for (int d = 0; d < 3; ++d)
        if (spread[d] < 0.5 * (1.0 - TIE)) zero = true;
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    if (!zero) {
        for (int oz = -wd[2]; oz <= wd[2]; ++oz)
            for (int oy = -wd[1]; oy <= wd[1]; ++oy)
                for (int ox = -wd[0]; ox <= wd[0]; ++ox) {
                    if (ox == 0 && oy == 0 && oz == 0) continue;
                    const int gs = nbr(v, inst, i + ox, j + oy, k + oz);
                    if (gs < 0) continue;
                    const double es[3] = {ox + W(WQ_XHX, gs) - xh[0], oy + W(WQ_XHY, gs) - xh[1],
                                          oz + W(WQ_XHZ, gs) - xh[2]};
                    for (int r = 0; r < 3; ++r)
                        for (int q = 0; q < 3; ++q) A[r][q] += es[r] * es[q];
                }
    }
    double inv[3][3];
    if (!zero) {
        const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
        const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
        const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
        if (!(fabs(det) > 0.0)) {
            zero = true;
        } else {
            const double id = 1.0 / det;
            inv[0][0] = c00 * id;
            inv[1][0] = c01 * id;
            inv[2][0] = c02 * id;
            inv[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
            inv[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
            inv[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
            inv[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
            inv[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
            inv[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
            double n1 = 0.0, ni = 0.0;
            for (int q = 0; q < 3; ++q) {
                n1 = fmax(n1, fabs(A[0][q]) + fabs(A[1][q]) + fabs(A[2][q]));
                ni = fmax(ni, fabs(inv[0][q]) + fabs(inv[1][q]) + fabs(inv[2][q]));
            }
            if (!(1.0 / (n1 * ni) >= 1e-10)) zero = true;
        }
    }
    if (!a.fill) {
        a.cnt[e] = zero ? 0 : npts;
        return;
    }
    if (zero) {
        a.nev[e] = 0;
        return;
    }
    int p = a.off[e];
    for (int oz = -wd[2]; oz <= wd[2]; ++oz)
        for (int oy = -wd[1]; oy <= wd[1]; ++oy)
            for (int ox = -wd[0]; ox <= wd[0]; ++ox) {
                if (ox == 0 && oy == 0 && oz == 0) continue;
                const int gs = nbr(v, inst, i + ox, j + oy, k + oz);
                if (gs < 0) continue;
                const double es[3] = {ox + W(WQ_XHX, gs) - xh[0], oy + W(WQ_XHY, gs) - xh[1],
                                      oz + W(WQ_XHZ, gs) - xh[2]};
                const bool own = a.small[(size_t)inst * v.G + gs] && W(WQ_KAPPA, gs) > 0.0;
                a.idx[p] = (uint32_t)gs | (own ? LSQ_QHAT : 0u);
                for (int r = 0; r < 3; ++r)
                    a.c[r * a.npts + p] = inv[r][0] * es[0] + inv[r][1] * es[1] + inv[r][2] * es[2];
                ++p;
            }
    const int32_t m = a.mask[(size_t)inst * v.G + g];
    int n = 0;
    double* evo = a.ev + (size_t)e * LSQ_MAXEV * 3;
    for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                if (!((m >> bit_of(ox, oy, oz)) & 1) || n >= LSQ_MAXEV) continue;
                const int gj = nbr(v, inst, i + ox, j + oy, k + oz);
                const int o[3] = {ox, oy, oz};
                for (int d = 0; d < 3; ++d)
                    evo[3 * n + d] = o[d] + (gj >= 0 ? gq(v, inst, GQ_VCX + d, gj) : 0.0) - xh[d];
                ++n;
            }
    a.nev[e] = (int8_t)n;
}

}  // namespace

WsrdView wsrd_view(const ebs_ctx* c) {
    WsrdView w;
    w.mask = c->d_mask;
    w.small = c->d_small;
    w.tier = c->d_tier;
    w.w = c->d_w;
    w.limiter = c->g.limiter;
    w.vt = c->g.small_vfrac;
    return w;
}

ebs_status wsrd_setup(ebs_ctx* cx) {
    if (cx->G == 0) return EBS_OK;
    if (!cx->d_chk && hipMalloc(&cx->d_chk, sizeof(int32_t)) != hipSuccess) {
        cx->err = "device allocation of the redistribution tables failed";
        return EBS_E_OOM;
    }
    EBS_HIP(cx, hipMemsetAsync(cx->d_chk, 0, sizeof(int32_t), cx->stream));
    WArgs a;
    a.v = geo_view(cx);
    a.mask = cx->d_mask;
    a.small = cx->d_small;
    a.tier = cx->d_tier;
    a.w = cx->d_w;
    a.vfrac = cx->g.small_vfrac;
    a.dv = cx->g.dx[0] * cx->g.dx[1] * cx->g.dx[2];
    a.bad = cx->d_chk;
    const dim3 grid((cx->G + 127) / 128, NINST), blk(128);
    hipLaunchKernelGGL(k_merge, grid, blk, 0, cx->stream, a);
    hipLaunchKernelGGL(k_count, grid, blk, 0, cx->stream, a);
    hipLaunchKernelGGL(k_kappa, grid, blk, 0, cx->stream, a);
    hipLaunchKernelGGL(k_omega, grid, blk, 0, cx->stream, a);
    hipLaunchKernelGGL(k_vhat, grid, blk, 0, cx->stream, a);
    EBS_HIP(cx, hipGetLastError());
    // work lists: small CVs with kappa > 0, and every CV the operator may change
    const size_t G = cx->G;
    std::vector<int8_t> small(NINST * G);
    std::vector<double> w((size_t)NINST * WQ_COUNT * G);
    EBS_HIP(cx, hipMemcpyAsync(small.data(), cx->d_small, NINST * G, hipMemcpyDeviceToHost, cx->stream));
    EBS_HIP(cx, hipMemcpyAsync(w.data(), cx->d_w, sizeof(double) * NINST * WQ_COUNT * G,
                               hipMemcpyDeviceToHost, cx->stream));
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    std::vector<int32_t> sl, al;
    for (int inst = 0; inst < NINST; ++inst) {
        sl.clear();
        al.clear();
        const double* N = &w[((size_t)inst * WQ_COUNT + WQ_N) * G];
        const double* K = &w[((size_t)inst * WQ_COUNT + WQ_KAPPA) * G];
        for (size_t g = 0; g < G; ++g) {
            const bool sm = small[inst * G + g] && K[g] > 0.0;
            if (sm) sl.push_back((int32_t)g);
            if (sm || N[g] > 1.0) al.push_back((int32_t)g);
        }
        cx->nsmall[inst] = (int32_t)sl.size();
        cx->nact[inst] = (int32_t)al.size();
        if (!sl.empty())
            EBS_HIP(cx, hipMemcpy(cx->d_smalllist + inst * G, sl.data(), sizeof(int32_t) * sl.size(),
                                  hipMemcpyHostToDevice));
        if (!al.empty())
            EBS_HIP(cx, hipMemcpy(cx->d_actlist + inst * G, al.data(), sizeof(int32_t) * al.size(),
                                  hipMemcpyHostToDevice));
    }
    // least-squares operators of the small CVs: count, prefix sum, fill
    int32_t S = 0, nsmax = 0;
    for (int inst = 0; inst < NINST; ++inst) {
        cx->sbase[inst] = S;
        S += cx->nsmall[inst];
        nsmax = std::max(nsmax, cx->nsmall[inst]);
    }
    cx->nlsq = S;
    auto alloc = [&](void** p, size_t bytes) -> bool {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
        return hipMalloc(p, bytes) == hipSuccess;
    };
    bool ok = alloc((void**)&cx->d_lsq_off, sizeof(int32_t) * (S + 1));
    ok &= alloc((void**)&cx->d_lsq_ev, sizeof(double) * 3 * LSQ_MAXEV * std::max(S, 1));
    ok &= alloc((void**)&cx->d_lsq_nev, std::max(S, 1));
    ok &= alloc((void**)&cx->d_q_idx, sizeof(int32_t) * LSQ_MAXEV * std::max(S, 1));
    ok &= alloc((void**)&cx->d_q_w, sizeof(double) * LSQ_MAXEV * std::max(S, 1));
    ok &= alloc((void**)&cx->d_q_den, sizeof(double) * std::max(S, 1));
    ok &= alloc((void**)&cx->d_q_n, std::max(S, 1));
    if (!ok) {
        cx->err = "device allocation of the least-squares tables failed";
        return EBS_E_OOM;
    }
    // Q-hat operators
    if (S > 0) {
        AArgs q{};
        q.v = geo_view(cx);
        q.mask = cx->d_mask;
        q.small = cx->d_small;
        q.w = cx->d_w;
        q.slist = cx->d_smalllist;
        for (int inst = 0; inst < NINST; ++inst) {
            q.ns[inst] = cx->nsmall[inst];
            q.sbase[inst] = cx->sbase[inst];
        }
        q.dv = cx->g.dx[0] * cx->g.dx[1] * cx->g.dx[2];
        hipLaunchKernelGGL(k_qtab, dim3((nsmax + 127) / 128, NINST), dim3(128), 0, cx->stream, q, cx->d_q_idx,
                           cx->d_q_w, cx->d_q_den, cx->d_q_n);
        EBS_HIP(cx, hipGetLastError());
    }
    LArgs L;
    L.bad = cx->d_chk;
    L.v = geo_view(cx);
    L.mask = cx->d_mask;
    L.small = cx->d_small;
    L.w = cx->d_w;
    L.slist = cx->d_smalllist;
    for (int inst = 0; inst < NINST; ++inst) {
        L.ns[inst] = cx->nsmall[inst];
        L.sbase[inst] = cx->sbase[inst];
    }
    L.fill = 0;
    L.cnt = cx->d_lsq_off;  // counts first, replaced by the offsets below
    L.off = nullptr;
    L.idx = nullptr;
    L.c = nullptr;
    L.ev = nullptr;
    L.nev = nullptr;
    const dim3 lgrid((std::max(nsmax, 1) + 63) / 64, NINST);
    if (S > 0) {
        hipLaunchKernelGGL(k_lsq, lgrid, dim3(64), 0, cx->stream, L);
        EBS_HIP(cx, hipGetLastError());
    }
    std::vector<int32_t> off(S + 1, 0);
    if (S > 0)
        EBS_HIP(cx, hipMemcpyAsync(off.data(), cx->d_lsq_off, sizeof(int32_t) * S, hipMemcpyDeviceToHost,
                                   cx->stream));
    int32_t outside = 0;
    EBS_HIP(cx, hipMemcpyAsync(&outside, cx->d_chk, sizeof(int32_t), hipMemcpyDeviceToHost, cx->stream));
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    if (outside != 0) {
        cx->err = "a redistribution neighbourhood member or fit point lies above the general range";
        return EBS_E_UNSUPPORTED;
    }
    int64_t P = 0;
    for (int32_t e = 0; e < S; ++e) {
        const int32_t n = off[e];
        off[e] = (int32_t)P;
        P += n;
    }
    if (P > INT32_MAX / 4) {
        cx->err = "least-squares tables too large";
        return EBS_E_UNSUPPORTED;
    }
    off[S] = (int32_t)P;
    cx->nlsq_pts = P;
    ok = alloc((void**)&cx->d_lsq_idx, sizeof(uint32_t) * std::max<int64_t>(P, 1));
    ok &= alloc((void**)&cx->d_lsq_c, sizeof(double) * 3 * std::max<int64_t>(P, 1));
    if (!ok) {
        cx->err = "device allocation of the least-squares tables failed";
        return EBS_E_OOM;
    }
    EBS_HIP(cx, hipMemcpyAsync(cx->d_lsq_off, off.data(), sizeof(int32_t) * (S + 1), hipMemcpyHostToDevice,
                               cx->stream));
    if (S > 0) {
        L.fill = 1;
        L.cnt = nullptr;
        L.off = cx->d_lsq_off;
        L.idx = cx->d_lsq_idx;
        L.c = cx->d_lsq_c;
        L.npts = P;
        L.ev = cx->d_lsq_ev;
        L.nev = cx->d_lsq_nev;
        hipLaunchKernelGGL(k_lsq, lgrid, dim3(64), 0, cx->stream, L);
        EBS_HIP(cx, hipGetLastError());
    }
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    // contributor lists of the final update: count, prefix sum, fill
    int32_t A = 0, namax = 0;
    for (int inst = 0; inst < NINST; ++inst) {
        cx->abase[inst] = A;
        A += cx->nact[inst];
        namax = std::max(namax, cx->nact[inst]);
    }
    ok = alloc((void**)&cx->d_wl_off, sizeof(int32_t) * (A + 1));
    ok &= alloc((void**)&cx->d_wl_self, sizeof(double) * 5 * std::max(A, 1));
    ok &= alloc((void**)&cx->d_wl_small, std::max(A, 1));
    if (!ok) {
        cx->err = "device allocation of the redistribution lists failed";
        return EBS_E_OOM;
    }
    WLArgs wl;
    wl.v = geo_view(cx);
    wl.mask = cx->d_mask;
    wl.small = cx->d_small;
    wl.w = cx->d_w;
    wl.alist = cx->d_actlist;
    for (int inst = 0; inst < NINST; ++inst) {
        wl.na[inst] = cx->nact[inst];
        wl.abase[inst] = cx->abase[inst];
    }
    wl.fill = 0;
    wl.cnt = cx->d_wl_off;
    wl.off = nullptr;
    wl.idx = nullptr;
    wl.geo4 = nullptr;
    wl.self = nullptr;
    wl.smallf = nullptr;
    const dim3 wgrid((std::max(namax, 1) + 127) / 128, NINST);
    if (A > 0) {
        hipLaunchKernelGGL(k_wlist, wgrid, dim3(128), 0, cx->stream, wl);
        EBS_HIP(cx, hipGetLastError());
    }
    std::vector<int32_t> woff(A + 1, 0);
    if (A > 0)
        EBS_HIP(cx, hipMemcpyAsync(woff.data(), cx->d_wl_off, sizeof(int32_t) * A, hipMemcpyDeviceToHost,
                                   cx->stream));
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    int64_t E = 0;
    for (int32_t e = 0; e < A; ++e) {
        const int32_t n = woff[e];
        woff[e] = (int32_t)E;
        E += n;
    }
    if (E > INT32_MAX / 4) {
        cx->err = "redistribution lists too large";
        return EBS_E_UNSUPPORTED;
    }
    woff[A] = (int32_t)E;
    ok = alloc((void**)&cx->d_wl_idx, sizeof(int32_t) * std::max<int64_t>(E, 1));
    ok &= alloc((void**)&cx->d_wl_geo, sizeof(double) * 4 * std::max<int64_t>(E, 1));
    if (!ok) {
        cx->err = "device allocation of the redistribution lists failed";
        return EBS_E_OOM;
    }
    EBS_HIP(cx, hipMemcpyAsync(cx->d_wl_off, woff.data(), sizeof(int32_t) * (A + 1), hipMemcpyHostToDevice,
                               cx->stream));
    if (A > 0) {
        wl.fill = 1;
        wl.cnt = nullptr;
        wl.off = cx->d_wl_off;
        wl.idx = cx->d_wl_idx;
        wl.geo4 = cx->d_wl_geo;
        wl.self = cx->d_wl_self;
        wl.smallf = cx->d_wl_small;
        hipLaunchKernelGGL(k_wlist, wgrid, dim3(128), 0, cx->stream, wl);
        EBS_HIP(cx, hipGetLastError());
    }
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    return EBS_OK;
}

namespace {

// the level of general cell g raised into its column's footprint top
__device__ inline void raise_top(const GeoView& v, int g, int32_t* ftop) {
    const int c = v.gcol[g];
    atomicMax(&ftop[c], col_g0(v.col[c]) + (g - v.col[c].z));
}

// every CV the redistribution writes (active lists) or reads beyond them
// (least-squares fit points)
__global__ void __launch_bounds__(256) k_tops(GeoView v, const int32_t* alist, int32_t na0, int32_t na1,
                                              int32_t na2, int32_t na3, const uint32_t* lidx, int64_t npts,
                                              int32_t* ftop) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t na[4] = {na0, na1, na2, na3};
    int64_t r = t;
    for (int inst = 0; inst < NINST; ++inst) {
        if (r < na[inst]) {
            raise_top(v, alist[(size_t)inst * v.G + r], ftop);
            return;
        }
        r -= na[inst];
    }
    if (r < npts) raise_top(v, (int)(lidx[r] & ~LSQ_QHAT), ftop);
}

}  // namespace

ebs_status redistribution_tops(ebs_ctx* cx, std::vector<int32_t>& ftop) {
    ftop.assign(cx->ncol, -1);
    if (cx->G == 0) return EBS_OK;
    int32_t* d = nullptr;
    if (hipMalloc(&d, sizeof(int32_t) * cx->ncol) != hipSuccess) {
        cx->err = "device allocation of the redistribution footprint failed";
        return EBS_E_OOM;
    }
    int64_t n = cx->nlsq_pts;
    for (int inst = 0; inst < NINST; ++inst) n += cx->nact[inst];
    hipError_t e = hipMemsetAsync(d, 0xFF, sizeof(int32_t) * cx->ncol, cx->stream);
    if (e == hipSuccess && n > 0) {
        hipLaunchKernelGGL(k_tops, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, cx->stream, geo_view(cx),
                           cx->d_actlist, cx->nact[0], cx->nact[1], cx->nact[2], cx->nact[3], cx->d_lsq_idx,
                           cx->nlsq_pts, d);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(ftop.data(), d, sizeof(int32_t) * cx->ncol, hipMemcpyDeviceToHost, cx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(cx->stream);
    (void)hipFree(d);
    if (e != hipSuccess) {
        cx->err = std::string("redistribution footprint: ") + hipGetErrorString(e);
        return EBS_E_HIP;
    }
    return EBS_OK;
}

template <typename T>
static ebs_status redistribute_t(ebs_ctx* cx, ebs_state* Uout) {
    void* const ou[5] = {Uout->rho, Uout->rhotheta, Uout->rhou, Uout->rhov, Uout->rhow};
    AArgs a;
    a.v = geo_view(cx);
    a.mask = cx->d_mask;
    a.small = cx->d_small;
    a.w = cx->d_w;
    a.uhat = cx->d_uhat;
    a.qhat = cx->d_qhat;
    a.sig = cx->d_sig;
    a.slist = cx->d_smalllist;
    a.alist = cx->d_actlist;
    int nsmax = 0, namax = 0;
    for (int inst = 0; inst < NINST; ++inst) {
        a.ns[inst] = cx->nsmall[inst];
        a.na[inst] = cx->nact[inst];
        a.sbase[inst] = cx->sbase[inst];
        nsmax = std::max(nsmax, cx->nsmall[inst]);
        namax = std::max(namax, cx->nact[inst]);
    }
    a.loff = cx->d_lsq_off;
    a.lidx = cx->d_lsq_idx;
    a.lc = cx->d_lsq_c;
    a.npts = cx->nlsq_pts;
    a.lev = cx->d_lsq_ev;
    a.lnev = cx->d_lsq_nev;
    for (int inst = 0; inst < NINST; ++inst) a.abase[inst] = cx->abase[inst];
    a.woff = cx->d_wl_off;
    a.widx = cx->d_wl_idx;
    a.wgeo = cx->d_wl_geo;
    a.aself = cx->d_wl_self;
    a.asmall = cx->d_wl_small;
    a.qidx = cx->d_q_idx;
    a.qw = cx->d_q_w;
    a.qden = cx->d_q_den;
    a.qn = cx->d_q_n;
    a.limiter = cx->g.limiter;
    a.dv = cx->g.dx[0] * cx->g.dx[1] * cx->g.dx[2];
    if (nsmax > 0) {
        // x extents from xcd_grid: each XCD takes a contiguous chunk of every
        // instance's list (xcd.h)
        hipLaunchKernelGGL(k_qhat, dim3(xcd_grid((nsmax + 127) / 128), NINST), dim3(128), 0, cx->stream, a);
        const int per = 256 / GRAD_LANES;
        hipLaunchKernelGGL(k_grad, dim3(xcd_grid((nsmax + per - 1) / per), NINST), dim3(256), 0, cx->stream, a);
    }
    if (namax > 0) {
        FArgs<T> F;
        F.a = a;
        F.nx = cx->nx;
        F.ny = cx->ny;
        F.nz = cx->nz;
        for (int f = 0; f < 5; ++f) F.out[f] = (T*)ou[f];
        hipLaunchKernelGGL(k_final<T>, dim3(xcd_grid(((long long)namax * FINAL_LANES + 127) / 128), NINST), dim3(128),
                           0, cx->stream, F);
    }
    EBS_HIP(cx, hipGetLastError());
    return EBS_OK;
}

ebs_status launch_redistribute(ebs_ctx* cx, const ebs_state* Uhat, ebs_state* Uout) {
    // copy the provisional state where R is the identity when the output is separate
    void* const in[5] = {Uhat->rho, Uhat->rhotheta, Uhat->rhou, Uhat->rhov, Uhat->rhow};
    void* const ou[5] = {Uout->rho, Uout->rhotheta, Uout->rhou, Uout->rhov, Uout->rhow};
    const size_t es = cx->g.precision == EBS_F32_BULK ? 4 : 8;
    const size_t nx = cx->nx, ny = cx->ny, nz = cx->nz;
    const size_t cnt[5] = {nx * ny * nz, nx * ny * nz, (nx + 1) * ny * nz, nx * (ny + 1) * nz,
                           nx * ny * (nz + 1)};
    for (int f = 0; f < 5; ++f)
        if (in[f] != ou[f])
            EBS_HIP(cx, hipMemcpyAsync(ou[f], in[f], es * cnt[f], hipMemcpyDeviceToDevice, cx->stream));
    if (cx->G == 0) return EBS_OK;
    if (cx->g.precision == EBS_F32_BULK) return redistribute_t<float>(cx, Uout);
    return redistribute_t<double>(cx, Uout);
}

}  // namespace ebs
