// Momentum diffusion (Sections 2.1 and 4.2): the diffusive flux of momentum
// is the viscous stress tau = lambda (div u) I + mu (grad u + grad u^T),
// lambda = -2/3 mu (the sign of Stokes' hypothesis; the paper prints 2/3
// mu).  On the staggered grid the c-momentum CV has its faces normal to c at
// cell centres (tau_cc) and its other faces at cell edges (tau_cd); velocity
// = momentum over the mean density of the fluid cells beside its face.
//
// Full faces (area fraction >= 1 - 1e-12) take the centred differences of
// the staggered grid; a cut face takes the stress from gradients fitted at
// its centroid, each velocity component over the fluid CVs of its own grid,
// 3 CVs along an axis on which the face centre lines up with that grid's CV
// centres and 4 (two on each side) otherwise; the EB is stress-free or
// no-slip (the fits at the facet centroid then prescribe zero velocity);
// the domain bottom and top are stress-free for the u and v CVs, the w CVs
// ending at the first and last cell centres feel tau_zz there with w = 0 on
// the walls.  The fit is the thermal diffusion's (quadratic, linear
// fallback, reciprocal condition number >= 1e-7).
//
// The fitted stresses are fixed linear combinations of velocities at fixed
// CVs, so their weights are built once; the velocities are those the
// advected-quantity pass of the stage computed for the general range and
// the positions above it.  Per stage:
//   k_visc_ops  a group of lanes per operator (cut face or facet of a CV):
//               its stress or facet term;
//   k_visc_gen  one thread per general cell and momentum: divergence over the
//               six faces (full faces by centred differences) and the facet,
//               added to the provisional momentum (FP64 copy and state).
// The cells above the general range, whose momentum CVs have only full
// faces, are updated with the thermal diffusion in one pass (regdiff.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ebs_internal.h"
#include "stage_common.h"
#include "xcd.h"

namespace ebs {

// least-squares weights shared with the thermal diffusion (diffusion.hip)
void lsq_weights(int np, const double (*e)[3], bool with_const, const double* del, double (*W)[3]);

namespace {

template <typename T>
struct ViscArgs {
    Dims D;
    GeoView v;
    const T* rho;
    const T* mom[3];
    T* out[3];
    double* uhat;             // [5][G] FP64 provisional state of the general cells
    const double* prim;       // [G + naux][4] advected quantities of the stage (theta, u, v, w)
    const int2* acol;         // [ncol] {first aux position, top of the aux range}
    const int32_t* op_off;    // [nop + 1]
    const uint32_t* op_pt;    // [pts] component << 28 | position of the velocity in prim
    const double* op_w;       // [pts]
    double* flux;             // [nop] stress of a face or facet term of a CV
    const int32_t* vtab;      // [G][3][7] operator of the lower x, y, z, upper x, y, z faces, facet
    int32_t nop;
    double mu, lam, cdt, dv;
    double rdel[3];
};

__device__ __forceinline__ size_t mom_index(const Dims& D, int e, int i, int j, int k) {
    if (e == 0) return ((size_t)k * D.ny + j) * (D.nx + 1) + i;
    if (e == 1) return ((size_t)k * (D.ny + 1) + j) * D.nx + i;
    return ((size_t)k * D.ny + j) * D.nx + i;
}

// area fraction of the lower d-face of the CV (i, j, k) of an instance
__device__ __forceinline__ double beta_at(const GeoView& v, int inst, int d, int i, int j, int k) {
    const int g = gidx(v, i, j, k);
    if (g == -2) return 0.0;
    if (g == -1) return 1.0;
    return gq(v, inst, GQ_BX + d, g);
}

// Velocity component e of the CV (i, j, k): the value the advected-quantity
// pass of the stage computed (momentum over the mean density of the fluid
// cells beside the face, zero where the CV is not fluid) for positions in
// the general or aux range; zero below the range and beyond the walls; the
// plain two-sided formula above the aux range (every CV there is regular).
template <typename T>
__device__ double vel_at(const ViscArgs<T>& a, int e, int i, int j, int k) {
    const int nx = a.D.nx, ny = a.D.ny, nz = a.D.nz;
    if (k < 0 || k >= nz) return 0.0;
    i = wrapi(i, nx);
    j = wrapi(j, ny);
    const int c = j * nx + i;
    const int4 ci = a.v.col[c];
    const int g0 = col_g0(ci), g1 = col_g1(ci);
    if (k < g0) return 0.0;
    if (k < g1) return a.prim[4 * (size_t)(ci.z + (k - g0)) + 1 + e];
    const int2 ac = a.acol[c];
    if (k < ac.y) return a.prim[4 * ((size_t)a.v.G + ac.x + (k - g1)) + 1 + e];
    if (e == 2 && k == 0) return 0.0;
    const int il = e == 0 ? wrapi(i - 1, nx) : i, jl = e == 1 ? wrapi(j - 1, ny) : j, kl = e == 2 ? k - 1 : k;
    const double s = (double)a.rho[((size_t)kl * ny + jl) * nx + il] + (double)a.rho[(size_t)k * ny * nx + c];
    return (double)a.mom[e][mom_index(a.D, e, i, j, k)] / (0.5 * s);
}

// stress tau_cd on the lower d-face of the c-momentum CV (i, j, k) from the
// centred differences of the staggered grid (a full face)
template <typename T>
__device__ double mac_stress(const ViscArgs<T>& a, int c, int d, int i, int j, int k) {
    const int oc[3] = {c == 0, c == 1, c == 2}, od[3] = {d == 0, d == 1, d == 2};
    if (d == c) {
        const int qi = i - oc[0], qj = j - oc[1], qk = k - oc[2];
        double div = 0.0;
#pragma unroll
        for (int e = 0; e < 3; ++e)
            div += (vel_at(a, e, qi + (e == 0), qj + (e == 1), qk + (e == 2)) - vel_at(a, e, qi, qj, qk)) * a.rdel[e];
        const double dudx = (vel_at(a, c, i, j, k) - vel_at(a, c, qi, qj, qk)) * a.rdel[c];
        return 2.0 * a.mu * dudx + a.lam * div;
    }
    const double a1 = (vel_at(a, c, i, j, k) - vel_at(a, c, i - od[0], j - od[1], k - od[2])) * a.rdel[d];
    const double a2 = (vel_at(a, d, i, j, k) - vel_at(a, d, i - oc[0], j - oc[1], k - oc[2])) * a.rdel[c];
    return a.mu * (a1 + a2);
}

// One operator per group of VO_LANES lanes: the lanes split its points and
// add their partial sums by a butterfly over the group.
constexpr int VO_LANES = 8;

template <typename T>
__global__ void __launch_bounds__(256) k_visc_ops(ViscArgs<T> a) {
    const int q = (xcd_block() * blockDim.x + threadIdx.x) / VO_LANES;
    const int lane = threadIdx.x % VO_LANES;
    const bool valid = q < a.nop;
    double s = 0.0;
    const int p1 = valid ? a.op_off[q + 1] : 0;
    // four points per lane and pass: their codes and weights, then their
    // velocities, are loaded together
    constexpr int U = 4;
    for (int p = (valid ? a.op_off[q] : 0) + lane; p < p1; p += U * VO_LANES) {
        uint32_t code[U];
        double w[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int pp = p + u * VO_LANES;
            code[u] = pp < p1 ? a.op_pt[pp] : 0u;
            w[u] = pp < p1 ? a.op_w[pp] : 0.0;
        }
        double vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) vv[u] = a.prim[4 * (size_t)(code[u] & 0x0FFFFFFFu) + 1 + (code[u] >> 28)];
#pragma unroll
        for (int u = 0; u < U; ++u) s += w[u] * vv[u];
    }
#pragma unroll
    for (int m = VO_LANES / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m, VO_LANES);
    if (valid && lane == 0) a.flux[q] = s;
}

template <typename T>
__device__ __forceinline__ void store_mom(const ViscArgs<T>& a, int c, int i, int j, int k, double val) {
    a.out[c][mom_index(a.D, c, i, j, k)] = (T)val;
    if (c == 0 && i == 0) a.out[0][mom_index(a.D, 0, a.D.nx, j, k)] = (T)val;
    if (c == 1 && j == 0) a.out[1][mom_index(a.D, 1, i, a.D.ny, k)] = (T)val;
}

// divergence of the stresses of the c-momentum CV (i, j, k): lower faces at
// (i, j, k), upper faces at the lower faces of the +d neighbours; op gives
// the operator of a face (or -1 for the centred differences)
template <typename T, class Op>
__device__ double visc_div(const ViscArgs<T>& a, int c, int i, int j, int k, const double* blo, Op&& op) {
    const int nx = a.D.nx, ny = a.D.ny, nz = a.D.nz;
    double br = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double lo = 0.0, hi = 0.0;
        if (blo[d] > 0.0) {
            const int o = op(d);
            lo = o >= 0 ? a.flux[o] : mac_stress(a, c, d, i, j, k);
        }
        const int ip = d == 0 ? wrapi(i + 1, nx) : i, jp = d == 1 ? wrapi(j + 1, ny) : j, kp = d == 2 ? k + 1 : k;
        // the u and v CVs end at the top wall, whose face is stress-free; the
        // w CVs' upper z-face at the top is the last cell centre
        const bool wall = d == 2 && c != 2 && kp == nz;
        const double bh = wall ? 0.0 : (kp == nz ? 1.0 : beta_at(a.v, c + 1, d, ip, jp, kp));
        if (bh > 0.0) {
            const int o = op(3 + d);
            hi = o >= 0 ? a.flux[o] : mac_stress(a, c, d, ip, jp, kp);
        }
        br += (bh * hi - blo[d] * lo) * a.rdel[d];
    }
    return br;
}

template <typename T>
__global__ void __launch_bounds__(256) k_visc_gen(ViscArgs<T> a) {
    const int g = xcd_block() * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (g >= a.v.G) return;
    const double alpha = gq(a.v, c + 1, GQ_ALPHA, g);
    if (!(alpha > 0.0)) return;  // not a fluid CV
    const int col = a.v.gcol[g];
    const int4 ci = a.v.col[col];
    const int i = col % a.D.nx, j = col / a.D.nx, k = col_g0(ci) + (g - ci.z);
    if (c == 2 && k == 0) return;  // the bottom wall is no w CV
    double blo[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const bool wall = d == 2 && c != 2 && k == 0;  // bottom wall of the u and v CVs
        blo[d] = wall ? 0.0 : gq(a.v, c + 1, GQ_BX + d, g);
    }
    const int32_t* vt = a.vtab + ((size_t)g * 3 + c) * 7;
    double br = visc_div(a, c, i, j, k, blo, [&](int f) { return (int)vt[f]; });
    if (vt[6] >= 0) br += a.flux[vt[6]] / a.dv;
    double* uh = a.uhat + (size_t)(2 + c) * a.v.G + g;
    const double val = *uh + a.cdt * br / alpha;
    *uh = val;
    store_mom(a, c, i, j, k, val);
}

// the CVs of component e whose velocities a fit around the nominal point xn
// (global cell units) uses: 3 along an axis where xn lines up with the
// component's CV centres, 4 (two on each side) otherwise
void stencil_range(int e, const double xn[3], int lo[3], int hi[3]) {
    for (int a = 0; a < 3; ++a) {
        const double off = a == e ? 0.0 : 0.5;
        const double t = xn[a] - off;
        const double m = std::floor(t + 0.5);
        if (std::fabs(t - m) < 0.25) {
            lo[a] = (int)m - 1;
            hi[a] = (int)m + 1;
        } else {
            const int f = (int)std::floor(t);
            lo[a] = f - 1;
            hi[a] = f + 2;
        }
    }
}

}  // namespace

ebs_status build_viscous(ebs_ctx* cx) {
    const int G = cx->G, nx = cx->nx, ny = cx->ny, nz = cx->nz;
    for (void** p : {(void**)&cx->d_vop_off, (void**)&cx->d_vop_pt, (void**)&cx->d_vop_w,
                     (void**)&cx->d_vflux, (void**)&cx->d_vtab}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    cx->nvop = 0;
    if (G == 0) return EBS_OK;
    const int NQ = GQ_N;
    std::vector<double> geo((size_t)NINST * NQ * G);
    EBS_HIP(cx, hipMemcpy(geo.data(), cx->d_geo, sizeof(double) * geo.size(), hipMemcpyDeviceToHost));
    auto Q = [&](int inst, int q, int g) { return geo[((size_t)inst * NQ + q) * G + g]; };
    auto mod = [](int i, int n) { return ((i % n) + n) % n; };
    auto gid = [&](int i, int j, int k) -> int {
        const int c = mod(j, ny) * nx + mod(i, nx);
        if (k < cx->h_g0[c]) return -2;
        if (k >= cx->h_g1[c]) return -1;
        return cx->h_goff[c] + (k - cx->h_g0[c]);
    };
    auto alpha_h = [&](int inst, int i, int j, int k) -> double {
        if (k < 0 || k > nz - 1) return 0.0;
        if (inst == 3 && k == 0) return 0.0;
        const int g = gid(i, j, k);
        if (g == -2) return 0.0;
        if (g == -1) return 1.0;
        return Q(inst, GQ_ALPHA, g);
    };
    // position of a fluid velocity CV in the advected-quantity array: general
    // index, or an aux position above the range; -1 if the aux range ends below
    auto pos_h = [&](int i, int j, int k) -> int64_t {
        const int c = mod(j, ny) * nx + mod(i, nx);
        if (k < cx->h_g1[c]) return cx->h_goff[c] + (k - cx->h_g0[c]);
        if (k < cx->h_gp[c]) return (int64_t)G + cx->h_aoff[c] + (k - cx->h_g1[c]);
        return -1;
    };
    bool reach_ok = true;
    auto vc_h = [&](int inst, int i, int j, int k, double vc[3]) {
        const int g = gid(i, j, k);
        for (int d = 0; d < 3; ++d) vc[d] = g >= 0 ? Q(inst, GQ_VCX + d, g) : 0.0;
    };
    const double* del = cx->g.dx;
    const double mu = cx->visc.mu, lam = -2.0 / 3.0 * cx->visc.mu;
    std::vector<int32_t> off(1, 0), vtab((size_t)G * 3 * 7, -1);
    std::vector<uint32_t> pts;
    std::vector<double> wts;
    double ev[64][3], W[64][3];
    uint32_t code[64];
    // the fluid CVs of component e in the stencil around xn, offsets from x
    auto gather = [&](int e, const double xn[3], const double x[3]) -> int {
        int lo[3], hi[3];
        stencil_range(e, xn, lo, hi);
        int np = 0;
        for (int k = lo[2]; k <= hi[2]; ++k)
            for (int j = lo[1]; j <= hi[1]; ++j)
                for (int i = lo[0]; i <= hi[0]; ++i) {
                    if (!(alpha_h(e + 1, i, j, k) > 0.0)) continue;
                    double vc[3];
                    vc_h(e + 1, i, j, k, vc);
                    const int idx[3] = {i, j, k};
                    for (int a = 0; a < 3; ++a) ev[np][a] = (idx[a] + 0.5 - (a == e ? 0.5 : 0.0) + vc[a]) - x[a];
                    const int64_t ps = pos_h(i, j, k);
                    if (ps < 0) reach_ok = false;
                    code[np] = ((uint32_t)e << 28) | (uint32_t)std::max<int64_t>(ps, 0);
                    ++np;
                }
        return np;
    };
    // stress weights: coefficient of velocity component e in tau_cd from a
    // fitted gradient row Wk
    auto coef = [&](int e, int c, int d, const double* Wk) {
        double t = 0.0;
        if (e == c) t += mu * Wk[d];
        if (e == d) t += mu * Wk[c];
        if (c == d) t += lam * Wk[e];
        return t;
    };
    const int tang[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    for (int col = 0; col < cx->ncol; ++col) {
        const int i = col % nx, j = col / nx;
        for (int k = cx->h_g0[col]; k < cx->h_g1[col]; ++k) {
            const int g = cx->h_goff[col] + (k - cx->h_g0[col]);
            for (int c = 0; c < 3; ++c) {
                const int s = c + 1;
                if (c == 2 && k == 0) continue;  // the bottom wall is no w CV
                const int idx[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    if (d == 2 && c != 2 && k == 0) continue;  // stress-free bottom wall
                    const double b = Q(s, GQ_BX + d, g);
                    if (!(b > 0.0 && b < 1.0 - 1e-12)) continue;
                    double xn[3], x[3];
                    for (int a = 0; a < 3; ++a) xn[a] = idx[a] + 0.5 - (a == c ? 0.5 : 0.0) - (a == d ? 0.5 : 0.0);
                    for (int a = 0; a < 3; ++a) x[a] = xn[a];
                    x[tang[d][0]] += Q(s, GQ_FX1 + 2 * d, g);
                    x[tang[d][1]] += Q(s, GQ_FX1 + 2 * d + 1, g);
                    for (int e = 0; e < 3; ++e) {
                        if (!(d == c || e == c || e == d)) continue;
                        const int np = gather(e, xn, x);
                        lsq_weights(np, ev, true, del, W);
                        for (int p = 0; p < np; ++p) {
                            pts.push_back(code[p]);
                            wts.push_back(coef(e, c, d, W[p]));
                        }
                    }
                    const int op = (int)off.size() - 1;
                    off.push_back((int32_t)pts.size());
                    vtab[((size_t)g * 3 + c) * 7 + d] = op;
                    const int gl = k - (d == 2) >= 0 ? gid(i - (d == 0), j - (d == 1), k - (d == 2)) : -2;
                    if (gl >= 0) vtab[((size_t)gl * 3 + c) * 7 + 3 + d] = op;
                }
                if (cx->visc.eb_mode == 1 && Q(s, GQ_ALPHA, g) > 0.0 && Q(s, GQ_AREA, g) > 0.0) {
                    double xn[3], x[3];
                    for (int a = 0; a < 3; ++a) {
                        xn[a] = idx[a] + 0.5 - (a == c ? 0.5 : 0.0);
                        x[a] = xn[a] + Q(s, GQ_EBX + a, g);
                    }
                    const double av[3] = {Q(s, GQ_AX, g) * del[1] * del[2], Q(s, GQ_AY, g) * del[0] * del[2],
                                          Q(s, GQ_AZ, g) * del[0] * del[1]};
                    for (int e = 0; e < 3; ++e) {
                        const int np = gather(e, xn, x);
                        lsq_weights(np, ev, false, del, W);
                        for (int p = 0; p < np; ++p) {
                            double t = 0.0;  // tau_c . n_out A, n_out A = -(area vector into the fluid)
                            for (int d = 0; d < 3; ++d) t -= av[d] * coef(e, c, d, W[p]);
                            pts.push_back(code[p]);
                            wts.push_back(t);
                        }
                    }
                    const int op = (int)off.size() - 1;
                    off.push_back((int32_t)pts.size());
                    vtab[((size_t)g * 3 + c) * 7 + 6] = op;
                }
            }
        }
    }
    if (!reach_ok) {
        cx->err = "a viscous fit reads a velocity above the stored aux range";
        return EBS_E_UNSUPPORTED;
    }
    const int nop = (int)off.size() - 1;
    const size_t np = std::max<size_t>(pts.size(), 1);
    bool ok = hipMalloc(&cx->d_vop_off, sizeof(int32_t) * (nop + 1)) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_vop_pt, sizeof(int32_t) * np) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_vop_w, sizeof(double) * np) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_vflux, sizeof(double) * std::max(nop, 1)) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_vtab, sizeof(int32_t) * vtab.size()) == hipSuccess;
    if (!ok) {
        cx->err = "viscous operator allocation failed";
        return EBS_E_OOM;
    }
    EBS_HIP(cx, hipMemcpy(cx->d_vop_off, off.data(), sizeof(int32_t) * (nop + 1), hipMemcpyHostToDevice));
    if (!pts.empty()) {
        EBS_HIP(cx, hipMemcpy(cx->d_vop_pt, pts.data(), sizeof(uint32_t) * pts.size(), hipMemcpyHostToDevice));
        EBS_HIP(cx, hipMemcpy(cx->d_vop_w, wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
    }
    EBS_HIP(cx, hipMemcpy(cx->d_vtab, vtab.data(), sizeof(int32_t) * vtab.size(), hipMemcpyHostToDevice));
    cx->nvop = nop;
    return EBS_OK;
}

template <typename T>
static ViscArgs<T> visc_args(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt) {
    ViscArgs<T> a;
    a.D = Dims{cx->nx, cx->ny, cx->nz};
    a.v = geo_view(cx);
    a.rho = (const T*)Ucur->rho;
    a.mom[0] = (const T*)Ucur->rhou;
    a.mom[1] = (const T*)Ucur->rhov;
    a.mom[2] = (const T*)Ucur->rhow;
    a.out[0] = (T*)Uh->rhou;
    a.out[1] = (T*)Uh->rhov;
    a.out[2] = (T*)Uh->rhow;
    a.uhat = cx->d_uhat;
    a.op_off = cx->d_vop_off;
    a.op_pt = cx->d_vop_pt;
    a.prim = cx->d_prim;
    a.acol = cx->d_acol;
    a.op_w = cx->d_vop_w;
    a.flux = cx->d_vflux;
    a.vtab = cx->d_vtab;
    a.nop = cx->nvop;
    a.mu = cx->visc.mu;
    a.lam = -2.0 / 3.0 * cx->visc.mu;
    a.cdt = cdt;
    a.dv = cx->g.dx[0] * cx->g.dx[1] * cx->g.dx[2];
    for (int d = 0; d < 3; ++d) a.rdel[d] = 1.0 / cx->g.dx[d];
    return a;
}

template <typename T>
static ebs_status visc_general_t(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt) {
    if (cx->G == 0) return EBS_OK;
    const ViscArgs<T> a = visc_args<T>(cx, Ucur, Uh, cdt);
    if (a.nop > 0)
        hipLaunchKernelGGL(k_visc_ops<T>, dim3(xcd_grid(((int64_t)a.nop * VO_LANES + 255) / 256)), dim3(256), 0,
                           cx->stream, a);
    hipLaunchKernelGGL(k_visc_gen<T>, dim3(xcd_grid((cx->G + 255) / 256), 3), dim3(256), 0, cx->stream, a);
    EBS_HIP(cx, hipGetLastError());
    return EBS_OK;
}

ebs_status launch_viscous_general(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt) {
    if (cx->g.precision == EBS_F32_BULK) return visc_general_t<float>(cx, Ucur, Uh, cdt);
    return visc_general_t<double>(cx, Ucur, Uh, cdt);
}


}  // namespace ebs
