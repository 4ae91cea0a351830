// Diffusion in the regular region (Section 4.2 on full faces): the thermal
// diffusion of rho theta (flux rho alpha_theta grad theta) and the momentum
// diffusion (viscous stress tau = lambda (div u) I + mu (grad u + grad u^T),
// lambda = -2/3 mu), added to what the regular-region stage kernel wrote for
// every cell at or above its column's general range.
//
// There every face is full and every cell the centred differences read is
// fluid (the top of the general range is chosen so that every cell the
// advective stencils of the regular region read is fluid, and these
// differences reach less far), so theta = rho theta / rho and every face
// velocity is u = 2 rho u / (rho_L + rho_R).  Flux of rho theta through a
// face: the mean density of its two cells times alpha_theta times the centred
// difference of theta; the bottom and top walls are adiabatic.  Stresses:
// tau_xx, tau_yy, tau_zz at cell centres from the six face velocities of the
// cell, the shear stresses at cell edges from the two velocities across the
// edge in each direction; the bottom and top walls are stress-free for the u
// and v CVs, the w CVs end at the cell centres of the first and last layers
// (w = 0 on the walls).
//
// A block owns a TX x TY tile of columns and marches up from the lowest
// regular level of the tile.  LDS rings hold the density planes p - 2, p - 1
// and p of the tile plus two cells on the low sides and one on the high sides
// (plane p enters while the update of the last iteration may still read
// plane p - 2), the velocity planes p - 2, p - 1, p and the theta planes
// p - 1, p of the tile plus one cell around it; plane p - 1 is then updated.
// Each shared stress or flux is evaluated by the same arithmetic on both
// sides of its face, so it enters the two CVs with opposite signs.
#include <hip/hip_runtime.h>

#include "ebs_internal.h"
#include "stage_common.h"
#include "xcd.h"

namespace ebs {
namespace {

template <typename T>
struct RegDiffArgs {
    Dims D;
    const int32_t* g1;
    const T* rho;
    const T* rt;
    const T* mom[3];
    T* out_rt;
    T* out[3];
    T al;             // alpha_theta
    T mu, mu2, lam;   // mu, 2 mu, lambda
    T cdt;
    T rd[3];
};

template <typename T, int TX, int TY, bool TH, bool VI>
__global__ void __launch_bounds__(TX * TY) k_diff_regular(RegDiffArgs<T> a) {
    constexpr int VX = TX + 2, VS = VX * (TY + 2);  // one cell around the tile
    constexpr int DX = TX + 3, DS = DX * (TY + 3);  // two cells on the low sides
    constexpr int NT = TX * TY;
    constexpr int NV = (VS + NT - 1) / NT, ND = (DS + NT - 1) / NT;
    __shared__ T dens[3][DS];  // planes p - 2, p - 1, p (slot p mod 3)
    __shared__ T vel[VI ? 3 : 1][VI ? 3 : 1][VI ? VS : 1];  // [slot][component][point]
    __shared__ T tha[TH ? 2 : 1][TH ? VS : 1];             // [slot][point]
    __shared__ int kmin_s;
    const int nx = a.D.nx, ny = a.D.ny, nz = a.D.nz;
    const int t = threadIdx.x;
    const int tx = t % TX, ty = t / TX;
    // tiles in row-major order, one contiguous run of rows of tiles per XCD
    // (xcd.h), so the halo lines two neighbouring tiles share stay in one L2
    const int ntx = (nx + TX - 1) / TX;
    const int tile = xcd_block();
    if (tile >= ntx * ((ny + TY - 1) / TY)) return;  // block uniform
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int i = x0 + tx, j = y0 + ty;
    const bool act = i < nx && j < ny;
    const int kg = act ? a.g1[j * nx + i] : nz;
    if (t == 0) kmin_s = nz;
    __syncthreads();
    atomicMin(&kmin_s, kg);
    __syncthreads();
    const int kmin = kmin_s;  // lowest regular level of the tile (block uniform)
    if (kmin >= nz) return;
    const size_t pc = (size_t)nx * ny, pu = (size_t)(nx + 1) * ny, pv = (size_t)nx * (ny + 1);
    // this thread's points of the two regions (row-major), -1 past the end
    int vpt[NV], dpt[ND];
    size_t vc[NV], vu[NV], dc[ND];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const int r = t + q * NT;
        vpt[q] = r < VS ? r : -1;
        const int rr = r < VS ? r : 0;
        const int X = wrapi(x0 - 1 + rr % VX, nx), Y = wrapi(y0 - 1 + rr / VX, ny);
        vc[q] = (size_t)Y * nx + X;
        vu[q] = (size_t)Y * (nx + 1) + X;
    }
#pragma unroll
    for (int q = 0; q < ND; ++q) {
        const int r = t + q * NT;
        dpt[q] = r < DS ? r : -1;
        const int rr = r < DS ? r : 0;
        const int X = wrapi(x0 - 2 + rr % DX, nx), Y = wrapi(y0 - 2 + rr / DX, ny);
        dc[q] = (size_t)Y * nx + X;
    }
    // raw values of the next plane: densities of the density points; rho
    // theta and momenta of the velocity points
    T rd_[ND], rt_[NV], ru_[NV], rv_[NV], rw_[NV];
    auto fetch = [&](int p) {
        const bool in = p >= 0 && p < nz;  // block uniform
#pragma unroll
        for (int q = 0; q < ND; ++q) rd_[q] = (in && dpt[q] >= 0) ? a.rho[(size_t)p * pc + dc[q]] : T(0);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const bool ok = in && vpt[q] >= 0;
            if (TH) rt_[q] = ok ? a.rt[(size_t)p * pc + vc[q]] : T(0);
            if (VI) {
                ru_[q] = ok ? a.mom[0][(size_t)p * pu + vu[q]] : T(0);
                rv_[q] = ok ? a.mom[1][(size_t)p * pv + vc[q]] : T(0);
                rw_[q] = ok ? a.mom[2][(size_t)p * pc + vc[q]] : T(0);
            }
        }
    };
    // face velocity: the momentum over the mean density of the two cells
    auto fv = [](T m, T r0, T r1) -> T {
        const T s = r0 + r1;
        return s > T(0) ? (T(2) * m) / s : T(0);
    };
    fetch(kmin - 2);
    const int me = (ty + 1) * VX + (tx + 1);   // own point in the velocity region
    const int dme = (ty + 2) * DX + (tx + 2);  // own point in the density region
    const T mu = a.mu, mu2 = a.mu2, lam = a.lam, rdx = a.rd[0], rdy = a.rd[1], rdz = a.rd[2];
    T thm1 = T(0), rhm1 = T(0);  // own theta and rho of the plane below the updated one
    // the output values of the own cell that the next update adds to (rho
    // theta, rho u, rho v, rho w of plane p - 1), loaded one iteration ahead
    T oo[4] = {T(0), T(0), T(0), T(0)};
    auto fetch_out = [&](int kk) {
        if (!(act && kk >= kmin && kk >= kg && kk < nz)) return;
        // read once and written back once by this launch: streaming accesses
        if (TH) oo[0] = __builtin_nontemporal_load(&a.out_rt[((size_t)kk * ny + j) * nx + i]);
        if (VI) {
            oo[1] = __builtin_nontemporal_load(&a.out[0][((size_t)kk * ny + j) * (nx + 1) + i]);
            oo[2] = __builtin_nontemporal_load(&a.out[1][((size_t)kk * (ny + 1) + j) * nx + i]);
            if (kk >= 1) oo[3] = __builtin_nontemporal_load(&a.out[2][((size_t)kk * ny + j) * nx + i]);
        }
    };
    fetch_out(kmin - 1);
    for (int p = kmin - 2; p <= nz; ++p) {
        // density plane p enters the ring (its slot held plane p - 3, which
        // no thread reads any more; planes p - 2 and p - 1, which the update
        // of the last iteration may still be reading, keep theirs)
        T* Dp = dens[(p + 3) % 3];
        const T* Dm = dens[(p + 2) % 3];
#pragma unroll
        for (int q = 0; q < ND; ++q)
            if (dpt[q] >= 0) Dp[dpt[q]] = rd_[q];
        __syncthreads();
        if (p >= kmin - 1) {
            // velocities and theta of plane p (zero beyond the walls; w zero on them)
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                const int r = vpt[q];
                if (r < 0) continue;
                const int lx = r % VX, ly = r / VX;
                const int d = (ly + 1) * DX + (lx + 1);  // the same point in the density region
                const bool in = p >= 0 && p < nz;
                if (TH) tha[p & 1][r] = (in && Dp[d] > T(0)) ? rt_[q] / Dp[d] : T(0);
                if (VI) {
                    T u = T(0), v = T(0), w = T(0);
                    if (in) {
                        u = fv(ru_[q], Dp[d - 1], Dp[d]);
                        v = fv(rv_[q], Dp[d - DX], Dp[d]);
                        if (p > 0) w = fv(rw_[q], Dm[d], Dp[d]);
                    }
                    T* Vs = &vel[(p + 3) % 3][0][0];
                    Vs[r] = u;
                    Vs[VS + r] = v;
                    Vs[2 * VS + r] = w;
                }
            }
        }
        fetch(p + 1);
        T on[4] = {oo[0], oo[1], oo[2], oo[3]};  // this update's output values
        fetch_out(p);
        __syncthreads();
        const int k = p - 1;  // the plane updated now
        if (k >= kmin && act && k >= kg) {
            if (TH) {
                // theta planes k (around the tile) and k + 1 (slot p); own theta
                // and rho of plane k - 1 from the registers
                const T* Tk = tha[k & 1];
                const T* Dk = dens[(k + 3) % 3];
                const T r0 = Dk[dme], t0 = Tk[me];
                auto face = [&](T rn, T tn) { return T(0.5) * (rn + r0) * a.al * (tn - t0); };
                T br = (face(Dk[dme + 1], Tk[me + 1]) + face(Dk[dme - 1], Tk[me - 1])) * (rdx * rdx);
                br += (face(Dk[dme + DX], Tk[me + VX]) + face(Dk[dme - DX], Tk[me - VX])) * (rdy * rdy);
                T bz = T(0);
                if (k + 1 < nz) bz += face(Dp[dme], tha[p & 1][me]);
                if (k > 0) bz += face(rhm1, thm1);
                br += bz * (rdz * rdz);
                const size_t o = ((size_t)k * ny + j) * nx + i;
                __builtin_nontemporal_store(on[0] + a.cdt * br, &a.out_rt[o]);
            }
            if (VI) {
                // velocity slots of planes k - 1, k, k + 1
                const T* V0 = &vel[(k + 3) % 3][0][0];
                const T* Vm = &vel[(k + 2) % 3][0][0];
                const T* Vp = &vel[(k + 4) % 3][0][0];
                auto U = [&](const T* V, int ox, int oy) { return V[me + oy * VX + ox]; };
                auto Vv = [&](const T* V, int ox, int oy) { return V[VS + me + oy * VX + ox]; };
                auto W = [&](const T* V, int ox, int oy) { return V[2 * VS + me + oy * VX + ox]; };
                // divergence of the cell (i + ox, j + oy) of a plane (slots S of
                // that plane and S1 of the plane above)
                auto div = [&](const T* S, const T* S1, int ox, int oy) {
                    T dv = (U(S, ox + 1, oy) - U(S, ox, oy)) * rdx;
                    dv += (Vv(S, ox, oy + 1) - Vv(S, ox, oy)) * rdy;
                    dv += (W(S1, ox, oy) - W(S, ox, oy)) * rdz;
                    return dv;
                };
                // shear stresses: xy at the edge (i + ox - 1/2, j + oy - 1/2) of
                // plane k; xz at (i + ox - 1/2) and yz at (j + oy - 1/2) between
                // the planes of slots Sm and S
                auto exy = [&](int ox, int oy) {
                    return mu * ((U(V0, ox, oy) - U(V0, ox, oy - 1)) * rdy + (Vv(V0, ox, oy) - Vv(V0, ox - 1, oy)) * rdx);
                };
                auto exz = [&](const T* Sm, const T* S, int ox) {
                    return mu * ((U(S, ox, 0) - U(Sm, ox, 0)) * rdz + (W(S, ox, 0) - W(S, ox - 1, 0)) * rdx);
                };
                auto eyz = [&](const T* Sm, const T* S, int oy) {
                    return mu * ((Vv(S, 0, oy) - Vv(Sm, 0, oy)) * rdz + (W(S, 0, oy) - W(S, 0, oy - 1)) * rdy);
                };
                const T d00 = div(V0, Vp, 0, 0);
                const T xy00 = exy(0, 0);
                const T xz_lo = exz(Vm, V0, 0), yz_lo = eyz(Vm, V0, 0);
                // u CV (faces at the cell centres i - 1 and i)
                {
                    const T t0 = mu2 * (U(V0, 0, 0) - U(V0, -1, 0)) * rdx + lam * div(V0, Vp, -1, 0);
                    const T t1 = mu2 * (U(V0, 1, 0) - U(V0, 0, 0)) * rdx + lam * d00;
                    const T zlo = k == 0 ? T(0) : xz_lo;
                    const T zhi = k == nz - 1 ? T(0) : exz(V0, Vp, 0);
                    const T br = (t1 - t0) * rdx + (exy(0, 1) - xy00) * rdy + (zhi - zlo) * rdz;
                    const size_t o = ((size_t)k * ny + j) * (nx + 1) + i;
                    const T val = on[1] + a.cdt * br;
                    __builtin_nontemporal_store(val, &a.out[0][o]);
                    if (i == 0) __builtin_nontemporal_store(val, &a.out[0][o + nx]);
                }
                // v CV (faces at the cell centres j - 1 and j)
                {
                    const T t0 = mu2 * (Vv(V0, 0, 0) - Vv(V0, 0, -1)) * rdy + lam * div(V0, Vp, 0, -1);
                    const T t1 = mu2 * (Vv(V0, 0, 1) - Vv(V0, 0, 0)) * rdy + lam * d00;
                    const T zlo = k == 0 ? T(0) : yz_lo;
                    const T zhi = k == nz - 1 ? T(0) : eyz(V0, Vp, 0);
                    const T br = (exy(1, 0) - xy00) * rdx + (t1 - t0) * rdy + (zhi - zlo) * rdz;
                    const size_t o = ((size_t)k * (ny + 1) + j) * nx + i;
                    const T val = on[2] + a.cdt * br;
                    __builtin_nontemporal_store(val, &a.out[1][o]);
                    if (j == 0) __builtin_nontemporal_store(val, &a.out[1][o + (size_t)ny * nx]);
                }
                // w CV (faces at the cell centres k - 1 and k; none on the bottom wall)
                if (k >= 1) {
                    const T t0 = mu2 * (W(V0, 0, 0) - W(Vm, 0, 0)) * rdz + lam * div(Vm, V0, 0, 0);
                    const T t1 = mu2 * (W(Vp, 0, 0) - W(V0, 0, 0)) * rdz + lam * d00;
                    const T br =
                        (exz(Vm, V0, 1) - xz_lo) * rdx + (eyz(Vm, V0, 1) - yz_lo) * rdy + (t1 - t0) * rdz;
                    const size_t o = ((size_t)k * ny + j) * nx + i;
                    __builtin_nontemporal_store(on[3] + a.cdt * br, &a.out[2][o]);
                }
            }
        }
        if (TH) {
            // own theta and rho of plane p - 1 for the update of plane p
            thm1 = tha[(p + 1) & 1][me];
            rhm1 = Dm[dme];
        }
    }
}

constexpr int RD_TX = 64, RD_TY = 8;

template <typename T, bool TH, bool VI>
ebs_status launch_t(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt, hipStream_t s) {
    RegDiffArgs<T> a;
    a.D = Dims{cx->nx, cx->ny, cx->nz};
    a.g1 = cx->d_g1;
    a.rho = (const T*)Ucur->rho;
    a.rt = (const T*)Ucur->rhotheta;
    a.mom[0] = (const T*)Ucur->rhou;
    a.mom[1] = (const T*)Ucur->rhov;
    a.mom[2] = (const T*)Ucur->rhow;
    a.out_rt = (T*)Uh->rhotheta;
    a.out[0] = (T*)Uh->rhou;
    a.out[1] = (T*)Uh->rhov;
    a.out[2] = (T*)Uh->rhow;
    a.al = (T)(TH ? cx->diff.alpha_theta : 0.0);
    const double mu = VI ? cx->visc.mu : 0.0;
    a.mu = (T)mu;
    a.mu2 = (T)(2.0 * mu);
    a.lam = (T)(-2.0 / 3.0 * mu);
    a.cdt = (T)cdt;
    for (int d = 0; d < 3; ++d) a.rd[d] = (T)(1.0 / cx->g.dx[d]);
    const dim3 grid(xcd_grid((long long)((cx->nx + RD_TX - 1) / RD_TX) * ((cx->ny + RD_TY - 1) / RD_TY)));
    hipLaunchKernelGGL((k_diff_regular<T, RD_TX, RD_TY, TH, VI>), grid, dim3(RD_TX * RD_TY), 0, s, a);
    EBS_HIP(cx, hipGetLastError());
    return EBS_OK;
}

template <typename T>
ebs_status launch_prec(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt, hipStream_t s) {
    if (cx->diff_on && cx->visc_on) return launch_t<T, true, true>(cx, Ucur, Uh, cdt, s);
    if (cx->diff_on) return launch_t<T, true, false>(cx, Ucur, Uh, cdt, s);
    if (cx->visc_on) return launch_t<T, false, true>(cx, Ucur, Uh, cdt, s);
    return EBS_OK;
}

}  // namespace

ebs_status launch_regular_diffusion(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt, hipStream_t s) {
    if (cx->g.precision == EBS_F32_BULK) return launch_prec<float>(cx, Ucur, Uh, cdt, s);
    return launch_prec<double>(cx, Ucur, Uh, cdt, s);
}

}  // namespace ebs
