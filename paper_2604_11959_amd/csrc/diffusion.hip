// Thermal diffusion of rho theta (Section 4.2): the diffusive flux of rho
// theta is rho alpha_theta grad(theta), and on cut faces and at the EB the
// gradient comes from a least-squares fit of a second-order polynomial over a
// local neighbourhood of cells (3 wide around a cell's EB facet, 4 wide along
// the normal of a face, so that a face's stencil is symmetric about it).
//
// Readings (where the paper defers to its reference): full faces (area
// fraction >= 1 - 1e-12) take the centred difference of theta; a cut face
// takes the normal component of the fitted gradient at its centroid; the fit is unweighted over the fluid cells
// of the stencil at their volume centroids, quadratic in mesh units about the
// evaluation point, linear when fewer than 10 points remain or the quadratic
// normal matrix has a reciprocal 1-norm condition number below 1e-7, and zero
// with fewer than 4 points or a linear matrix as poorly conditioned; the EB
// is adiabatic or held at theta_wall, the facet fit then passing through the
// wall value at the facet centroid (no constant term); face density = mean of
// the two cells, facet density = the cut cell's; top and bottom walls are
// adiabatic.
//
// Every fit depends on the geometry only, so its weights are built once: the
// gradient component a stage needs is a fixed linear combination of the theta
// values of the stencil cells.  Per stage:
//   k_diff_ops  a group of lanes per operator (cut face or EB facet): its
//               flux;
//   k_diff_gen  one thread per general cell: divergence over its six faces
//               (full faces by centred differences) and the facet, added to
//               the provisional rho theta (FP64 copy and the output state).
// The cells above the general range, where every face is full, are updated
// with the momentum diffusion in one pass (regdiff.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "ebs_internal.h"
#include "stage_common.h"
#include "xcd.h"

namespace ebs {
namespace {

template <typename T>
struct DiffArgs {
    Dims D;
    GeoView v;
    const T* cur_rho;
    const T* cur_rt;
    T* out_rt;
    double* uhat_rt;          // [G] FP64 provisional rho theta of the general cells
    const double* prim;       // [G + naux][4] advected quantities of the stage (theta first)
    const int32_t* op_off;    // [nop + 1]
    const int32_t* op_idx;    // [pts] position of each stencil point in prim
    const double* op_w;       // [pts] weight of its theta
    const int32_t* op_cell;   // [nop] linear index of the operator's cell | direction << 30 (3 = facet)
    double* flux;             // [nop] flux density (face) or facet term
    const int32_t* dtab;      // [G][7] operator of the lower x, y, z, upper x, y, z face and the facet
    int32_t nop;
    double alpha, theta_wall, cdt, dv;
    double rdel[3];
};

template <typename T>
__device__ __forceinline__ double theta_at(const DiffArgs<T>& a, uint32_t c) {
    return (double)a.cur_rt[c] / (double)a.cur_rho[c];
}

__device__ __forceinline__ uint32_t lin(const Dims& D, int i, int j, int k) {
    return ((uint32_t)k * D.ny + j) * D.nx + i;
}

// One operator per group of DO_LANES lanes: the lanes split its stencil
// points (theta from the advected-quantity pass of the stage) and add their
// partial sums by a butterfly over the group.
constexpr int DO_LANES = 8;

template <typename T>
__global__ void __launch_bounds__(256) k_diff_ops(DiffArgs<T> a) {
    const int q = (xcd_block() * blockDim.x + threadIdx.x) / DO_LANES;
    const int lane = threadIdx.x % DO_LANES;
    const bool valid = q < a.nop;
    const int32_t m = valid ? a.op_cell[q] : 0;
    const int d = (int)((uint32_t)m >> 30);
    // facet: the weights act on theta - theta_wall
    const double sh = d == 3 ? a.theta_wall : 0.0;
    double s = 0.0;
    const int e = valid ? a.op_off[q + 1] : 0;
    for (int p = (valid ? a.op_off[q] : 0) + lane; p < e; p += DO_LANES)
        s += a.op_w[p] * (a.prim[4 * (size_t)a.op_idx[p]] - sh);
#pragma unroll
    for (int mm = DO_LANES / 2; mm >= 1; mm >>= 1) s += __shfl_xor(s, mm, DO_LANES);
    if (!valid || lane != 0) return;
    const uint32_t c = (uint32_t)m & 0x3FFFFFFFu;
    if (d == 3) {
        a.flux[q] = -(double)a.cur_rho[c] * a.alpha * s;
        return;
    }
    // the cell below the face along d
    const int nx = a.D.nx, ny = a.D.ny;
    const int i = (int)(c % nx), j = (int)((c / nx) % ny), k = (int)(c / ((uint32_t)nx * ny));
    const uint32_t cl = d == 0 ? lin(a.D, wrapi(i - 1, nx), j, k) : d == 1 ? lin(a.D, i, wrapi(j - 1, ny), k)
                                                                          : lin(a.D, i, j, k - 1);
    const double rf = 0.5 * ((double)a.cur_rho[cl] + (double)a.cur_rho[c]);
    a.flux[q] = rf * a.alpha * s;
}

// area fraction of the lower d-face of the cell-centred CV at (i, j, k)
__device__ __forceinline__ double beta0(const GeoView& v, int d, int i, int j, int k) {
    const int g = gidx(v, i, j, k);
    if (g == -2) return 0.0;
    if (g == -1) return 1.0;
    return gq(v, 0, GQ_BX + d, g);
}

template <typename T>
__global__ void __launch_bounds__(256) k_diff_gen(DiffArgs<T> a) {
    const int g = xcd_block() * blockDim.x + threadIdx.x;
    if (g >= a.v.G) return;
    if (a.v.type[g] == 0) return;  // cell-centred CV without fluid
    const int c = a.v.gcol[g];
    const int4 ci = a.v.col[c];
    const int nx = a.D.nx, ny = a.D.ny, nz = a.D.nz;
    const int i = c % nx, j = c / nx, k = col_g0(ci) + (g - ci.z);
    const uint32_t me = lin(a.D, i, j, k);
    const double tme = theta_at(a, me), rme = (double)a.cur_rho[me];
    double br = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // lower face
        double lo = 0.0;
        const bool wall_lo = d == 2 && k == 0;
        const double bl = wall_lo ? 0.0 : gq(a.v, 0, GQ_BX + d, g);
        if (bl > 0.0) {
            const int op = a.dtab[(size_t)g * 7 + d];
            if (op >= 0) {
                lo = a.flux[op];
            } else {
                const uint32_t cl = d == 0 ? lin(a.D, wrapi(i - 1, nx), j, k)
                                  : d == 1 ? lin(a.D, i, wrapi(j - 1, ny), k) : lin(a.D, i, j, k - 1);
                lo = 0.5 * ((double)a.cur_rho[cl] + rme) * a.alpha * (tme - theta_at(a, cl)) * a.rdel[d];
            }
        }
        // upper face: the lower face of the neighbour along +d
        double hi = 0.0;
        const int ip = d == 0 ? wrapi(i + 1, nx) : i, jp = d == 1 ? wrapi(j + 1, ny) : j, kp = d == 2 ? k + 1 : k;
        const bool wall_hi = d == 2 && kp == nz;
        const double bh = wall_hi ? 0.0 : beta0(a.v, d, ip, jp, kp);
        if (bh > 0.0) {
            const int op = a.dtab[(size_t)g * 7 + 3 + d];
            if (op >= 0) {
                hi = a.flux[op];
            } else {
                const uint32_t cu = lin(a.D, ip, jp, kp);
                hi = 0.5 * ((double)a.cur_rho[cu] + rme) * a.alpha * (theta_at(a, cu) - tme) * a.rdel[d];
            }
        }
        br += (bh * hi - bl * lo) * a.rdel[d];
    }
    const int eo = a.dtab[(size_t)g * 7 + 6];
    if (eo >= 0) br += a.flux[eo] / a.dv;
    const double val = a.uhat_rt[g] + a.cdt * br / gq(a.v, 0, GQ_ALPHA, g);
    a.uhat_rt[g] = val;
    a.out_rt[me] = (T)val;
}

// ---------------------------------------------------------------- set-up

// n x n Gauss-Jordan inverse with partial pivoting; 1-norm reciprocal
// condition number.  false if singular.
bool invert(int n, const double (&M)[10][10], double (&Inv)[10][10], double& rcond) {
    double A[10][10];
    for (int r = 0; r < n; ++r)
        for (int q = 0; q < n; ++q) {
            A[r][q] = M[r][q];
            Inv[r][q] = r == q ? 1.0 : 0.0;
        }
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::fabs(A[r][col]) > std::fabs(A[piv][col])) piv = r;
        if (!(std::fabs(A[piv][col]) > 0.0)) return false;
        if (piv != col)
            for (int q = 0; q < n; ++q) {
                std::swap(A[col][q], A[piv][q]);
                std::swap(Inv[col][q], Inv[piv][q]);
            }
        const double p = A[col][col];
        for (int q = 0; q < n; ++q) {
            A[col][q] /= p;
            Inv[col][q] /= p;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const double f = A[r][col];
            for (int q = 0; q < n; ++q) {
                A[r][q] -= f * A[col][q];
                Inv[r][q] -= f * Inv[col][q];
            }
        }
    }
    double n1 = 0.0, ni = 0.0;
    for (int q = 0; q < n; ++q) {
        double ca = 0.0, cb = 0.0;
        for (int r = 0; r < n; ++r) {
            ca += std::fabs(M[r][q]);
            cb += std::fabs(Inv[r][q]);
        }
        n1 = std::max(n1, ca);
        ni = std::max(ni, cb);
    }
    rcond = 1.0 / (n1 * ni);
    return true;
}

int basis_row(const double e[3], bool quad, bool with_const, double (&row)[10]) {
    int n = 0;
    if (with_const) row[n++] = 1.0;
    row[n++] = e[0];
    row[n++] = e[1];
    row[n++] = e[2];
    if (quad) {
        row[n++] = 0.5 * e[0] * e[0];
        row[n++] = 0.5 * e[1] * e[1];
        row[n++] = 0.5 * e[2] * e[2];
        row[n++] = e[0] * e[1];
        row[n++] = e[0] * e[2];
        row[n++] = e[1] * e[2];
    }
    return n;
}

}  // namespace

// Weights of the fitted gradient (physical units, per direction) at the
// evaluation point from np points at mesh-unit offsets e: grad_d =
// sum_s W[s][d] q_s.  All zero when no fit qualifies.  Also used by the
// momentum diffusion.
void lsq_weights(int np, const double (*e)[3], bool with_const, const double* del, double (*W)[3]) {
    for (int s = 0; s < np; ++s) W[s][0] = W[s][1] = W[s][2] = 0.0;
    for (int quad = 1; quad >= 0; --quad) {
        double row[10];
        const int nb = basis_row(e[0], quad, with_const, row);
        if (np < nb) continue;
        double M[10][10] = {{0.0}};
        for (int s = 0; s < np; ++s) {
            basis_row(e[s], quad, with_const, row);
            for (int r = 0; r < nb; ++r)
                for (int q = 0; q < nb; ++q) M[r][q] += row[r] * row[q];
        }
        double Inv[10][10], rc = 0.0;
        if (!invert(nb, M, Inv, rc) || !(rc >= 1e-7)) continue;
        const int o = with_const ? 1 : 0;
        for (int s = 0; s < np; ++s) {
            basis_row(e[s], quad, with_const, row);
            for (int d = 0; d < 3; ++d) {
                double w = 0.0;
                for (int q = 0; q < nb; ++q) w += Inv[o + d][q] * row[q];
                W[s][d] = w / del[d];
            }
        }
        return;
    }
}

// Builds the fit operators of every cut face of the cell-centred instance
// inside the general range and, with an isothermal EB, of every cut cell's
// facet, and the per-cell operator table.
ebs_status build_diffusion(ebs_ctx* cx) {
    const int G = cx->G, nx = cx->nx, ny = cx->ny, nz = cx->nz;
    for (void** p : {(void**)&cx->d_dop_off, (void**)&cx->d_dop_idx, (void**)&cx->d_dop_w, (void**)&cx->d_dop_cell,
                     (void**)&cx->d_dflux, (void**)&cx->d_dtab}) {
        if (*p) (void)hipFree(*p);
        *p = nullptr;
    }
    cx->ndop = 0;
    if (G == 0) return EBS_OK;
    // instance-0 geometry of the general cells
    const int NQ = GQ_N;
    std::vector<double> geo((size_t)NQ * G);
    std::vector<int8_t> ty(G);
    EBS_HIP(cx, hipMemcpy(geo.data(), cx->d_geo, sizeof(double) * NQ * G, hipMemcpyDeviceToHost));
    EBS_HIP(cx, hipMemcpy(ty.data(), cx->d_type, G, hipMemcpyDeviceToHost));
    auto Q = [&](int q, int g) { return geo[(size_t)q * G + g]; };
    // general index of (i, j, k): -2 below the range, -1 above
    auto gid = [&](int i, int j, int k) -> int {
        const int c = wrapi(j, ny) * nx + wrapi(i, nx);
        if (k < cx->h_g0[c]) return -2;
        if (k >= cx->h_g1[c]) return -1;
        return cx->h_goff[c] + (k - cx->h_g0[c]);
    };
    // fluid test and volume-centroid offset (mesh units) of a cell
    auto cell = [&](int i, int j, int k, double vc[3]) -> bool {
        vc[0] = vc[1] = vc[2] = 0.0;
        if (k < 0 || k >= nz) return false;
        const int g = gid(i, j, k);
        if (g == -2) return false;
        if (g == -1) return true;
        if (ty[g] == 0) return false;
        for (int d = 0; d < 3; ++d) vc[d] = Q(GQ_VCX + d, g);
        return true;
    };
    // position of a fluid cell in the advected-quantity array: general index,
    // or an aux position above the range; -1 if the aux range ends below
    bool reach_ok = true;
    auto pos = [&](int i, int j, int k) -> int32_t {
        const int c = wrapi(j, ny) * nx + wrapi(i, nx);
        if (k < cx->h_g1[c]) return cx->h_goff[c] + (k - cx->h_g0[c]);
        if (k < cx->h_gp[c]) return (int32_t)(G + cx->h_aoff[c] + (k - cx->h_g1[c]));
        reach_ok = false;
        return 0;
    };
    const double* del = cx->g.dx;
    std::vector<int32_t> off(1, 0), idx, ocell, dtab((size_t)7 * G, -1);
    std::vector<double> wts;
    double e[36][3], W[36][3];
    int32_t pidx[36];
    const int tang[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    // columns in order: general cells are numbered column by column
    for (int col = 0; col < cx->ncol; ++col) {
        const int i = col % nx, j = col / nx;
        for (int k = cx->h_g0[col]; k < cx->h_g1[col]; ++k) {
            const int g = cx->h_goff[col] + (k - cx->h_g0[col]);
            if (ty[g] == 0) continue;
            // lower faces with 0 < beta < 1
            for (int d = 0; d < 3; ++d) {
                if (d == 2 && k == 0) continue;
                // cut face: 0 < beta < 1 - 1e-12 (a face that the terrain only
                // touches counts as full, so the last-bit rounding of the
                // geometry cannot switch the gradient method)
                const double b = Q(GQ_BX + d, g);
                if (!(b > 0.0 && b < 1.0 - 1e-12)) continue;
                const int e1 = tang[d][0], e2 = tang[d][1];
                double xf[3] = {0.5, 0.5, 0.5};  // face centroid in mesh units from the cell corner
                xf[d] = 0.0;
                xf[e1] += Q(GQ_FX1 + 2 * d, g);
                xf[e2] += Q(GQ_FX1 + 2 * d + 1, g);
                int lo[3] = {-1, -1, -1}, hi[3] = {1, 1, 1};
                lo[d] = -2;
                int np = 0;
                for (int oz = lo[2]; oz <= hi[2]; ++oz)
                    for (int oy = lo[1]; oy <= hi[1]; ++oy)
                        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                            double vc[3];
                            if (!cell(i + ox, j + oy, k + oz, vc)) continue;
                            const int o3[3] = {ox, oy, oz};
                            for (int a = 0; a < 3; ++a) e[np][a] = (o3[a] + 0.5 + vc[a]) - xf[a];
                            pidx[np] = pos(i + ox, j + oy, k + oz);
                            ++np;
                        }
                lsq_weights(np, e, true, del, W);
                const int op = (int)ocell.size();
                for (int s = 0; s < np; ++s) {
                    idx.push_back(pidx[s]);
                    wts.push_back(W[s][d]);
                }
                off.push_back((int32_t)idx.size());
                ocell.push_back((int32_t)(((int64_t)k * ny + j) * nx + i) | (int32_t)(d << 30));
                dtab[(size_t)g * 7 + d] = op;
                // the same face is the upper d-face of the cell below along d
                const int gl = gid(i - (d == 0), j - (d == 1), k - (d == 2));
                if (gl >= 0) dtab[(size_t)gl * 7 + 3 + d] = op;
            }
            // EB facet (isothermal wall)
            if (cx->diff.eb_mode == 1 && Q(GQ_AREA, g) > 0.0) {
                const double xe[3] = {0.5 + Q(GQ_EBX, g), 0.5 + Q(GQ_EBY, g), 0.5 + Q(GQ_EBZ, g)};
                int np = 0;
                for (int oz = -1; oz <= 1; ++oz)
                    for (int oy = -1; oy <= 1; ++oy)
                        for (int ox = -1; ox <= 1; ++ox) {
                            double vc[3];
                            if (!cell(i + ox, j + oy, k + oz, vc)) continue;
                            const int o3[3] = {ox, oy, oz};
                            for (int a = 0; a < 3; ++a) e[np][a] = (o3[a] + 0.5 + vc[a]) - xe[a];
                            pidx[np] = pos(i + ox, j + oy, k + oz);
                            ++np;
                        }
                lsq_weights(np, e, false, del, W);
                // grad(theta) . (area vector into the fluid, physical)
                const double av[3] = {Q(GQ_AX, g) * del[1] * del[2], Q(GQ_AY, g) * del[0] * del[2],
                                      Q(GQ_AZ, g) * del[0] * del[1]};
                const int op = (int)ocell.size();
                for (int s = 0; s < np; ++s) {
                    idx.push_back(pidx[s]);
                    wts.push_back(W[s][0] * av[0] + W[s][1] * av[1] + W[s][2] * av[2]);
                }
                off.push_back((int32_t)idx.size());
                ocell.push_back((int32_t)(((int64_t)k * ny + j) * nx + i) | (int32_t)(3u << 30));
                dtab[(size_t)g * 7 + 6] = op;
            }
        }
    }
    const int nop = (int)ocell.size();
    if (!reach_ok) {
        cx->err = "a diffusion fit reads a cell above the stored aux range";
        return EBS_E_UNSUPPORTED;
    }
    if ((int64_t)nx * ny * nz > (int64_t)1 << 30) {
        cx->err = "diffusion operators index cells with 30 bits";
        return EBS_E_UNSUPPORTED;
    }
    const size_t np = std::max<size_t>(idx.size(), 1);
    bool ok = hipMalloc(&cx->d_dop_off, sizeof(int32_t) * (nop + 1)) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_dop_idx, sizeof(int32_t) * np) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_dop_w, sizeof(double) * np) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_dop_cell, sizeof(int32_t) * std::max(nop, 1)) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_dflux, sizeof(double) * std::max(nop, 1)) == hipSuccess;
    ok = ok && hipMalloc(&cx->d_dtab, sizeof(int32_t) * 7 * (size_t)G) == hipSuccess;
    if (!ok) {
        cx->err = "diffusion operator allocation failed";
        return EBS_E_OOM;
    }
    EBS_HIP(cx, hipMemcpy(cx->d_dop_off, off.data(), sizeof(int32_t) * (nop + 1), hipMemcpyHostToDevice));
    if (!idx.empty()) {
        EBS_HIP(cx, hipMemcpy(cx->d_dop_idx, idx.data(), sizeof(int32_t) * idx.size(), hipMemcpyHostToDevice));
        EBS_HIP(cx, hipMemcpy(cx->d_dop_w, wts.data(), sizeof(double) * wts.size(), hipMemcpyHostToDevice));
    }
    if (nop > 0) EBS_HIP(cx, hipMemcpy(cx->d_dop_cell, ocell.data(), sizeof(int32_t) * nop, hipMemcpyHostToDevice));
    EBS_HIP(cx, hipMemcpy(cx->d_dtab, dtab.data(), sizeof(int32_t) * 7 * (size_t)G, hipMemcpyHostToDevice));
    cx->ndop = nop;
    cx->ndop_pts = (int64_t)idx.size();
    return EBS_OK;
}

template <typename T>
static DiffArgs<T> diff_args(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt) {
    DiffArgs<T> a;
    a.D = Dims{cx->nx, cx->ny, cx->nz};
    a.v = geo_view(cx);
    a.cur_rho = (const T*)Ucur->rho;
    a.cur_rt = (const T*)Ucur->rhotheta;
    a.out_rt = (T*)Uh->rhotheta;
    a.uhat_rt = cx->d_uhat ? cx->d_uhat + (size_t)cx->G : nullptr;
    a.prim = cx->d_prim;
    a.op_off = cx->d_dop_off;
    a.op_idx = cx->d_dop_idx;
    a.op_w = cx->d_dop_w;
    a.op_cell = cx->d_dop_cell;
    a.flux = cx->d_dflux;
    a.dtab = cx->d_dtab;
    a.nop = cx->ndop;
    a.alpha = cx->diff.alpha_theta;
    a.theta_wall = cx->diff.theta_wall;
    a.cdt = cdt;
    a.dv = cx->g.dx[0] * cx->g.dx[1] * cx->g.dx[2];
    for (int d = 0; d < 3; ++d) a.rdel[d] = 1.0 / cx->g.dx[d];
    return a;
}

template <typename T>
static ebs_status diff_general_t(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt) {
    if (cx->G == 0) return EBS_OK;
    const DiffArgs<T> a = diff_args<T>(cx, Ucur, Uh, cdt);
    if (a.nop > 0)
        hipLaunchKernelGGL(k_diff_ops<T>, dim3(xcd_grid(((int64_t)a.nop * DO_LANES + 255) / 256)), dim3(256), 0,
                           cx->stream, a);
    hipLaunchKernelGGL(k_diff_gen<T>, dim3(xcd_grid((cx->G + 255) / 256)), dim3(256), 0, cx->stream, a);
    EBS_HIP(cx, hipGetLastError());
    return EBS_OK;
}

ebs_status launch_diffusion_general(ebs_ctx* cx, const ebs_state* Ucur, ebs_state* Uh, double cdt) {
    if (cx->g.precision == EBS_F32_BULK) return diff_general_t<float>(cx, Ucur, Uh, cdt);
    return diff_general_t<double>(cx, Ucur, Uh, cdt);
}


}  // namespace ebs
