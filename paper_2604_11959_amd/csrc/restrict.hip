// Restriction (averaging down) of a state onto the grid coarsened by 2, and
// the merged geometry of that grid (Section 4.3: coarse volume and area
// fractions from the fine subcells; cell-centred variables averaged with
// volume weights, face-centred ones with area weights, so that the mass of
// every coarse cell and the mass flux through every coarse face are those of
// the fine cells and faces they cover).
//
// One thread per coarse cell, x fastest: consecutive threads read consecutive
// pairs of fine cells, so the fine state streams through once per launch.  The
// fine geometry is resolved per fine column from the packed column record:
// below the general range every instance is covered, above it every instance
// is regular (fractions 1), inside it the general records hold the values.
// Sums are taken in FP64 for both state precisions.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ebs_internal.h"
#include "stage_common.h"

namespace ebs {
namespace {

template <typename T>
struct RArgs {
    Dims D;   // fine grid
    Dims C;   // coarse grid
    GeoView v;
    const T* in[5];
    T* out[5];         // coarse state (null in geometry mode)
    double* geo_out;   // [4][C cells]: alpha, beta x, y, z of the lower faces (null in state mode)
};

// the four fine lower d-faces on the coarse lower d-face of (I, J, K)
__device__ __forceinline__ void face_child(int d, int I, int J, int K, int u, int w, int& i, int& j, int& k) {
    i = 2 * I + (d == 0 ? 0 : u);
    j = 2 * J + (d == 1 ? 0 : (d == 0 ? u : w));
    k = 2 * K + (d == 2 ? 0 : w);
}

// two adjacent elements (even index) in one load
template <typename T>
struct Pair {
    T x, y;
};
template <typename T>
__device__ __forceinline__ Pair<T> ld2(const T* p, size_t i) {
    using V = typename std::conditional<sizeof(T) == 4, float2, double2>::type;
    const V v = *reinterpret_cast<const V*>(p + i);
    return Pair<T>{(T)v.x, (T)v.y};
}

// fine-cell geometry from the packed record of the cell's column
__device__ __forceinline__ double cgeo(const GeoView& v, const int4& ci, int inst, int q, int k) {
    const int g0 = col_g0(ci);
    if (k < g0) return 0.0;                      // every instance covered
    if (k >= col_g1(ci)) return (q != GQ_ALPHA || cv_plane(v, inst, k)) ? 1.0 : 0.0;  // regular
    return gq(v, inst, q, ci.z + (k - g0));
}

template <typename T>
__global__ void __launch_bounds__(256) k_restrict(RArgs<T> a) {
    const int I = blockIdx.x * blockDim.x + threadIdx.x, J = blockIdx.y, K = blockIdx.z;
    if (I >= a.C.nx) return;
    const size_t oc = ((size_t)K * a.C.ny + J) * a.C.nx + I;
    // the four fine columns (2I + q, 2J + b): every child cell and every fine
    // face on the coarse lower faces lies in one of them
    int4 cr[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int q = 0; q < 2; ++q) cr[b][q] = a.v.col[(2 * J + b) * a.D.nx + 2 * I + q];
    if (a.geo_out) {
        const size_t NC = (size_t)a.C.nx * a.C.ny * a.C.nz;
        double al = 0.0;
        for (int c = 0; c < 2; ++c)
            for (int b = 0; b < 2; ++b)
                for (int q = 0; q < 2; ++q) al += cgeo(a.v, cr[b][q], 0, GQ_ALPHA, 2 * K + c);
        a.geo_out[oc] = al / 8.0;
        for (int d = 0; d < 3; ++d) {
            double sm = 0.0;
            for (int u = 0; u < 2; ++u)
                for (int w = 0; w < 2; ++w) {
                    int i, j, k;
                    face_child(d, I, J, K, u, w, i, j, k);
                    sm += cgeo(a.v, cr[j - 2 * J][i - 2 * I], 0, GQ_BX + d, k);
                }
            a.geo_out[(size_t)(1 + d) * NC + oc] = sm / 4.0;
        }
        return;
    }
    // state loads first (independent of the geometry): pairs along x
    Pair<T> r[2][2], t[2][2], vv[2], ww[2];
    T uu[2][2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const size_t id = ic(a.D, 2 * I, 2 * J + b, 2 * K + c);
            r[c][b] = ld2(a.in[0], id);
            t[c][b] = ld2(a.in[1], id);
            uu[c][b] = a.in[2][iu(a.D, 2 * I, 2 * J + b, 2 * K + c)];
        }
#pragma unroll
    for (int c = 0; c < 2; ++c) vv[c] = ld2(a.in[3], iv(a.D, 2 * I, 2 * J, 2 * K + c));
#pragma unroll
    for (int b = 0; b < 2; ++b) ww[b] = ld2(a.in[4], ic(a.D, 2 * I, 2 * J + b, 2 * K));
    // cell-centred fields: volume weights
    double sw = 0.0, s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double w = cgeo(a.v, cr[b][q], 0, GQ_ALPHA, 2 * K + c);
                if (w > 0.0) {
                    sw += w;
                    s0 += w * (double)(q ? r[c][b].y : r[c][b].x);
                    s1 += w * (double)(q ? t[c][b].y : t[c][b].x);
                }
            }
    put_field<T>(a.C, a.out, 0, I, J, K, (T)(sw > 0.0 ? s0 / sw : 0.0));
    put_field<T>(a.C, a.out, 1, I, J, K, (T)(sw > 0.0 ? s1 / sw : 0.0));
    // momenta on the coarse lower faces: area weights, or the volume
    // fractions of the staggered CVs where the coarse face has no open area
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double val = 0.0;
        if (!(d == 2 && K == 0)) {
            double sb = 0.0, sub = 0.0;
            double xs[2][2];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int w = 0; w < 2; ++w) {
                    int i, j, k;
                    face_child(d, I, J, K, u, w, i, j, k);
                    xs[u][w] = d == 0 ? (double)uu[w][u]
                             : d == 1 ? (double)(u ? vv[w].y : vv[w].x)
                                      : (double)(u ? ww[w].y : ww[w].x);
                    const double bt = cgeo(a.v, cr[j - 2 * J][i - 2 * I], 0, GQ_BX + d, k);
                    if (bt > 0.0) { sb += bt; sub += bt * xs[u][w]; }
                }
            if (sb > 0.0) {
                val = sub / sb;
            } else {
                double sa = 0.0, sua = 0.0;
                for (int u = 0; u < 2; ++u)
                    for (int w = 0; w < 2; ++w) {
                        int i, j, k;
                        face_child(d, I, J, K, u, w, i, j, k);
                        const double al = cgeo(a.v, cr[j - 2 * J][i - 2 * I], d + 1, GQ_ALPHA, k);
                        if (al > 0.0) { sa += al; sua += al * xs[u][w]; }
                    }
                val = sa > 0.0 ? sua / sa : 0.0;
            }
        }
        put_field<T>(a.C, a.out, 2 + d, I, J, K, (T)val);
    }
}

template <typename T>
ebs_status launch_restrict_t(ebs_ctx* cx, const ebs_state* Uf, ebs_state* Uc, double* geo_out) {
    RArgs<T> a;
    a.D = Dims{cx->nx, cx->ny, cx->nz};
    a.C = Dims{cx->nx / 2, cx->ny / 2, cx->nz / 2};
    a.v = geo_view(cx);
    const void* const in[5] = {Uf ? Uf->rho : nullptr, Uf ? Uf->rhotheta : nullptr, Uf ? Uf->rhou : nullptr,
                               Uf ? Uf->rhov : nullptr, Uf ? Uf->rhow : nullptr};
    void* const out[5] = {Uc ? Uc->rho : nullptr, Uc ? Uc->rhotheta : nullptr, Uc ? Uc->rhou : nullptr,
                          Uc ? Uc->rhov : nullptr, Uc ? Uc->rhow : nullptr};
    for (int f = 0; f < 5; ++f) {
        a.in[f] = (const T*)in[f];
        a.out[f] = (T*)out[f];
    }
    a.geo_out = geo_out;
    const dim3 blk(256), grid((a.C.nx + 255) / 256, a.C.ny, a.C.nz);
    hipLaunchKernelGGL(k_restrict<T>, grid, blk, 0, cx->stream, a);
    EBS_HIP(cx, hipGetLastError());
    return EBS_OK;
}

}  // namespace

ebs_status launch_restrict(ebs_ctx* cx, const ebs_state* Uf, ebs_state* Uc, double* geo_out) {
    if (cx->g.precision == EBS_F32_BULK) return launch_restrict_t<float>(cx, Uf, Uc, geo_out);
    return launch_restrict_t<double>(cx, Uf, Uc, geo_out);
}

}  // namespace ebs
