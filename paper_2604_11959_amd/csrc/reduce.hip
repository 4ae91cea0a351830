// Conserved sums: sum over the fluid CVs of V * U for each field, accumulated
// in double-double (error-free two-sum) per thread and per block; the block
// partials are combined on the host in a fixed order, so the result does not
// depend on scheduling.
#include <hip/hip_runtime.h>

#include <vector>

#include "ebs_internal.h"

namespace ebs {
namespace {

struct DD {
    double hi, lo;
};

__host__ __device__ inline DD two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__host__ __device__ inline DD dd_add(DD x, double y) {
    DD s = two_sum(x.hi, y);
    s.lo += x.lo;
    return two_sum(s.hi, s.lo);
}

__host__ __device__ inline DD dd_add(DD x, DD y) {
    DD s = two_sum(x.hi, y.hi);
    s.lo += x.lo + y.lo;
    return two_sum(s.hi, s.lo);
}

template <typename T>
struct SumArgs {
    GeoView v;
    const T* f;
    int field;
    int nx, ny, nz;
    double dv;
    double* part;  // [blocks][2]
};

constexpr int SUM_BLOCK = 256;

template <typename T>
__global__ void __launch_bounds__(SUM_BLOCK) k_sum(SumArgs<T> a) {
    const int inst = a.field < 2 ? 0 : a.field - 1;
    const int k0 = inst == 3 ? 1 : 0, k1 = inst == 3 ? a.nz - 1 : a.nz;
    const int64_t n = (int64_t)a.nx * a.ny * (k1 - k0);
    DD acc = {0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % a.nx);
        const int j = (int)((t / a.nx) % a.ny);
        const int k = k0 + (int)(t / ((int64_t)a.nx * a.ny));
        const int g = gidx(a.v, i, j, k);
        double al;
        if (g == -2) continue;
        if (g == -1) {
            al = 1.0;
        } else {
            if (a.v.type[(size_t)inst * a.v.G + g] == 0) continue;
            al = gq(a.v, inst, GQ_ALPHA, g);
        }
        size_t idx;
        if (a.field == 2) idx = ((size_t)k * a.ny + j) * (a.nx + 1) + i;
        else if (a.field == 3) idx = ((size_t)k * (a.ny + 1) + j) * a.nx + i;
        else idx = ((size_t)k * a.ny + j) * a.nx + i;
        acc = dd_add(acc, al * a.dv * (double)a.f[idx]);
    }
    __shared__ double sh[SUM_BLOCK], sl[SUM_BLOCK];
    sh[threadIdx.x] = acc.hi;
    sl[threadIdx.x] = acc.lo;
    __syncthreads();
    for (int s = SUM_BLOCK / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            DD x = {sh[threadIdx.x], sl[threadIdx.x]};
            DD y = {sh[threadIdx.x + s], sl[threadIdx.x + s]};
            DD z = dd_add(x, y);
            sh[threadIdx.x] = z.hi;
            sl[threadIdx.x] = z.lo;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        a.part[2 * blockIdx.x] = sh[0];
        a.part[2 * blockIdx.x + 1] = sl[0];
    }
}

}  // namespace

template <typename T>
static ebs_status sums_t(ebs_ctx* cx, const ebs_state* U, double hi[5], double lo[5]) {
    const void* const fs[5] = {U->rho, U->rhotheta, U->rhou, U->rhov, U->rhow};
    const int blocks = 1024;
    if (!cx->d_part) {
        if (hipMalloc(&cx->d_part, sizeof(double) * 2 * blocks * 5) != hipSuccess) {
            cx->err = "allocation of the sum partials failed";
            return EBS_E_OOM;
        }
    }
    for (int f = 0; f < 5; ++f) {
        SumArgs<T> a;
        a.v = geo_view(cx);
        a.f = (const T*)fs[f];
        a.field = f;
        a.nx = cx->nx;
        a.ny = cx->ny;
        a.nz = cx->nz;
        a.dv = cx->g.dx[0] * cx->g.dx[1] * cx->g.dx[2];
        a.part = cx->d_part + (size_t)2 * blocks * f;
        hipLaunchKernelGGL(k_sum<T>, dim3(blocks), dim3(SUM_BLOCK), 0, cx->stream, a);
        EBS_HIP(cx, hipGetLastError());
    }
    std::vector<double> h((size_t)2 * blocks * 5);
    EBS_HIP(cx, hipMemcpyAsync(h.data(), cx->d_part, sizeof(double) * h.size(), hipMemcpyDeviceToHost,
                               cx->stream));
    EBS_HIP(cx, hipStreamSynchronize(cx->stream));
    for (int f = 0; f < 5; ++f) {
        DD acc = {0.0, 0.0};
        for (int b = 0; b < blocks; ++b) {
            const DD p = {h[(size_t)2 * blocks * f + 2 * b], h[(size_t)2 * blocks * f + 2 * b + 1]};
            acc = dd_add(acc, p);
        }
        hi[f] = acc.hi;
        lo[f] = acc.lo;
    }
    return EBS_OK;
}

ebs_status conserved_sums(ebs_ctx* cx, const ebs_state* U, double hi[5], double lo[5]) {
    if (cx->g.precision == EBS_F32_BULK) return sums_t<float>(cx, U, hi, lo);
    return sums_t<double>(cx, U, hi, lo);
}

}  // namespace ebs
