// Shared helpers of the stage kernels (state layout, upwind face value,
// field selection and the write of a field value with its periodic repeat).
#pragma once

#include <hip/hip_runtime.h>

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

}  // namespace
}  // namespace ebs
