// ebs_coarsened_geometry_noalloc: the merged coarse geometry of Section 4.3
// (the same kernel as ebs_coarsened_geometry) staged through a fixed device
// array instead of a buffer allocated per call, for callers that cannot
// allocate device memory.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy for the life of the process.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in for
// the symbol): the device address of each GPU's copy is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept.  The
// kernel writes every one of the 4 x (coarse cells) entries it stages, so
// nothing has to be cleared between calls.  Calls on one GPU share the array;
// a per-device mutex serialises them within the process for the whole call
// (launch and copies to the host).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ebs_internal.h"

namespace {

constexpr size_t COARSE_MAX = (size_t)EBS_COARSE_GEO_MAX_CELLS;
constexpr int MAX_DEVICES = 64;

// alpha and the three lower-face area fractions of at most COARSE_MAX coarse
// cells (16 MiB)
static __device__ __align__(256) double scratch[4 * COARSE_MAX];

std::mutex g_lock[MAX_DEVICES];
double* g_ptr[MAX_DEVICES] = {nullptr};

ebs_status fail(ebs_ctx* c, ebs_status st, const char* msg) {
    if (c) c->err = msg;
    return st;
}

}  // namespace

extern "C" ebs_status ebs_coarsened_geometry_noalloc(ebs_ctx* c, double* alpha, double* bx, double* by,
                                                     double* bz) {
    if (!c) return EBS_E_ARG;
    if (!alpha || !bx || !by || !bz) return fail(c, EBS_E_ARG, "null output array");
    if ((c->nx | c->ny | c->nz) & 1) return fail(c, EBS_E_UNSUPPORTED, "restriction needs even grid sizes");
    const size_t NC = (size_t)(c->nx / 2) * (c->ny / 2) * (c->nz / 2);
    if (NC > COARSE_MAX)
        return fail(c, EBS_E_UNSUPPORTED,
                    "coarse grid exceeds the static staging buffer (EBS_COARSE_GEO_MAX_CELLS coarse cells)");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    int dev = 0;
    EBS_HIP(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(c, EBS_E_UNSUPPORTED, "device index beyond the library's table");
    std::lock_guard<std::mutex> hold(g_lock[dev]);
    if (!g_ptr[dev]) {
        // first call on this device (current): the address of its copy
        double* p = nullptr;
        EBS_HIP(c, hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(c, EBS_E_HIP, "no device address for the staging buffer");
        g_ptr[dev] = p;
    }
    double* const buf = g_ptr[dev];
    ebs_status st = ebs::launch_restrict(c, nullptr, nullptr, buf);
    if (st != EBS_OK) return st;
    double* const dst[4] = {alpha, bx, by, bz};
    for (int q = 0; q < 4; ++q)
        EBS_HIP(c, hipMemcpyAsync(dst[q], buf + q * NC, sizeof(double) * NC, hipMemcpyDeviceToHost, c->stream));
    EBS_HIP(c, hipStreamSynchronize(c->stream));
    return EBS_OK;
}
