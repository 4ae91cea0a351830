// C ABI of the ebstag library: argument checks, context lifetime, geometry
// export, the Runge-Kutta driver (with optional HIP-graph capture), timing and
// the tile autotuner.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "ebs_internal.h"

namespace ebs {

ebs_status hip_fail(ebs_ctx* c, hipError_t e, const char* what) {
    if (c) {
        c->err = std::string("HIP error: ") + hipGetErrorString(e) + " in " + what;
    }
    return EBS_E_HIP;
}

GeoView geo_view(const ebs_ctx* c) {
    GeoView v;
    v.nx = c->nx;
    v.ny = c->ny;
    v.nz = c->nz;
    v.dx = c->g.dx[0];
    v.dy = c->g.dx[1];
    v.dz = c->g.dx[2];
    v.lo_z = c->g.lo[2];
    v.G = c->G;
    v.g0 = c->d_g0;
    v.g1 = c->d_g1;
    v.goff = c->d_goff;
    v.gcol = c->d_gcol;
    v.col = c->d_col;
    v.Ge = c->Ge;
    v.gcole = c->d_gcole;
    v.fflag = c->d_fflag;
    v.kf = c->d_kf;
    v.kr = c->d_kr;
    v.geo = c->d_geo;
    v.type = c->d_type;
    v.type4 = c->d_type4;
    return v;
}

}  // namespace ebs

using namespace ebs;

namespace {

bool state_ok(const ebs_state* s) {
    return s && s->rho && s->rhotheta && s->rhou && s->rhov && s->rhow;
}

ebs_status fail(ebs_ctx* c, ebs_status st, const char* msg) {
    if (c) c->err = msg;
    return st;
}

void free_ptr(void* p) {
    if (p) (void)hipFree(p);
}

void drop_graph(ebs_ctx* c) {
    if (c->graph.exec) (void)hipGraphExecDestroy((hipGraphExec_t)c->graph.exec);
    if (c->graph.graph) (void)hipGraphDestroy((hipGraph_t)c->graph.graph);
    c->graph.exec = nullptr;
    c->graph.graph = nullptr;
}

bool same_state(const ebs_state& a, const ebs_state& b) { return std::memcmp(&a, &b, sizeof(a)) == 0; }

// bytes of each state array (rho, rhotheta, rhou, rhov, rhow) of the context's grid
void field_bytes(const ebs_ctx* c, size_t out[5]) {
    const size_t es = c->g.precision == EBS_F32_BULK ? 4 : 8;
    const size_t nx = c->nx, ny = c->ny, nz = c->nz;
    out[0] = out[1] = es * nx * ny * nz;
    out[2] = es * (nx + 1) * ny * nz;
    out[3] = es * nx * (ny + 1) * nz;
    out[4] = es * nx * ny * (nz + 1);
}

const void* field_ptr(const ebs_state* s, int f) {
    const void* const p[5] = {s->rho, s->rhotheta, s->rhou, s->rhov, s->rhow};
    return p[f];
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Does any array of `out` overlap an array of `in`?  With same_ok, array f
// of out may coincide exactly with array f of in (an in-place update that
// reads each element before the same thread writes it).
bool states_overlap(const ebs_ctx* c, const ebs_state* out, const ebs_state* in, bool same_ok) {
    size_t nb[5];
    field_bytes(c, nb);
    for (int f = 0; f < 5; ++f)
        for (int g = 0; g < 5; ++g) {
            if (same_ok && f == g && field_ptr(out, f) == field_ptr(in, g)) continue;
            if (ranges_overlap(field_ptr(out, f), nb[f], field_ptr(in, g), nb[g])) return true;
        }
    return false;
}

// do two arrays of one state overlap
bool state_self_overlap(const ebs_ctx* c, const ebs_state* s) {
    size_t nb[5];
    field_bytes(c, nb);
    for (int f = 0; f < 5; ++f)
        for (int g = f + 1; g < 5; ++g)
            if (ranges_overlap(field_ptr(s, f), nb[f], field_ptr(s, g), nb[g])) return true;
    return false;
}

ebs_status rk3_enqueue(ebs_ctx* c, ebs_state* U, ebs_state* S, double dt) {
    static const double cs[3] = {1.0 / 3.0, 0.5, 1.0};
    ebs_state* cur = U;
    ebs_state* outs[3] = {&S[0], &S[1], U};
    for (int s = 0; s < 3; ++s) {
        // the redistribution only touches general-range cells, so it runs while
        // the regular-region kernel of the same stage may still be running
        ebs_status st = launch_advance(c, U, cur, outs[s], cs[s] * dt, true);
        if (st != EBS_OK) return st;
        st = launch_redistribute(c, outs[s], outs[s]);
        if (st != EBS_OK) return st;
        st = join_side(c);
        if (st != EBS_OK) return st;
        cur = outs[s];
    }
    return EBS_OK;
}

}  // namespace

extern "C" {

const char* ebs_last_error(const ebs_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

ebs_status ebs_create(const ebs_grid* grid, const ebs_box* boxes, int32_t nbox, void* hip_stream,
                      ebs_ctx** out) {
    if (!grid || !out) return EBS_E_ARG;
    *out = nullptr;
    const ebs_grid& g = *grid;
    if (g.n[0] < 8 || g.n[1] < 8 || g.n[2] < 4 || g.n[2] > 32767) return EBS_E_ARG;
    if ((int64_t)g.n[0] * g.n[1] * g.n[2] > (int64_t)1 << 31) return EBS_E_UNSUPPORTED;
    // every field array must stay below 4 GiB (32-bit byte offsets in the kernels)
    const int64_t es = g.precision == EBS_F32_BULK ? 4 : 8;
    if ((int64_t)(g.n[0] + 1) * (g.n[1] + 1) * (g.n[2] + 1) * es >= ((int64_t)1 << 32)) return EBS_E_UNSUPPORTED;
    for (int d = 0; d < 3; ++d)
        if (!(g.dx[d] > 0.0) || !isfinite(g.dx[d]) || !isfinite(g.lo[d])) return EBS_E_ARG;
    if (!(g.small_vfrac > 0.0 && g.small_vfrac < 1.0)) return EBS_E_ARG;
    if (g.precision != EBS_F64 && g.precision != EBS_F32_BULK) return EBS_E_ARG;
    if (g.limiter < 0 || g.limiter > 2 || g.eb_flux < 0 || g.eb_flux > 1) return EBS_E_ARG;
    if ((g.periodic & 0x7u) != 0x3u) return EBS_E_UNSUPPORTED;
    if (nbox < 0 || (nbox > 0 && !boxes)) return EBS_E_ARG;
    ebs_ctx* c = new (std::nothrow) ebs_ctx();
    if (!c) return EBS_E_OOM;
    c->g = g;
    c->nx = g.n[0];
    c->ny = g.n[1];
    c->nz = g.n[2];
    c->ncol = c->nx * c->ny;
    c->stream = (hipStream_t)hip_stream;
    if (g.precision == EBS_F64) {  // double LDS rings: smaller default tile
        c->tile_x = 16;
        c->tile_y = 4;
    }
    if (nbox == 0) {
        ebs_box b = {{0, 0, 0}, {c->nx, c->ny, c->nz}};
        c->boxes.push_back(b);
    } else {
        // the boxes must tile the domain exactly once
        std::vector<uint8_t> cover((size_t)c->nx * c->ny * c->nz, 0);
        for (int b = 0; b < nbox; ++b) {
            const ebs_box& B = boxes[b];
            for (int d = 0; d < 3; ++d)
                if (B.lo[d] < 0 || B.hi[d] > g.n[d] || B.lo[d] >= B.hi[d]) {
                    delete c;
                    return EBS_E_ARG;
                }
            for (int k = B.lo[2]; k < B.hi[2]; ++k)
                for (int j = B.lo[1]; j < B.hi[1]; ++j)
                    for (int i = B.lo[0]; i < B.hi[0]; ++i) {
                        uint8_t& v = cover[((size_t)k * c->ny + j) * c->nx + i];
                        if (v) {
                            delete c;
                            return EBS_E_ARG;
                        }
                        v = 1;
                    }
            c->boxes.push_back(B);
        }
        for (uint8_t v : cover)
            if (!v) {
                delete c;
                return EBS_E_ARG;
            }
    }
    // LDS a block may use (the regular-region tiles are checked against it)
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, 0) == hipSuccess && lds_max > 0)
        c->lds_max = lds_max;
    // side stream (default priority) and fork / join events for running the
    // regular-region kernel concurrently with the general range
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        ebs_destroy(c);
        return EBS_E_HIP;
    }
    const size_t ncol = c->ncol;
    bool ok = hipMalloc(&c->d_kf, sizeof(int32_t) * NINST * ncol) == hipSuccess;
    ok = ok && hipMalloc(&c->d_kr, sizeof(int32_t) * NINST * ncol) == hipSuccess;
    ok = ok && hipMalloc(&c->d_g0, sizeof(int32_t) * ncol) == hipSuccess;
    ok = ok && hipMalloc(&c->d_g1, sizeof(int32_t) * ncol) == hipSuccess;
    if (!ok) {
        ebs_destroy(c);
        return EBS_E_OOM;
    }
    *out = c;
    return EBS_OK;
}

ebs_status ebs_destroy(ebs_ctx* c) {
    if (!c) return EBS_OK;
    drop_graph(c);
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    if (c->side) (void)hipStreamDestroy(c->side);
    void* ptrs[] = {c->d_kf,   c->d_kr,        c->d_g0,      c->d_g1,   c->d_goff, c->d_gcol,
                    c->d_geo,  c->d_type,      c->d_mask,    c->d_small, c->d_tier, c->d_w,
                    c->d_smalllist, c->d_actlist, c->d_lsq_off, c->d_lsq_idx, c->d_lsq_c, c->d_lsq_ev, c->d_lsq_nev, c->d_wl_off, c->d_wl_idx, c->d_wl_geo, c->d_wl_self, c->d_wl_small, c->d_uhat, c->d_qhat, c->d_sig,  c->d_tiles, c->d_prim, c->d_fh, c->d_type4, c->d_col, c->d_gcole, c->d_fflag, c->d_cbase, c->d_cut_n, c->d_cut_w, c->d_bfc,
                    c->d_ptab, c->d_ftab, c->d_utab, c->d_sten, c->d_upd, c->d_q_idx, c->d_q_w, c->d_q_den, c->d_q_n, c->d_chk, c->d_part, c->d_dummy,
                    c->d_srcf, c->d_srcd, c->d_srcv, c->d_dop_off, c->d_dop_idx, c->d_dop_w, c->d_dop_cell,
                    c->d_dflux, c->d_dtab, c->d_vop_off, c->d_vop_pt, c->d_vop_w, c->d_vflux,
                    c->d_vtab, c->d_acol};
    for (void* p : ptrs) free_ptr(p);
    delete c;
    return EBS_OK;
}

// Everything after the upload of a validated terrain (d_h) or level set
// (d_phi), both device arrays.
static ebs_status build_from(ebs_ctx* c, const double* d_h, const double* d_phi) {
    // The build replaces every table the stages read.  Work queued on the
    // context's streams may still read them, and a graph captured on the old
    // tables must never be replayed: wait, drop the graph, and leave the
    // context without geometry until the whole build has succeeded.
    EBS_HIP(c, hipStreamSynchronize(c->stream));
    if (c->side) EBS_HIP(c, hipStreamSynchronize(c->side));
    c->join_pending = false;
    drop_graph(c);
    c->have_geom = false;
    c->have_adv = false;
    // The general range is built three times at most: with the footprint of
    // the small CVs (mode 1), then with the cells the resulting redistribution
    // tables actually touch (mode 2).  The set-up steps check that every
    // stencil, interpolation and redistribution read stays inside the range;
    // a check that fails falls back to the previous mode (mode 0 takes every
    // CV below kr as possibly small).  ebs_set_range_rule caps the strictest
    // mode tried.
    auto build_all = [&](int mode) -> ebs_status {
        c->range_mode = mode;
        ebs_status r = build_geometry(c, d_h, d_phi);
        (void)hipStreamSynchronize(c->stream);
        if (r == EBS_OK) r = build_cut_faces(c);
        if (r == EBS_OK) r = build_stencils(c);
        if (r == EBS_OK) r = wsrd_setup(c);
        return r;
    };
    ebs_status st = build_all(std::min(c->range_rule, 1));
    if (st == EBS_OK && c->range_rule == 2) {
        std::vector<int32_t> ftop;
        st = redistribution_tops(c, ftop);
        if (st == EBS_OK) {
            c->h_ftop.swap(ftop);
            st = build_all(2);
            if (st == EBS_E_UNSUPPORTED) st = build_all(1);
        }
    }
    if (st == EBS_E_UNSUPPORTED && c->range_mode != 0) st = build_all(0);
    if (st != EBS_OK) return st;
    st = build_tiles(c);
    if (st != EBS_OK) return st;
    if (c->diff_on) {
        st = build_diffusion(c);
        if (st != EBS_OK) return st;
    }
    if (c->visc_on) {
        st = build_viscous(c);
        if (st != EBS_OK) return st;
    }
    EBS_HIP(c, hipStreamSynchronize(c->stream));
    c->have_geom = true;
    return EBS_OK;
}

ebs_status ebs_build_geometry_terrain(ebs_ctx* c, const double* h_nodes, int32_t on_device) {
    if (!c || !h_nodes) return fail(c, EBS_E_ARG, "null argument");
    const size_t nn = (size_t)(c->nx + 1) * (c->ny + 1);
    std::vector<double> h(nn);
    if (on_device) {
        EBS_HIP(c, hipMemcpy(h.data(), h_nodes, sizeof(double) * nn, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(h.data(), h_nodes, sizeof(double) * nn);
    }
    const double ztop_clear = c->g.lo[2] + (double)(c->nz - 1) * c->g.dx[2];
    for (size_t q = 0; q < nn; ++q) {
        if (!isfinite(h[q])) return fail(c, EBS_E_ARG, "non-finite terrain height");
        if (!(h[q] < ztop_clear)) return fail(c, EBS_E_ARG, "terrain reaches the top cell layer");
    }
    const int W = c->nx + 1;
    for (int j = 0; j <= c->ny; ++j)
        if (h[(size_t)j * W + c->nx] != h[(size_t)j * W]) return fail(c, EBS_E_ARG, "terrain not periodic in x");
    for (int i = 0; i <= c->nx; ++i)
        if (h[(size_t)c->ny * W + i] != h[i]) return fail(c, EBS_E_ARG, "terrain not periodic in y");
    double* d_h = nullptr;
    if (hipMalloc(&d_h, sizeof(double) * nn) != hipSuccess) return fail(c, EBS_E_OOM, "terrain upload");
    hipError_t e = hipMemcpy(d_h, h.data(), sizeof(double) * nn, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d_h);
        return hip_fail(c, e, "terrain upload");
    }
    const ebs_status st = build_from(c, d_h, nullptr);
    (void)hipFree(d_h);
    return st;
}

ebs_status ebs_build_geometry_levelset(ebs_ctx* c, const double* phi_nodes, int32_t on_device) {
    if (!c || !phi_nodes) return fail(c, EBS_E_ARG, "null argument");
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const size_t plane = (size_t)(nx + 1) * (ny + 1), nn = plane * (nz + 1);
    std::vector<double> f(nn);
    if (on_device) {
        EBS_HIP(c, hipMemcpy(f.data(), phi_nodes, sizeof(double) * nn, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(f.data(), phi_nodes, sizeof(double) * nn);
    }
    for (size_t q = 0; q < nn; ++q)
        if (!isfinite(f[q])) return fail(c, EBS_E_ARG, "non-finite level set");
    const int W = nx + 1;
    for (int k = 0; k <= nz; ++k) {
        const double* P = f.data() + (size_t)k * plane;
        for (int j = 0; j <= ny; ++j)
            if (P[(size_t)j * W + nx] != P[(size_t)j * W]) return fail(c, EBS_E_ARG, "level set not periodic in x");
        for (int i = 0; i <= nx; ++i)
            if (P[(size_t)ny * W + i] != P[i]) return fail(c, EBS_E_ARG, "level set not periodic in y");
    }
    for (size_t q = 0; q < plane; ++q)
        if (!(f[(size_t)(nz - 1) * plane + q] > 0.0)) return fail(c, EBS_E_ARG, "level set reaches the top cell layer");
    for (int k = 0; k < nz; ++k)
        for (size_t q = 0; q < plane; ++q)
            if (!(f[(size_t)(k + 1) * plane + q] >= f[(size_t)k * plane + q]))
                return fail(c, EBS_E_UNSUPPORTED, "level set decreases along z (the column structure needs it nondecreasing)");
    double* d_phi = nullptr;
    if (hipMalloc(&d_phi, sizeof(double) * nn) != hipSuccess) return fail(c, EBS_E_OOM, "level-set upload");
    hipError_t e = hipMemcpy(d_phi, f.data(), sizeof(double) * nn, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d_phi);
        return hip_fail(c, e, "level-set upload");
    }
    const ebs_status st = build_from(c, nullptr, d_phi);
    (void)hipFree(d_phi);
    return st;
}

ebs_status ebs_build_geometry_merged(ebs_ctx* c, const double* fine_nodes, int32_t kind, int32_t on_device) {
    if (!c || !fine_nodes) return fail(c, EBS_E_ARG, "null argument");
    if (kind != 0 && kind != 1) return fail(c, EBS_E_ARG, "kind must be 0 (terrain) or 1 (level set)");
    const int nx = 2 * c->nx, ny = 2 * c->ny, nz = 2 * c->nz;
    const size_t plane = (size_t)(nx + 1) * (ny + 1), nn = kind == 0 ? plane : plane * (nz + 1);
    std::vector<double> f(nn);
    if (on_device) {
        EBS_HIP(c, hipMemcpy(f.data(), fine_nodes, sizeof(double) * nn, hipMemcpyDeviceToHost));
    } else {
        std::memcpy(f.data(), fine_nodes, sizeof(double) * nn);
    }
    for (size_t q = 0; q < nn; ++q)
        if (!isfinite(f[q])) return fail(c, EBS_E_ARG, "non-finite fine nodal value");
    const int W = nx + 1;
    const int nplanes = kind == 0 ? 1 : nz + 1;
    for (int k = 0; k < nplanes; ++k) {
        const double* P = f.data() + (size_t)k * plane;
        for (int j = 0; j <= ny; ++j)
            if (P[(size_t)j * W + nx] != P[(size_t)j * W]) return fail(c, EBS_E_ARG, "fine nodes not periodic in x");
        for (int i = 0; i <= nx; ++i)
            if (P[(size_t)ny * W + i] != P[i]) return fail(c, EBS_E_ARG, "fine nodes not periodic in y");
    }
    if (kind == 0) {
        const double ztop_clear = c->g.lo[2] + (double)(c->nz - 1) * c->g.dx[2];
        for (size_t q = 0; q < nn; ++q)
            if (!(f[q] < ztop_clear)) return fail(c, EBS_E_ARG, "terrain reaches the top cell layer");
    } else {
        // the coarse top layer starts at fine node plane nz - 2
        for (size_t q = 0; q < plane; ++q)
            if (!(f[(size_t)(nz - 2) * plane + q] > 0.0)) return fail(c, EBS_E_ARG, "level set reaches the top cell layer");
        for (int k = 0; k < nz; ++k)
            for (size_t q = 0; q < plane; ++q)
                if (!(f[(size_t)(k + 1) * plane + q] >= f[(size_t)k * plane + q]))
                    return fail(c, EBS_E_UNSUPPORTED, "level set decreases along z (the column structure needs it nondecreasing)");
    }
    double* d_f = nullptr;
    if (hipMalloc(&d_f, sizeof(double) * nn) != hipSuccess) return fail(c, EBS_E_OOM, "fine node upload");
    hipError_t e = hipMemcpy(d_f, f.data(), sizeof(double) * nn, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(d_f);
        return hip_fail(c, e, "fine node upload");
    }
    c->geo_merged = 1;
    const ebs_status st = kind == 0 ? build_from(c, d_f, nullptr) : build_from(c, nullptr, d_f);
    c->geo_merged = 0;
    (void)hipFree(d_f);
    return st;
}

ebs_status ebs_geometry_export(ebs_ctx* c, int32_t inst, int32_t qty, double* host, size_t n) {
    if (!c || !host) return fail(c, EBS_E_ARG, "null argument");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    if (inst < 0 || inst > 3 || qty < 0 || qty >= EBS_Q_COUNT) return fail(c, EBS_E_ARG, "bad instance or quantity");
    const int nx = c->nx, ny = c->ny, nz = c->nz;
    const int ex = nx + (inst == 1), ey = ny + (inst == 2), ez = nz + (inst == 3);
    if (n != (size_t)ex * ey * ez) return fail(c, EBS_E_ARG, "wrong element count");
    const size_t G = std::max(c->G, 1);
    std::vector<double> geo, w;
    std::vector<int8_t> ty, sm, tr;
    std::vector<int32_t> mk;
    std::vector<int32_t> kf(c->ncol), kr(c->ncol);
    EBS_HIP(c, hipMemcpy(kf.data(), c->d_kf + (size_t)inst * c->ncol, sizeof(int32_t) * c->ncol, hipMemcpyDeviceToHost));
    EBS_HIP(c, hipMemcpy(kr.data(), c->d_kr + (size_t)inst * c->ncol, sizeof(int32_t) * c->ncol, hipMemcpyDeviceToHost));
    if (c->G > 0) {
        if (qty < GQ_N) {
            geo.resize(G);
            EBS_HIP(c, hipMemcpy(geo.data(), c->d_geo + ((size_t)inst * GQ_N + qty) * c->G, sizeof(double) * c->G, hipMemcpyDeviceToHost));
        }
        ty.resize(G);
        EBS_HIP(c, hipMemcpy(ty.data(), c->d_type + (size_t)inst * c->G, c->G, hipMemcpyDeviceToHost));
        if (qty > EBS_Q_TYPE) {
            sm.resize(G); tr.resize(G); mk.resize(G);
            w.resize((size_t)WQ_COUNT * G);
            EBS_HIP(c, hipMemcpy(sm.data(), c->d_small + (size_t)inst * c->G, c->G, hipMemcpyDeviceToHost));
            EBS_HIP(c, hipMemcpy(tr.data(), c->d_tier + (size_t)inst * c->G, c->G, hipMemcpyDeviceToHost));
            EBS_HIP(c, hipMemcpy(mk.data(), c->d_mask + (size_t)inst * c->G, sizeof(int32_t) * c->G, hipMemcpyDeviceToHost));
            EBS_HIP(c, hipMemcpy(w.data(), c->d_w + (size_t)inst * WQ_COUNT * c->G, sizeof(double) * WQ_COUNT * c->G, hipMemcpyDeviceToHost));
        }
    }
    auto value = [&](int i, int j, int k) -> double {
        const bool cv = inst == 3 ? (k >= 1 && k <= nz - 1) : (k <= nz - 1);
        if (!cv) return 0.0;
        const int col = j * nx + i;
        const int a = c->h_g0[col], b = c->h_g1[col];
        int t;  // type
        int gi = -1;
        if (k < a) t = 0;
        else if (k >= b) t = 1;
        else { gi = c->h_goff[col] + (k - a); t = ty[gi]; }
        if (qty == EBS_Q_TYPE) return t;
        if (qty < GQ_N) {
            if (gi >= 0) return geo[gi];
            if (t == 0) return 0.0;
            return (qty == GQ_ALPHA || qty == GQ_BX || qty == GQ_BY || qty == GQ_BZ) ? 1.0 : 0.0;
        }
        if (t == 0) return 0.0;
        if (gi < 0) {  // regular CV outside the general range: trivial neighbourhood
            switch (qty) {
                case EBS_Q_MASK: return (double)(1 << 13);
                case EBS_Q_NCOUNT: return 1.0;
                case EBS_Q_OMEGA: return 1.0;
                case EBS_Q_VHAT: return 1.0;
                default: return 0.0;
            }
        }
        switch (qty) {
            case EBS_Q_SMALL: return sm[gi];
            case EBS_Q_TIER: return tr[gi];
            case EBS_Q_MASK: return (double)mk[gi];
            case EBS_Q_NCOUNT: return w[(size_t)WQ_N * G + gi];
            case EBS_Q_KAPPA: return w[(size_t)WQ_KAPPA * G + gi];
            case EBS_Q_OMEGA: return w[(size_t)WQ_OMEGA * G + gi];
            case EBS_Q_VHAT: return w[(size_t)WQ_VHAT * G + gi];
            case EBS_Q_XHAT_X: return w[(size_t)WQ_XHX * G + gi];
            case EBS_Q_XHAT_Y: return w[(size_t)WQ_XHY * G + gi];
            default: return w[(size_t)WQ_XHZ * G + gi];
        }
    };
    (void)kf; (void)kr;
    for (int k = 0; k < ez; ++k)
        for (int j = 0; j < ey; ++j)
            for (int i = 0; i < ex; ++i)
                host[((size_t)k * ey + j) * ex + i] = value(i % nx, j % ny, k);
    return EBS_OK;
}

ebs_status ebs_geometry_stats(ebs_ctx* c, int64_t* out) {
    if (!c || !out) return fail(c, EBS_E_ARG, "null argument");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    const size_t G = c->G;
    std::vector<int8_t> ty(std::max<size_t>(G, 1)), sm(std::max<size_t>(G, 1)), tr(std::max<size_t>(G, 1));
    for (int inst = 0; inst < NINST; ++inst) {
        int64_t* o = out + 8 * inst;
        for (int q = 0; q < 8; ++q) o[q] = 0;
        if (G > 0) {
            EBS_HIP(c, hipMemcpy(ty.data(), c->d_type + inst * G, G, hipMemcpyDeviceToHost));
            EBS_HIP(c, hipMemcpy(sm.data(), c->d_small + inst * G, G, hipMemcpyDeviceToHost));
            EBS_HIP(c, hipMemcpy(tr.data(), c->d_tier + inst * G, G, hipMemcpyDeviceToHost));
        }
        for (size_t g = 0; g < G; ++g) {
            if (ty[g] == 2) o[0]++;
            if (sm[g]) o[1]++;
            if (ty[g] == 0) o[2]++;
            if (tr[g] >= 1 && tr[g] <= 3) o[2 + tr[g]]++;
            if (ty[g] == 1) o[7]++;
        }
        o[6] = (int64_t)G;
        // covered and regular CVs outside the general range
        const int kmin = inst == 3 ? 1 : 0, kmax = c->nz - 1;
        for (int col = 0; col < c->ncol; ++col) {
            o[2] += std::max(0, std::min(c->h_g0[col], kmax + 1) - kmin);
            o[7] += std::max(0, kmax + 1 - std::max(c->h_g1[col], kmin));
        }
    }
    return EBS_OK;
}

ebs_status ebs_alpha_histogram(ebs_ctx* c, int32_t inst, const double* edges, int32_t nbins, int64_t* counts) {
    if (!c || !edges || !counts) return fail(c, EBS_E_ARG, "null argument");
    if (inst < 0 || inst > 3 || nbins < 1) return fail(c, EBS_E_ARG, "bad instance or bin count");
    for (int b = 0; b < nbins; ++b)
        if (!(edges[b] < edges[b + 1])) return fail(c, EBS_E_ARG, "bin edges must increase");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    for (int b = 0; b < nbins; ++b) counts[b] = 0;
    // bin of a fluid volume fraction a: [edges[b], edges[b+1]), the last bin closed
    auto put = [&](double a, int64_t n) {
        if (n <= 0 || a < edges[0] || a > edges[nbins]) return;
        int b = (int)(std::upper_bound(edges, edges + nbins + 1, a) - edges) - 1;
        if (b >= nbins) b = nbins - 1;
        counts[b] += n;
    };
    if (c->G > 0) {
        std::vector<double> al((size_t)c->G);
        std::vector<int8_t> ty((size_t)c->G);
        EBS_HIP(c, hipMemcpy(al.data(), c->d_geo + ((size_t)inst * GQ_N + GQ_ALPHA) * c->G, sizeof(double) * c->G,
                             hipMemcpyDeviceToHost));
        EBS_HIP(c, hipMemcpy(ty.data(), c->d_type + (size_t)inst * c->G, c->G, hipMemcpyDeviceToHost));
        for (size_t g = 0; g < (size_t)c->G; ++g)
            if (ty[g] != 0) put(al[g], 1);
    }
    // regular CVs above the general range (alpha = 1); below it every CV is covered
    const int kmin = inst == 3 ? 1 : 0, kmax = c->nz - 1;
    int64_t reg = 0;
    for (int col = 0; col < c->ncol; ++col) reg += std::max(0, kmax + 1 - std::max(c->h_g1[col], kmin));
    put(1.0, reg);
    return EBS_OK;
}

ebs_status ebs_advance_stage(ebs_ctx* c, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uhat, double cdt) {
    if (!c) return EBS_E_ARG;
    if (!state_ok(Un) || !state_ok(Ucur) || !state_ok(Uhat)) return fail(c, EBS_E_ARG, "null state pointer");
    if (!isfinite(cdt)) return fail(c, EBS_E_ARG, "non-finite time step");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    // the stencil reads neighbours of Ucur while other threads write Uhat, so
    // no array of Uhat may overlap any array of Ucur; Uhat may coincide with
    // Un field by field (each element of Un is read only by the thread that
    // writes the same element of Uhat), but not overlap it otherwise
    if (state_self_overlap(c, Uhat)) return fail(c, EBS_E_ARG, "output arrays overlap each other");
    if (states_overlap(c, Uhat, Ucur, false)) return fail(c, EBS_E_ARG, "output overlaps the stencil input");
    if (states_overlap(c, Uhat, Un, true)) return fail(c, EBS_E_ARG, "output partly overlaps U^n");
    const ebs_status st = launch_advance(c, Un, Ucur, Uhat, cdt);
    c->have_adv = st == EBS_OK;
    if (st == EBS_OK) c->last_uhat = *Uhat;
    return st;
}

ebs_status ebs_redistribute(ebs_ctx* c, const ebs_state* Uhat, ebs_state* Uout) {
    if (!c) return EBS_E_ARG;
    if (!state_ok(Uhat) || !state_ok(Uout)) return fail(c, EBS_E_ARG, "null state pointer");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    // the cut range is redistributed from the FP64 copy the last advance kept
    if (!c->have_adv || !same_state(*Uhat, c->last_uhat))
        return fail(c, EBS_E_ORDER, "Uhat is not the output of the last ebs_advance_stage");
    if (state_self_overlap(c, Uout)) return fail(c, EBS_E_ARG, "output arrays overlap each other");
    if (states_overlap(c, Uout, Uhat, true)) return fail(c, EBS_E_ARG, "output partly overlaps Uhat");
    return launch_redistribute(c, Uhat, Uout);
}

ebs_status ebs_rk3_step(ebs_ctx* c, ebs_state* U, ebs_state* scratch, double dt, int32_t use_graph) {
    if (!c) return EBS_E_ARG;
    if (!state_ok(U) || !scratch || !state_ok(&scratch[0]) || !state_ok(&scratch[1]))
        return fail(c, EBS_E_ARG, "null state pointer");
    if (!isfinite(dt)) return fail(c, EBS_E_ARG, "non-finite time step");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    // U, S0 and S1 serve as stage inputs and outputs in turn: they must be
    // three disjoint states
    if (state_self_overlap(c, U) || state_self_overlap(c, &scratch[0]) || state_self_overlap(c, &scratch[1]) ||
        states_overlap(c, U, &scratch[0], false) || states_overlap(c, U, &scratch[1], false) ||
        states_overlap(c, &scratch[0], &scratch[1], false))
        return fail(c, EBS_E_ARG, "U and the two scratch states must not overlap");
    // the stages overwrite the provisional copy ebs_redistribute reads
    c->have_adv = false;
    if (!use_graph || c->timing) return rk3_enqueue(c, U, scratch, dt);
    const bool hit = c->graph.exec && same_state(c->graph.U, *U) && same_state(c->graph.S0, scratch[0]) &&
                     same_state(c->graph.S1, scratch[1]) && c->graph.dt == dt;
    if (!hit) {
        drop_graph(c);
        hipStream_t s = c->stream;
        bool own = false;
        if (!s) {  // the legacy null stream cannot be captured
            EBS_HIP(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            own = true;
        }
        hipStream_t saved = c->stream;
        c->stream = s;
        EBS_HIP(c, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        ebs_status st = rk3_enqueue(c, U, scratch, dt);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        c->stream = saved;
        if (st != EBS_OK) return st;
        if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return hip_fail(c, e, "hipGraphInstantiate");
        }
        if (own) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
        c->graph.graph = graph;
        c->graph.exec = exec;
        c->graph.U = *U;
        c->graph.S0 = scratch[0];
        c->graph.S1 = scratch[1];
        c->graph.dt = dt;
    }
    EBS_HIP(c, hipGraphLaunch((hipGraphExec_t)c->graph.exec, c->stream));
    return EBS_OK;
}

ebs_status ebs_conserved_sums(ebs_ctx* c, const ebs_state* U, double hi[5], double lo[5]) {
    if (!c || !hi || !lo) return EBS_E_ARG;
    if (!state_ok(U)) return fail(c, EBS_E_ARG, "null state pointer");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    return conserved_sums(c, U, hi, lo);
}

ebs_status ebs_set_tile(ebs_ctx* c, int32_t tx, int32_t ty, int32_t tz, int32_t span) {
    if (!c) return EBS_E_ARG;
    if (!(tx == 16 || tx == 32 || tx == 64) || !(ty == 2 || ty == 4 || ty == 8 || ty == 16) ||
        tx * ty < 64 || tx * ty > 1024)
        return fail(c, EBS_E_ARG, "unsupported tile shape");
    if (!(tz == 0 || tz == 16 || tz == 32 || tz == 64 || tz == 128 || tz == 256))
        return fail(c, EBS_E_ARG, "unsupported tile height");
    if (span != 0 && span != 1) return fail(c, EBS_E_ARG, "tile span must be 0 or 1");
    if ((tx + 5) * (ty + 5) > 4 * tx * ty)
        return fail(c, EBS_E_ARG, "tile shape has more halo points than the block covers");
    if (bulk_lds_bytes(tx, ty, c->g.precision, c->src_on) > (size_t)c->lds_max)
        return fail(c, EBS_E_ARG, "tile shape needs more LDS than a block may use");
    c->tile_x = tx;
    c->tile_y = ty;
    if (tz) c->tile_z = tz;
    c->tile_span = span;
    drop_graph(c);
    if (c->have_geom) return build_tiles(c);
    return EBS_OK;
}

ebs_status ebs_set_sources(ebs_ctx* c, const ebs_source_params* prm, const double* rt0, const double* rho0) {
    if (!c) return EBS_E_ARG;
    if (!prm) {
        if (c->src_on) drop_graph(c);
        c->src_on = false;
        return EBS_OK;
    }
    if (!rt0 || !rho0) return fail(c, EBS_E_ARG, "null reference-state array");
    const ebs_source_params q = *prm;
    if (!(q.P00 > 0 && std::isfinite(q.P00)) || !(q.R > 0 && std::isfinite(q.R)) ||
        !(q.gamma > 1 && std::isfinite(q.gamma)) || !(q.g >= 0 && std::isfinite(q.g)))
        return fail(c, EBS_E_ARG, "source constants out of range");
    if (c->g.eb_flux != EBS_EB_WALL) return fail(c, EBS_E_UNSUPPORTED, "sources need the no-flux EB closure");
    if (bulk_lds_bytes(c->tile_x, c->tile_y, c->g.precision, true) > (size_t)c->lds_max)
        return fail(c, EBS_E_UNSUPPORTED, "the tile shape leaves no LDS for the pressure planes");
    const int nz = c->nz;
    // per level: p0 (the equation-of-state pressure of rho theta0), rho
    // theta0 (split into a part exact in the state precision and the rest),
    // 1 / rho theta0, rho0; p' = p0 ((rho theta / rho theta0)^gamma - 1)
    std::vector<double> td((size_t)5 * nz);
    std::vector<float> tf((size_t)5 * nz);
    for (int k = 0; k < nz; ++k) {
        if (!(rt0[k] > 0 && std::isfinite(rt0[k])) || !(rho0[k] > 0 && std::isfinite(rho0[k])))
            return fail(c, EBS_E_ARG, "reference state must be positive and finite");
        const double p0 = q.P00 * std::pow(q.R * rt0[k] / q.P00, q.gamma);
        td[0 * nz + k] = p0;
        td[1 * nz + k] = rt0[k];
        td[2 * nz + k] = 0.0;
        td[3 * nz + k] = 1.0 / rt0[k];
        td[4 * nz + k] = rho0[k];
        const float hi = (float)rt0[k];
        tf[0 * nz + k] = (float)p0;
        tf[1 * nz + k] = hi;
        tf[2 * nz + k] = (float)(rt0[k] - (double)hi);
        tf[3 * nz + k] = (float)(1.0 / rt0[k]);
        tf[4 * nz + k] = (float)rho0[k];
    }
    if (!c->d_srcd && hipMalloc(&c->d_srcd, sizeof(double) * 5 * nz) != hipSuccess) {
        c->d_srcd = nullptr;
        return fail(c, EBS_E_OOM, "source tables");
    }
    // FP32 power table after the level values (see pprime in bulk.hip): for
    // m = -32..32, R' = 2^(-m/8) in FP32, R' - 1, c = R'^(-gamma), c - 1
    const int ntab = 4 * 65;
    tf.resize((size_t)5 * nz + ntab);
    for (int m = -32; m <= 32; ++m) {
        const float r = (float)std::exp2(-m / 8.0);
        const double cm = std::pow((double)r, -q.gamma);
        float* e = &tf[(size_t)5 * nz + 4 * (m + 32)];
        e[0] = r;
        e[1] = (float)((double)r - 1.0);
        e[2] = (float)cm;
        e[3] = (float)(cm - 1.0);
    }
    if (!c->d_srcf && hipMalloc(&c->d_srcf, sizeof(float) * (5 * nz + ntab)) != hipSuccess) {
        c->d_srcf = nullptr;
        return fail(c, EBS_E_OOM, "source tables");
    }
    // stages already queued on the context stream may still read the tables
    EBS_HIP(c, hipStreamSynchronize(c->stream));
    EBS_HIP(c, hipMemcpy(c->d_srcd, td.data(), sizeof(double) * 5 * nz, hipMemcpyHostToDevice));
    EBS_HIP(c, hipMemcpy(c->d_srcf, tf.data(), sizeof(float) * tf.size(), hipMemcpyHostToDevice));
    c->src = q;
    c->src_on = true;
    drop_graph(c);
    return EBS_OK;
}

ebs_status ebs_set_diffusion(ebs_ctx* c, const ebs_diffusion_params* prm) {
    if (!c) return EBS_E_ARG;
    if (prm) {
        if (!(prm->alpha_theta >= 0.0 && std::isfinite(prm->alpha_theta)) || (prm->eb_mode != 0 && prm->eb_mode != 1) ||
            !std::isfinite(prm->theta_wall))
            return fail(c, EBS_E_ARG, "diffusion parameters out of range");
    }
    // stages already queued may read the operators
    EBS_HIP(c, hipStreamSynchronize(c->stream));
    if (c->side) EBS_HIP(c, hipStreamSynchronize(c->side));
    drop_graph(c);
    if (!prm) {
        c->diff_on = false;
        return EBS_OK;
    }
    const bool was_on = c->diff_on;
    c->diff = *prm;
    c->diff_on = true;
    if (c->have_geom) {
        // the fits read theta at positions above the general range, which
        // the aux range of the stencil tables then holds
        ebs_status st = (was_on || c->visc_on) ? EBS_OK : build_stencils(c);
        if (st == EBS_OK) st = build_diffusion(c);
        if (st != EBS_OK) {
            c->diff_on = false;
            c->have_geom = false;  // tables half rebuilt: a new geometry build is needed
            return st;
        }
    }
    return EBS_OK;
}

ebs_status ebs_set_viscosity(ebs_ctx* c, const ebs_viscosity_params* prm) {
    if (!c) return EBS_E_ARG;
    if (prm && (!(prm->mu >= 0.0 && std::isfinite(prm->mu)) || (prm->eb_mode != 0 && prm->eb_mode != 1)))
        return fail(c, EBS_E_ARG, "viscosity parameters out of range");
    // stages already queued may read the operators
    EBS_HIP(c, hipStreamSynchronize(c->stream));
    if (c->side) EBS_HIP(c, hipStreamSynchronize(c->side));
    drop_graph(c);
    if (!prm) {
        c->visc_on = false;  // (the wider aux range stays until the next build)
        return EBS_OK;
    }
    const bool was_on = c->visc_on;
    c->visc = *prm;
    c->visc_on = true;
    if (c->have_geom) {
        // the fits read velocities at positions above the general range,
        // which the aux range of the stencil tables then holds
        ebs_status st = (was_on || c->diff_on) ? EBS_OK : build_stencils(c);
        if (st == EBS_OK) st = build_viscous(c);
        if (st != EBS_OK) {
            c->visc_on = false;
            c->have_geom = false;  // tables half rebuilt: a new geometry build is needed
            return st;
        }
    }
    return EBS_OK;
}

ebs_status ebs_restrict(ebs_ctx* c, const ebs_state* Uf, ebs_state* Uc) {
    if (!c) return EBS_E_ARG;
    if (!state_ok(Uf) || !state_ok(Uc)) return fail(c, EBS_E_ARG, "null state pointer");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    if ((c->nx | c->ny | c->nz) & 1) return fail(c, EBS_E_UNSUPPORTED, "restriction needs even grid sizes");
    // the fine state is read in pairs of x-neighbours (one 2-element load)
    const uintptr_t al = c->g.precision == EBS_F32_BULK ? 8 : 16;
    const void* const fine[5] = {Uf->rho, Uf->rhotheta, Uf->rhou, Uf->rhov, Uf->rhow};
    for (const void* p : fine)
        if ((uintptr_t)p % al) return fail(c, EBS_E_ARG, "fine state arrays must be aligned to two elements");
    return launch_restrict(c, Uf, Uc, nullptr);
}

ebs_status ebs_coarsened_geometry(ebs_ctx* c, double* alpha, double* bx, double* by, double* bz) {
    if (!c) return EBS_E_ARG;
    if (!alpha || !bx || !by || !bz) return fail(c, EBS_E_ARG, "null output array");
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    if ((c->nx | c->ny | c->nz) & 1) return fail(c, EBS_E_UNSUPPORTED, "restriction needs even grid sizes");
    const size_t NC = (size_t)(c->nx / 2) * (c->ny / 2) * (c->nz / 2);
    double* d = nullptr;
    if (hipMalloc(&d, sizeof(double) * 4 * NC) != hipSuccess) return fail(c, EBS_E_OOM, "coarse geometry buffer");
    ebs_status st = launch_restrict(c, nullptr, nullptr, d);
    hipError_t e = st == EBS_OK ? hipStreamSynchronize(c->stream) : hipSuccess;
    double* const dst[4] = {alpha, bx, by, bz};
    for (int q = 0; q < 4 && st == EBS_OK && e == hipSuccess; ++q)
        e = hipMemcpy(dst[q], d + q * NC, sizeof(double) * NC, hipMemcpyDeviceToHost);
    (void)hipFree(d);
    if (st != EBS_OK) return st;
    if (e != hipSuccess) return hip_fail(c, e, "coarse geometry");
    return EBS_OK;
}

ebs_status ebs_set_range_rule(ebs_ctx* c, int32_t rule) {
    if (!c) return EBS_E_ARG;
    if (rule < 0 || rule > 2) return fail(c, EBS_E_ARG, "range rule must be 0, 1 or 2");
    c->range_rule = rule;
    return EBS_OK;
}

ebs_status ebs_set_overlap(ebs_ctx* c, int32_t enable) {
    if (!c) return EBS_E_ARG;
    c->overlap = enable != 0;
    drop_graph(c);
    return EBS_OK;
}

ebs_status ebs_set_persistent(ebs_ctx* c, int32_t enable) {
    if (!c) return EBS_E_ARG;
    c->persistent = enable != 0;
    drop_graph(c);
    return EBS_OK;
}

ebs_status ebs_get_tile(const ebs_ctx* c, int32_t* tx, int32_t* ty, int32_t* tz, int32_t* span) {
    if (!c || !tx || !ty || !tz || !span) return EBS_E_ARG;
    *tx = c->tile_x;
    *ty = c->tile_y;
    *tz = c->tile_z;
    *span = c->tile_span;
    return EBS_OK;
}

ebs_status ebs_timing_enable(ebs_ctx* c, int32_t enable) {
    if (!c) return EBS_E_ARG;
    c->timing = enable != 0;
    c->ev_used = 0;
    return EBS_OK;
}

ebs_status ebs_timing_read(ebs_ctx* c, double* ms_total, int64_t* launches) {
    if (!c || !ms_total || !launches) return EBS_E_ARG;
    EBS_HIP(c, hipStreamSynchronize(c->stream));
    double tot = 0.0;
    for (size_t q = 0; q + 1 < c->ev_used; q += 2) {
        float ms = 0.f;
        EBS_HIP(c, hipEventElapsedTime(&ms, c->ev_pool[q], c->ev_pool[q + 1]));
        tot += ms;
    }
    *ms_total = tot;
    *launches = (int64_t)(c->ev_used / 2);
    c->ev_used = 0;
    return EBS_OK;
}

ebs_status ebs_algorithmic_bytes(const ebs_ctx* c, double out[2]) {
    if (!c || !out) return EBS_E_ARG;
    if (!c->have_geom) return EBS_E_ORDER;
    out[0] = c->alg_bytes[0];
    out[1] = c->alg_bytes[1];
    return EBS_OK;
}

ebs_status ebs_autotune(ebs_ctx* c, const char* cache_json_path) {
    if (!c) return EBS_E_ARG;
    if (!c->have_geom) return fail(c, EBS_E_ORDER, "geometry not built");
    const char* prec = c->g.precision == EBS_F32_BULK ? "f32bulk" : "f64";
    char key[160];
    std::snprintf(key, sizeof(key), "%s_%dx%dx%d_b%zu%s", prec, c->nx, c->ny, c->nz, c->boxes.size(),
                  c->src_on ? "_src" : "");
    // cached choice
    if (cache_json_path) {
        std::ifstream in(cache_json_path);
        if (in) {
            std::stringstream ss;
            ss << in.rdbuf();
            const std::string txt = ss.str();
            const std::string pat = std::string("\"") + key + "\": [";
            const size_t p = txt.find(pat);
            if (p != std::string::npos) {
                int tx = 0, ty = 0, tz = 0, sp = 0, ps = 0;
                const int got = std::sscanf(txt.c_str() + p + pat.size(), "%d, %d, %d, %d, %d", &tx, &ty, &tz, &sp, &ps);
                if (got >= 4 && ebs_set_tile(c, tx, ty, tz, sp) == EBS_OK) {
                    c->persistent = got == 5 && ps != 0;
                    return EBS_OK;
                }
            }
        }
    }
    // the timing stages overwrite the provisional copy ebs_redistribute reads
    c->have_adv = false;
    // scratch states
    const size_t es = c->g.precision == EBS_F32_BULK ? 4 : 8;
    const size_t nx = c->nx, ny = c->ny, nz = c->nz;
    const size_t cnt[5] = {nx * ny * nz, nx * ny * nz, (nx + 1) * ny * nz, nx * (ny + 1) * nz, nx * ny * (nz + 1)};
    void* buf[3][5] = {{nullptr}};
    ebs_state st[3];
    for (int s = 0; s < 3; ++s) {
        for (int f = 0; f < 5; ++f) {
            if (hipMalloc(&buf[s][f], es * cnt[f]) != hipSuccess) {
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 5; ++b) free_ptr(buf[a][b]);
                return fail(c, EBS_E_OOM, "autotune scratch");
            }
            (void)hipMemsetAsync(buf[s][f], 0, es * cnt[f], c->stream);
        }
        st[s] = {buf[s][0], buf[s][1], buf[s][2], buf[s][3], buf[s][4]};
    }
    // timing only: the values (zeros) do not change the work done.  Each
    // repetition is the three stages of a step: U^n = U_cur once, then twice
    // with separate U^n and U_cur.
    (void)hipStreamSynchronize(c->stream);
    auto three = [&]() {
        (void)launch_advance(c, &st[0], &st[0], &st[1], 0.0);
        (void)launch_advance(c, &st[0], &st[1], &st[2], 0.0);
        (void)launch_advance(c, &st[0], &st[2], &st[1], 0.0);
    };
    const int cxy[][2] = {{16, 4}, {16, 8}, {16, 16}, {32, 4}, {32, 8}, {32, 16}, {64, 2}, {64, 4}, {64, 8}, {64, 16}};
    const int cz[] = {16, 32, 64, 128, 256};
    double best = 1e300;
    int bx = c->tile_x, by = c->tile_y, bz = c->tile_z, bs = c->tile_span, bp = c->persistent ? 1 : 0;
    const bool was_timing = c->timing;
    c->timing = false;
    hipEvent_t e0, e1;
    EBS_HIP(c, hipEventCreate(&e0));
    EBS_HIP(c, hipEventCreate(&e1));
    constexpr int NZ = (int)(sizeof(cz) / sizeof(cz[0]));
    for (int q = 0; q < (int)(sizeof(cxy) / sizeof(cxy[0])) * NZ * 2; ++q) {
        const int cd[4] = {cxy[q / (2 * NZ)][0], cxy[q / (2 * NZ)][1], cz[(q / 2) % NZ], q % 2};
        // a height at or above nz tiles whole columns, as the next smaller
        // height at or above nz already did
        if ((q / 2) % NZ > 0 && cz[(q / 2) % NZ - 1] >= c->nz) continue;
        if (ebs_set_tile(c, cd[0], cd[1], cd[2], cd[3]) != EBS_OK) continue;
        for (int ps = 0; ps < 2; ++ps) {  // grid over every tile, or persistent
            c->persistent = ps != 0;
            three();
            (void)hipEventRecord(e0, c->stream);
            const int reps = 3;
            for (int rep = 0; rep < reps; ++rep) three();
            (void)hipEventRecord(e1, c->stream);
            (void)hipEventSynchronize(e1);
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (ms < best) { best = ms; bx = cd[0]; by = cd[1]; bz = cd[2]; bs = cd[3]; bp = ps; }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->timing = was_timing;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 5; ++b) free_ptr(buf[a][b]);
    ebs_status sst = ebs_set_tile(c, bx, by, bz, bs);
    if (sst != EBS_OK) return sst;
    c->persistent = bp != 0;
    if (cache_json_path) {
        std::string txt;
        {
            std::ifstream in(cache_json_path);
            if (in) {
                std::stringstream ss;
                ss << in.rdbuf();
                txt = ss.str();
            }
        }
        // append the entry to a flat JSON object
        const size_t close = txt.rfind('}');
        char ent[256];
        std::snprintf(ent, sizeof(ent), "\"%s\": [%d, %d, %d, %d, %d]", key, bx, by, bz, bs, bp);
        if (close == std::string::npos) {
            txt = std::string("{\n  ") + ent + "\n}\n";
        } else {
            const bool empty = txt.find('"') == std::string::npos;
            txt = txt.substr(0, close) + (empty ? "  " : ",\n  ") + ent + "\n}\n";
        }
        std::ofstream outf(cache_json_path);
        outf << txt;
    }
    return EBS_OK;
}

}  // extern "C"
