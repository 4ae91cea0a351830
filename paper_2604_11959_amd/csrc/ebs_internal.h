// Internal declarations of the ebstag library (not part of the C ABI).
//
// Data layout in device memory
// ----------------------------
// The terrain is a height function, so in every xy-column each of the four
// instances is covered below a level kf, cut in a band, and regular above a
// level kr.  The library stores geometry only for a per-column "general"
// range of cell positions [g0, g1):
//     g0 = min over instances of kf (below: every instance covered),
//     g1 = max over instances and over the 7 x 7 neighbouring columns of kr,
//          plus 3 (above: every CV and every CV within the flux stencil and
//          the redistribution radius is regular), clamped to nz; g1 = g0
//          (empty range) when every CV in that window is regular down to the
//          bottom wall.
// General cells are numbered column by column (goff[c] + k - g0[c]); each has
// a geometry record per instance (structure of arrays, GQ_* quantities) and
// redistribution data.  Everything above g1 is processed by the regular-region
// kernel, which reads no geometry at all.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "ebstag.h"

namespace ebs {

constexpr int NINST = 4;
// geometry record quantities (same order as the EBS_Q_* export ids 0..19)
enum : int {
    GQ_ALPHA = 0, GQ_BX, GQ_BY, GQ_BZ, GQ_FX1, GQ_FX2, GQ_FY1, GQ_FY2, GQ_FZ1, GQ_FZ2,
    GQ_VCX, GQ_VCY, GQ_VCZ, GQ_AX, GQ_AY, GQ_AZ, GQ_AREA, GQ_EBX, GQ_EBY, GQ_EBZ, GQ_N
};
// redistribution tables per general cell and instance (doubles)
enum : int { WQ_N = 0, WQ_KAPPA, WQ_OMEGA, WQ_VHAT, WQ_XHX, WQ_XHY, WQ_XHZ, WQ_COUNT };

// reach of the regular-region stencils (cells, laterally and downwards) and of
// the redistribution footprint of a small CV (neighbourhood, fit points)
constexpr int GEN_RXY = 3;
constexpr int GEN_RZ = 3;
constexpr int WSRD_RXY = 2;
constexpr int WSRD_RZ = 2;
// tie / threshold tolerance of the discrete redistribution decisions
constexpr double TIE = 1e-12;

// Read-only view of the geometry passed to kernels by value.
struct GeoView {
    int nx, ny, nz;
    double dx, dy, dz;
    double lo_z;
    int32_t G;                 // number of general cells
    const int32_t* g0;         // [ncol]
    const int32_t* g1;         // [ncol]
    const int32_t* goff;       // [ncol]
    const int4* col;           // [ncol] {g0 | g1 << 16, g1e, goff, goffe}: one load per lookup
    int32_t Ge;                // cells of the extended face range (see below)
    const int32_t* gcole;      // [Ge] column of each cell of the extended face range
    const uint32_t* fflag;     // [G] lower-face flags: FF_POS / FF_FULL bits per (instance, dir)
    const int32_t* gcol;       // [G] column of each general cell
    const int32_t* kf;         // [4][ncol] first fluid CV level
    const int32_t* kr;         // [4][ncol] first regular level
    const double* geo;         // [4][GQ_N][G]
    const int8_t* type;        // [4][G]
    const uint32_t* type4;     // [G] the four instance types packed, byte s = instance s
};

struct WsrdView {
    const int32_t* mask;       // [4][G] 27-bit member mask (0 = not a fluid CV)
    const int8_t* small;       // [4][G]
    const int8_t* tier;        // [4][G]
    const double* w;           // [4][WQ_COUNT][G]
    int limiter;
    double vt;                 // V_target / (dx dy dz)
};

// A state as typed device pointers (T = double or float)
template <typename T>
struct StateP {
    T* f[5];
};

__host__ __device__ inline int wrapi(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Column range info.  Planes [g0, g1) form the column's general range (general
// index goff + k - g0).  Provisional face fluxes are kept for the longer range
// [g0, g1e), g1e = min(nz, max(g1 + 1, g1 of the -x and -y neighbours)), with
// index goffe + k - g0: it holds the lower faces of every CV whose face is an
// upper face of a general CV.
__host__ __device__ inline int col_g0(const int4& c) { return c.x & 0xFFFF; }
__host__ __device__ inline int col_g1(const int4& c) { return (int)((uint32_t)c.x >> 16); }
__host__ __device__ inline int4 col_pack(int g0, int g1, int g1e, int goff, int goffe) {
    return make_int4(g0 | (g1 << 16), g1e, goff, goffe);
}

// lower-face flags of a general cell: area fraction > 0, and == 1
__host__ __device__ constexpr uint32_t ff_pos(int inst, int d) { return 1u << (inst * 3 + d); }
__host__ __device__ constexpr uint32_t ff_full(int inst, int d) { return 1u << (16 + inst * 3 + d); }

// general index of cell position (i, j, k) (i, j wrapped), -2 below the general
// range (every instance covered), -1 above it (every instance regular)
__device__ inline int gidx(const GeoView& v, int i, int j, int k) {
    const int4 ci = v.col[j * v.nx + i];
    const int g0 = col_g0(ci);
    if (k < g0) return -2;
    if (k >= col_g1(ci)) return -1;
    return ci.z + (k - g0);
}

// is plane k a CV plane of instance inst
__device__ inline bool cv_plane(const GeoView& v, int inst, int k) {
    return inst == 3 ? (k >= 1 && k <= v.nz - 1) : (k >= 0 && k <= v.nz - 1);
}

__device__ inline double gq(const GeoView& v, int inst, int q, int g) {
    return v.geo[((size_t)inst * GQ_N + q) * v.G + g];
}

}  // namespace ebs

// ---------------------------------------------------------------- context
struct ebs_tile {
    int32_t x0, y0, z0;
    int16_t ex, ey, ez, flags;  // extents; flags: offset of the first plane with regular-region work
};

struct ebs_graph_cache {
    void* exec = nullptr;  // hipGraphExec_t
    void* graph = nullptr; // hipGraph_t
    ebs_state U{}, S0{}, S1{};
    double dt = 0.0;
};

struct ebs_ctx {
    ebs_grid g{};
    int nx = 0, ny = 0, nz = 0;
    int ncol = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;        // regular-region kernel, concurrent with the general range
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool join_pending = false;
    bool overlap = false;              // use the side stream (ebs_set_overlap)
    bool persistent = false;           // regular-region grid of resident blocks only (ebs_set_persistent)
    std::vector<ebs_box> boxes;
    std::string err = "no error";

    // geometry
    bool have_geom = false;
    int32_t* d_kf = nullptr;
    int32_t* d_kr = nullptr;
    int32_t* d_g0 = nullptr;
    int32_t* d_g1 = nullptr;
    int32_t* d_goff = nullptr;
    int32_t* d_gcol = nullptr;
    int4* d_col = nullptr;
    int32_t G = 0;
    int32_t Ge = 0;                  // cells of the extended face range
    int32_t* d_gcole = nullptr;      // [Ge]
    uint32_t* d_fflag = nullptr;     // [G]
    int32_t* d_cbase = nullptr;      // [G] first cut-face record of each general cell
    // cut-face interpolation records (stage.hip): {n0, n1, n2, own |
    // (instance * 3 + direction) << 28} and [5][ncut] {b, c0..c3}
    int4* d_cut_n = nullptr;
    double* d_cut_w = nullptr;
    double* d_bfc = nullptr;         // [2][ncut] interpolated flux per record (per stage)
    int32_t ncut = 0;
    double* d_geo = nullptr;
    int8_t* d_type = nullptr;
    uint32_t* d_type4 = nullptr;
    std::vector<int32_t> h_g0, h_g1, h_goff, h_g1e;
    // general range rule: 0 loose (every CV below kr possibly small), 1 tight
    // (footprint window of the small CVs), 2 exact (the cells the
    // redistribution reads or writes, h_ftop, per column)
    int range_mode = 1;
    int geo_merged = 0;  // the build in progress merges the geometry of the grid refined by 2
    int range_rule = 2;  // the strictest mode the geometry build tries (ebs_set_range_rule)
    // momentum sources (ebs_set_sources): per-level tables [5][nz] of p0,
    // rho theta0 (high, low part), 1 / rho theta0, rho0 in the state precision
    // and in FP64; per position of the prims pass {p', rho'} (FP64)
    bool src_on = false;
    ebs_source_params src{};
    float* d_srcf = nullptr;
    double* d_srcd = nullptr;
    double* d_srcv = nullptr;  // [G + naux][2] {p', rho'} per position of the prims pass (sources on)
    std::vector<int32_t> h_ftop;  // [ncol] highest level the redistribution touches, -1 if none

    // redistribution
    int32_t* d_mask = nullptr;
    int8_t* d_small = nullptr;
    int8_t* d_tier = nullptr;
    double* d_w = nullptr;
    int32_t* d_smalllist = nullptr;  // [4][G] general indices of small CVs with kappa > 0
    int32_t nsmall[4] = {0, 0, 0, 0};
    int32_t* d_actlist = nullptr;    // [4][G] general indices of CVs R may change
    int32_t nact[4] = {0, 0, 0, 0};
    int32_t sbase[4] = {0, 0, 0, 0};  // offset of each instance in the concatenated small list
    int32_t nlsq = 0;                 // small CVs with kappa > 0, all instances
    int64_t nlsq_pts = 0;             // least-squares fit points, all small CVs
    int32_t* d_lsq_off = nullptr;     // [nlsq + 1] first fit point of each small CV
    uint32_t* d_lsq_idx = nullptr;    // [pts] general index (| flag: Q-hat is the CV's own)
    double* d_lsq_c = nullptr;        // [3][pts] A^-1 e_s in mesh units
    double* d_lsq_ev = nullptr;       // [nlsq][8][3] limiter evaluation offsets
    int8_t* d_lsq_nev = nullptr;      // [nlsq]
    int32_t abase[4] = {0, 0, 0, 0};  // offset of each instance in the concatenated active list
    int32_t* d_wl_off = nullptr;      // [A + 1] contributors of each active CV (CSR)
    int32_t* d_wl_idx = nullptr;      // [E] general index of the contributing small CV
    double* d_wl_geo = nullptr;       // [E][4] kappa_r and the centroid offset
    double* d_wl_self = nullptr;      // [A][5] omega, N and the own centroid offset
    int8_t* d_wl_small = nullptr;     // [A]
    int32_t* d_q_idx = nullptr;       // [nlsq][8] Q-hat operator: the CV, then its members
    double* d_q_w = nullptr;          // [nlsq][8] its weights
    double* d_q_den = nullptr;        // [nlsq] V-hat
    int8_t* d_q_n = nullptr;          // [nlsq] entries used
    int32_t* d_chk = nullptr;         // set-up check counter

    // per-stage buffers (cut region, double)
    double* d_uhat = nullptr;  // [5][G] provisional state of the last advance
    double* d_qhat = nullptr;  // [5][G]
    double* d_sig = nullptr;   // [5][3][G]
    double* d_prim = nullptr;  // [G + naux][4] advected quantities: general range, then aux positions
    int32_t naux = 0;          // positions above the general range read by the face-range stencils
                               // (and, with momentum diffusion, by its fits and centred differences)
    std::vector<int32_t> h_gp, h_aoff;  // [ncol] top of the aux range, first aux position
    int2* d_acol = nullptr;             // [ncol] {first aux position, top of the aux range}
    int4* d_ptab = nullptr;    // [G + naux] cell table of the prims pass
    int4* d_ftab = nullptr;    // [Ge] cell table of the flux pass
    int4* d_utab = nullptr;    // [G] cell table of the update pass
    uint32_t* d_sten = nullptr; // [10][Ge] stencil table of the face range (see build_stencils)
    int32_t* d_upd = nullptr;   // [9][G] update table: ge, flags, first record of the +x, +y, +z faces
    double* d_fh = nullptr;    // [5][3][Ge] provisional lower-face fluxes (extended range)

    // regular-region tiles
    int tile_x = 32, tile_y = 8, tile_z = 64;
    int tile_span = 0;  // 1: tiles cut from the whole domain instead of per box
    int lds_max = 64 * 1024;  // LDS per block of the device
    std::vector<ebs_tile> h_tiles;
    ebs_tile* d_tiles = nullptr;
    int32_t ntiles = 0;
    double alg_bytes[2] = {0, 0};

    // sums
    double* d_part = nullptr;
    int npart = 0;

    // timing
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;

    ebs_graph_cache graph;
    double* d_dummy = nullptr;
    // thermal diffusion of rho theta (ebs_set_diffusion): fit operators of
    // the cut faces and facets (CSR over linear cell indices), their flux per
    // stage, and per general cell the operator of each face and of the facet
    bool diff_on = false;
    ebs_diffusion_params diff{};
    int32_t ndop = 0;
    int64_t ndop_pts = 0;
    int32_t* d_dop_off = nullptr;   // [ndop + 1]
    int32_t* d_dop_idx = nullptr;   // [pts]
    double* d_dop_w = nullptr;      // [pts]
    int32_t* d_dop_cell = nullptr;  // [ndop] cell | direction << 30 (3 = facet)
    double* d_dflux = nullptr;      // [ndop]
    int32_t* d_dtab = nullptr;      // [G][7]
    // momentum diffusion (ebs_set_viscosity): fit operators of the cut faces
    // and facets of the u, v and w CVs (CSR over velocity points), their
    // stress per stage, and per general cell and momentum the operator of
    // each face and of the facet
    bool visc_on = false;
    ebs_viscosity_params visc{};
    int32_t nvop = 0;
    int32_t* d_vop_off = nullptr;  // [nvop + 1]
    uint32_t* d_vop_pt = nullptr;  // [pts] component << 28 | position in the advected-quantity array
    double* d_vop_w = nullptr;     // [pts]
    double* d_vflux = nullptr;     // [nvop]
    int32_t* d_vtab = nullptr;     // [G][3][7]
    // output of the last ebs_advance_stage: the cut range of ebs_redistribute
    // is read from d_uhat, which holds that advance's provisional state
    bool have_adv = false;
    ebs_state last_uhat{};
};

namespace ebs {
// geometry (geom.hip)
// exactly one of d_h (terrain heights) and d_phi (level set) is non-null
ebs_status build_geometry(ebs_ctx* c, const double* d_h, const double* d_phi);
// stage kernels (stage.hip)
// defer_join: leave the regular-region kernel running on the side stream;
// join_side() makes the context stream wait for it
ebs_status launch_advance(ebs_ctx* c, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uhat,
                          double cdt, bool defer_join = false);
ebs_status join_side(ebs_ctx* c);
ebs_status build_tiles(ebs_ctx* c);
ebs_status build_cut_faces(ebs_ctx* c);
ebs_status build_stencils(ebs_ctx* c);
// per column the highest level the redistribution reads or writes (its
// active CVs and least-squares fit points), from the current tables
ebs_status redistribution_tops(ebs_ctx* c, std::vector<int32_t>& ftop);
// regular-region kernel (bulk.hip) on the given stream, with its timing events
ebs_status launch_bulk(ebs_ctx* c, const ebs_state* Un, const ebs_state* Ucur, ebs_state* Uhat, double cdt,
                       hipStream_t stream);
size_t bulk_lds_bytes(int tx, int ty, int precision, bool sources);
ebs_status launch_restrict(ebs_ctx* cx, const ebs_state* Uf, ebs_state* Uc, double* geo_out);
// thermal diffusion (diffusion.hip): operators, and the passes of one stage
// over the general range (context stream)
ebs_status build_diffusion(ebs_ctx* c);
ebs_status launch_diffusion_general(ebs_ctx* c, const ebs_state* Ucur, ebs_state* Uhat, double cdt);
// momentum diffusion (viscous.hip), the same
ebs_status build_viscous(ebs_ctx* c);
ebs_status launch_viscous_general(ebs_ctx* c, const ebs_state* Ucur, ebs_state* Uhat, double cdt);
// thermal and momentum diffusion above the general range (regdiff.hip), one
// pass on the given stream for whichever of the two is on
ebs_status launch_regular_diffusion(ebs_ctx* c, const ebs_state* Ucur, ebs_state* Uhat, double cdt,
                                    hipStream_t stream);
// redistribution (wsrd.hip)
ebs_status wsrd_setup(ebs_ctx* c);
ebs_status launch_redistribute(ebs_ctx* c, const ebs_state* Uhat, ebs_state* Uout);
// sums (reduce.hip)
ebs_status conserved_sums(ebs_ctx* c, const ebs_state* U, double hi[5], double lo[5]);

GeoView geo_view(const ebs_ctx* c);
WsrdView wsrd_view(const ebs_ctx* c);
ebs_status hip_fail(ebs_ctx* c, hipError_t e, const char* what);
}  // namespace ebs

#define EBS_HIP(ctx, call)                                              \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return ebs::hip_fail((ctx), e_, #call);   \
    } while (0)
