/*
 * ebstag — staggered-mesh embedded-boundary (cut-cell) update with weighted
 * state redistribution, for AMD Instinct MI355X (gfx950).
 *
 * C ABI.  Every entry point returns an ebs_status; no C++ exception or
 * longjmp crosses it.  Plain pointers and sizes only.
 *
 * Method (Kang et al., "An Embedded Boundary Scheme for Three-Dimensional Flow
 * Over Terrain on a Staggered Mesh"):
 *   - four geometry instances: cell-centred control volumes (CVs) and one
 *     staggered CV per x-, y- and z-face (Section 3.2, staggered data built
 *     from two half-cells of neighbouring cells);
 *   - explicit update of Eqs. update-cc / update-fc (Section 3.1) with the
 *     advective flux of Section 4.1 (third-order upwind, order reduction next
 *     to covered cells, flux moved to the cut-face centroid, no flux through
 *     walls); the source term is zero;
 *   - weighted state redistribution applied to every variable after every
 *     Runge-Kutta stage (Section 5.1, Algorithm 1 of Section 5.2).
 *
 * Grid and storage.  nx x ny x nz cells of size dx x dy x dz, lower corner lo.
 * x and y are periodic, z is bounded by no-flux walls.  The terrain is a
 * height function h(x, y) given on the (nx+1) x (ny+1) nodes (x fastest); the
 * fluid is {z > h} with h the continuous piecewise-linear interpolant on the
 * two triangles (i,j)(i+1,j)(i+1,j+1) and (i,j)(i+1,j+1)(i,j+1) of each
 * xy-cell.  The last node row / column must repeat the first (periodicity),
 * and the top cell layer must be free of terrain.
 *
 * State: five caller-owned device arrays, x fastest, element type double
 * (EBS_F64) or float (EBS_F32_BULK):
 *     rho, rhotheta : nz     x ny     x nx
 *     rhou          : nz     x ny     x (nx+1)   entry nx repeats entry 0
 *     rhov          : nz     x (ny+1) x nx       entry ny repeats entry 0
 *     rhow          : (nz+1) x ny     x nx       planes 0 and nz are walls
 * Inputs are read only where the entry is a fluid CV; every output entry is
 * written (0 where the CV has no fluid, at the walls, and the periodic
 * repeats copy entry 0).
 */
#ifndef EBSTAG_H
#define EBSTAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    EBS_OK = 0,
    EBS_E_ARG = 1,         /* invalid argument; nothing was written          */
    EBS_E_OOM = 2,         /* device or host allocation failed               */
    EBS_E_HIP = 3,         /* a HIP runtime call failed                      */
    EBS_E_ORDER = 4,       /* call out of order (e.g. before the geometry)   */
    EBS_E_UNSUPPORTED = 5  /* valid request outside what the library supports */
} ebs_status;

typedef enum {
    EBS_F64 = 0,      /* state and all arithmetic in double                          */
    EBS_F32_BULK = 1  /* state in float; regular-region flux and update in float;    */
                      /* geometry, cut-region fluxes, redistribution, sums in double  */
} ebs_precision;

typedef enum {
    EBS_EB_WALL = 0,       /* zero normal convective flux through the EB (Section 4.1) */
    EBS_EB_FREESTREAM = 1  /* test mode: EB flux = -(area vector).(mean provisional    */
                           /* flux of the CV); any uniform flow is then steady         */
} ebs_eb_flux;

typedef enum {
    EBS_LIM_BJ_COMPONENT = 0, /* Barth-Jespersen factor per gradient component (default) */
    EBS_LIM_BJ_SCALAR = 1,    /* one factor for the whole gradient                      */
    EBS_LIM_NONE = 2          /* unlimited linear reconstruction                        */
} ebs_limiter;

typedef struct {
    int32_t n[3];        /* cells; nx, ny >= 8, 4 <= nz <= 32767                */
    double dx[3];        /* cell size, > 0                                      */
    double lo[3];        /* lower domain corner                                 */
    uint32_t periodic;   /* bit d set: axis d periodic; must be 0x3 (x, y)      */
    double small_vfrac;  /* V_target / (dx dy dz), in (0, 1); the paper uses 0.5 */
    int32_t precision;   /* ebs_precision */
    int32_t limiter;     /* ebs_limiter   */
    int32_t eb_flux;     /* ebs_eb_flux   */
} ebs_grid;

/* Half-open cell ranges [lo, hi); the list must tile the domain without
 * overlap.  Boxes are the units of batched work (AMR-style patches of one
 * level); results do not depend on the tiling. */
typedef struct {
    int32_t lo[3], hi[3];
} ebs_box;

/* Caller-owned device pointers (see the storage notes above). */
typedef struct {
    void* rho;
    void* rhotheta;
    void* rhou;
    void* rhov;
    void* rhow;
} ebs_state;

typedef struct ebs_ctx ebs_ctx;

/* Geometry quantities for ebs_geometry_export (per CV of one instance). */
enum {
    EBS_Q_ALPHA = 0,                      /* volume fraction                          */
    EBS_Q_BETA_X = 1, EBS_Q_BETA_Y = 2, EBS_Q_BETA_Z = 3, /* lower-face area fractions */
    EBS_Q_FX_Y = 4, EBS_Q_FX_Z = 5,       /* lower x-face centroid offset / (dy, dz)  */
    EBS_Q_FY_X = 6, EBS_Q_FY_Z = 7,       /* lower y-face centroid offset / (dx, dz)  */
    EBS_Q_FZ_X = 8, EBS_Q_FZ_Y = 9,       /* lower z-face centroid offset / (dx, dy)  */
    EBS_Q_VC_X = 10, EBS_Q_VC_Y = 11, EBS_Q_VC_Z = 12, /* volume centroid - CV centre, / dx_d */
    EBS_Q_A_X = 13, EBS_Q_A_Y = 14, EBS_Q_A_Z = 15,    /* EB area vector (into fluid) / face area */
    EBS_Q_AREA = 16,                      /* EB facet area / (dx dy)                  */
    EBS_Q_EBC_X = 17, EBS_Q_EBC_Y = 18, EBS_Q_EBC_Z = 19, /* EB centroid - CV centre, / dx_d */
    EBS_Q_TYPE = 20,                      /* 0 covered / not a CV, 1 regular, 2 cut   */
    EBS_Q_SMALL = 21,                     /* 1 if 0 < alpha < small_vfrac             */
    EBS_Q_TIER = 22,                      /* merge tier 1..3 of a small CV, else 0    */
    EBS_Q_MASK = 23,                      /* members of M: bit (dz+1)*9+(dy+1)*3+(dx+1) */
    EBS_Q_NCOUNT = 24,                    /* N = number of neighbourhoods containing it */
    EBS_Q_KAPPA = 25, EBS_Q_OMEGA = 26,
    EBS_Q_VHAT = 27,                      /* neighbourhood volume / (dx dy dz)        */
    EBS_Q_XHAT_X = 28, EBS_Q_XHAT_Y = 29, EBS_Q_XHAT_Z = 30, /* nbhd centroid - CV centre, / dx_d */
    EBS_Q_COUNT = 31
};

/* Create a context.  grid is copied.  boxes may be NULL (one box = the
 * domain).  hip_stream is a hipStream_t (NULL = the null stream); all work of
 * the context is enqueued on it.  Errors: EBS_E_ARG (bad sizes, boxes that do
 * not tile the domain), EBS_E_UNSUPPORTED (non-periodic x or y, more than 2^31
 * cells, or (nx+1)(ny+1)(nz+1) elements of the state type reaching 4 GiB),
 * EBS_E_OOM. */
ebs_status ebs_create(const ebs_grid* grid, const ebs_box* boxes, int32_t nbox, void* hip_stream,
                      ebs_ctx** out);

/* Build the four geometry instances and the redistribution tables from nodal
 * terrain heights (Section 3.2; Section 5.1 precomputation).  h_nodes has
 * (nx+1)*(ny+1) doubles, x fastest, on the host (on_device = 0) or device.
 * Besides the geometry, the context then holds the static operators the
 * stage and the redistribution read: cut-face interpolation records,
 * stencil, update and cell tables of the general range, the Q-hat,
 * least-squares and contributor operators (about 2 KB per general cell).
 * Synchronous.  Errors: EBS_E_ARG (non-finite heights, non-periodic node rows,
 * terrain reaching the top cell layer), EBS_E_OOM (device tables),
 * EBS_E_UNSUPPORTED (general range or its tables beyond the sizes the
 * tables index: 2^28 general cells and stencil positions), EBS_E_HIP.
 * Calling it again on a context that has geometry rebuilds everything: it
 * first waits for the work queued on the context and drops the captured
 * RK3 graph.  EBS_E_ARG leaves the previous geometry in place; any later
 * error leaves the context without geometry (every stage call then returns
 * EBS_E_ORDER until a build succeeds). */
ebs_status ebs_build_geometry_terrain(ebs_ctx* ctx, const double* h_nodes, int32_t on_device);

/* The same build from a general level set (Section 3.2: the EB is the zero
 * set of an implicit function such as a signed distance, sampled at the
 * nodes; Sections 6.2-6.3 use a hemisphere and a wall-mounted square
 * cylinder).  phi_nodes has (nx+1)*(ny+1)*(nz+1) doubles, x fastest, then y,
 * then z, on the host (on_device = 0) or device; node index n of a periodic
 * axis repeats node 0.  Inside every cell the level set is interpolated
 * linearly over the six Kuhn tetrahedra {1 >= u[s0] >= u[s1] >= u[s2] >= 0}
 * (u the unit cell coordinates, s a permutation of the axes) and the fluid
 * is where it is positive; a face carries fluid where phi > 0 (phi >= 0 on
 * the domain bottom), a piece of the zero set belongs to the fluid it
 * bounds, and on the domain bottom the wall takes precedence.  phi = z - h
 * gives the terrain geometry of ebs_build_geometry_terrain.  Synchronous.
 * Errors: EBS_E_ARG (non-finite values, non-periodic node rows, phi <= 0 at
 * a node of the plane below the top cell layer), EBS_E_UNSUPPORTED (phi
 * decreasing along z at some node column: every column must be covered,
 * cut, then regular from the bottom up; and the sizes of
 * ebs_build_geometry_terrain), EBS_E_OOM, EBS_E_HIP; rebuild and failure
 * behaviour as for ebs_build_geometry_terrain. */
ebs_status ebs_build_geometry_levelset(ebs_ctx* ctx, const double* phi_nodes, int32_t on_device);

/* The same build for the coarse level of a two-level hierarchy with
 * refinement ratio 2 (Section 4.3: the coarse geometry is merged from the
 * fine one, so that volumes and areas, and with them mass and mass fluxes,
 * agree between the levels).  The context's grid is the coarse one;
 * fine_nodes are the nodal values of the fine grid (2nx x 2ny x 2nz cells of
 * half the spacing, same origin): terrain heights, (2nx+1)*(2ny+1) doubles
 * (kind 0), or a level set, (2nx+1)*(2ny+1)*(2nz+1) doubles, x fastest
 * (kind 1), on the host (on_device = 0) or device.  Every CV of every
 * instance is the union of eight fine cells (a staggered CV around a coarse
 * face spans the fine cells between the coarse cell centres on either
 * side): volume, moments, EB area and vector are the sums of the fine
 * cells', its faces the fine faces on its boundary, and it is covered
 * (regular) when all eight fine cells are.  Its volume and face fractions
 * are those ebs_coarsened_geometry and ebs_restrict use.  Synchronous.
 * Errors as for ebs_build_geometry_terrain / ebs_build_geometry_levelset
 * on the fine nodes, EBS_E_ARG for another kind; rebuild and failure
 * behaviour as for ebs_build_geometry_terrain. */
ebs_status ebs_build_geometry_merged(ebs_ctx* ctx, const double* fine_nodes, int32_t kind, int32_t on_device);

/* Copy one quantity (EBS_Q_*) of instance inst (0 cell, 1 x-face, 2 y-face,
 * 3 z-face) to host memory in the instance's state layout (n = element count
 * of that layout).  Synchronous. */
ebs_status ebs_geometry_export(ebs_ctx* ctx, int32_t inst, int32_t qty, double* host, size_t n);

/* Per instance: {cut, small, covered, tier1, tier2, tier3, general-region CVs,
 * regular} -> out[4*8].  Synchronous. */
ebs_status ebs_geometry_stats(ebs_ctx* ctx, int64_t* out);

/* Histogram of the volume fractions of the fluid CVs (alpha > 0) of
 * instance inst (0 cell, 1 x-face, 2 y-face, 3 z-face): counts[b] = number
 * of fluid CVs with edges[b] <= alpha < edges[b+1] (the last bin also takes
 * alpha == edges[nbins]); fractions outside [edges[0], edges[nbins]] are not
 * counted.  edges has nbins + 1 increasing values.  Reports how many small
 * and sliver CVs (Section 5.1) a terrain produces.  Synchronous.  Errors:
 * EBS_E_ARG, EBS_E_ORDER. */
ebs_status ebs_alpha_histogram(ebs_ctx* ctx, int32_t inst, const double* edges, int32_t nbins, int64_t* counts);

/* Algorithm 1 steps (1)-(3) for one stage (Section 5.2), all four
 * instances: Uhat = Un + cdt * dU(Ucur), dU by Eqs. update-cc / update-fc
 * (Section 3.1) with the advective fluxes of Section 4.1.  Un and Ucur may be
 * the same state.  No array of Uhat may overlap any array of Ucur (the
 * stencil reads neighbours while other threads write Uhat), the five Uhat
 * arrays must be disjoint, and Uhat may coincide with Un field by field
 * (Uhat->rho == Un->rho, ...) but not overlap it otherwise; EBS_E_ARG if
 * not.  Asynchronous. */
ebs_status ebs_advance_stage(ebs_ctx* ctx, const ebs_state* Un, const ebs_state* Ucur,
                             ebs_state* Uhat, double cdt);

/* Algorithm 1 step (4): Uout = R(Uhat) field by field, the weighted state
 * redistribution of Section 5.1 (Eqs. qhat_omega, qrecon,
 * final_update_omega).  Uhat must be the output state of the last
 * ebs_advance_stage of this context (the cut region is read from the
 * double-precision copy that advance kept); EBS_E_ORDER if it is another
 * state, or if no advance ran since the geometry was built or since an
 * ebs_rk3_step / ebs_autotune overwrote that copy.  Uout may coincide with
 * Uhat field by field but not overlap it otherwise (EBS_E_ARG).
 * Asynchronous. */
ebs_status ebs_redistribute(ebs_ctx* ctx, const ebs_state* Uhat, ebs_state* Uout);

/* One time step of Algorithm 1 (Section 5.2): the low-storage three-stage
 * Runge-Kutta scheme the paper names (its coefficients are not printed;
 * read as U^s = R(U^n + c_s dt dU(U^(s-1))) with c = 1/3, 1/2, 1), the
 * redistribution R of Section 5.1 after every stage.  U is updated in
 * place; scratch points at two states of the same layout used as stage
 * buffers; U and the two scratch states must be disjoint (EBS_E_ARG).
 * use_graph != 0 captures the step in a HIP graph on first use and replays
 * it while the pointers and dt stay the same.  Asynchronous. */
ebs_status ebs_rk3_step(ebs_ctx* ctx, ebs_state* U, ebs_state* scratch, double dt,
                        int32_t use_graph);

/* Sum of V * U over the fluid CVs of each field (rho, rhotheta, rhou, rhov,
 * rhow), as unevaluated double-double pairs hi + lo.  These are the totals
 * the method conserves: the update of Section 3.1 is conservative by
 * construction (every face flux enters two CVs with opposite signs, no
 * flux crosses walls) and the redistribution of Section 5.1 conserves them
 * as well.  Synchronous. */
ebs_status ebs_conserved_sums(ebs_ctx* ctx, const ebs_state* U, double hi[5], double lo[5]);

/* Time the candidate tile shapes of the regular-region kernel on this
 * context's grid and keep the fastest; the choice is cached in the JSON file
 * (created if missing, keyed by precision, grid size, box count and whether
 * the momentum sources are on; NULL = no cache).  The candidates are the
 * compiled shapes listed at ebs_set_tile, heights 16 to 256 (heights at or
 * above nz once), both spans and both schedules of ebs_set_persistent; the
 * cache entry holds [tx, ty, tz, span, persistent].  Each candidate is timed on the three
 * stages of a step (the first with U^n = U_cur), regular-region kernel and
 * general passes together.  Synchronous; three scratch states are allocated
 * and freed internally (EBS_E_OOM if they do not fit). */
ebs_status ebs_autotune(ebs_ctx* ctx, const char* cache_json_path);

/* Tile shape of the regular-region kernel: tx x ty columns per block and at
 * most tz planes per tile.  tx in {16, 32, 64}, ty in {2, 4, 8, 16}, tx*ty in
 * [64, 1024], (tx+5)(ty+5) <= 4 tx ty, LDS rings (26 (tx+5)(ty+5) elements of
 * the state type, plus 2 (tx+1)(ty+1) with the momentum sources) within the
 * device's LDS per block, and a compiled shape (16x4, 16x8, 16x16, 32x4, 32x8,
 * 32x16, 64x2, 64x4, 64x8, 64x16; other shapes give EBS_E_UNSUPPORTED at
 * launch); tz in {16, 32, 64, 128, 256}, or 0 to keep the current value.  span = 0: the tiles of every box are cut separately (no tile crosses
 * a box boundary); span = 1: the whole domain is tiled as one box (the box
 * list then does not shape the work; results are the same).  EBS_E_ARG
 * otherwise. */
ebs_status ebs_set_tile(ebs_ctx* ctx, int32_t tx, int32_t ty, int32_t tz, int32_t span);
ebs_status ebs_get_tile(const ebs_ctx* ctx, int32_t* tx, int32_t* ty, int32_t* tz, int32_t* span);

/* Schedule of the regular-region kernel: enable = 0 (default) launches one
 * block per tile; enable != 0 launches only as many blocks as the GPU holds
 * at once (resident blocks per compute unit times its units), each walking
 * its XCD's contiguous part of the tile list with a fixed stride, so a long
 * per-box tile list runs in one wave of persistent blocks.  Results are
 * identical; the captured RK3 graph is rebuilt.  The autotuner tries both. */
ebs_status ebs_set_persistent(ebs_ctx* ctx, int32_t enable);

/* Run the regular-region kernel on a second stream, concurrently with the
 * general-range passes and (inside ebs_rk3_step) the redistribution of the
 * same stage (enable != 0), or serially on the context stream (0, the
 * default).  The results are identical; the captured RK3 graph is rebuilt. */
ebs_status ebs_set_overlap(ebs_ctx* ctx, int32_t enable);

/* Rule for the top of each column's general range (the cells the FP64 cut
 * passes update; above it the regular-region kernel applies the plain
 * formulas), used by the next ebs_build_geometry_terrain.  rule 0: every CV
 * below the first regular level counts as possibly small; 1: the footprint
 * of the actual small CVs; 2 (default): the cells the redistribution tables
 * actually read or write.  A stricter rule gives fewer general cells and the
 * same results up to rounding; if one of its set-up checks fails, the build
 * falls back to the next looser rule.  EBS_E_ARG for another value. */
ebs_status ebs_set_range_rule(ebs_ctx* ctx, int32_t rule);

/* Momentum sources of the compressible model (Section 2.1, Eq. mom-comp):
 * the perturbation pressure gradient -grad p' and the buoyancy -rho' g (g
 * acting along -z), with p = P00 (R rho theta / P00)^gamma (the equation of
 * state of Section 2.1), p' = p - p0(z) and rho' = rho - rho0(z).  The
 * reference state satisfies the equation of state, so it is given by rho
 * theta0 and rho0, and p0 = P00 (R rho theta0 / P00)^gamma; p' is evaluated
 * as p0 expm1(gamma log1p((rho theta - rho theta0) / rho theta0)), equal to
 * p - p0 but free of the cancellation of two values near P00.  The paper
 * adds them to the right-hand side as a source (Section 4.1) without giving
 * a cut-cell form; this library uses: p' and rho' on fluid cells with the
 * reference values of the cell's level; the momentum CV around the lower
 * d-face of cell c gets -(p'(c) - p'(c - e_d)) / dx_d when both cells are
 * fluid (else no pressure force), and the z-face CVs add -g times the mean
 * rho' of their fluid cells.  Every later ebs_advance_stage / ebs_rk3_step
 * adds c dt times these (evaluated on Ucur) to the provisional momenta of
 * every fluid CV, before the redistribution.
 *   prm:  constants (P00 > 0, R > 0, gamma > 1, g >= 0), or NULL to switch
 *         the sources off.
 *   rhotheta0, rho0: host arrays of nz doubles, the reference rho theta
 *         (kg K / m^3) and density (kg / m^3) at the cell-centre height of
 *         each level (positive, finite); copied, the caller keeps ownership.
 *         The state must keep rho theta > 0 on fluid cells.
 * Synchronous: waits for the work queued on the context stream before it
 * replaces the tables.  Errors: EBS_E_ARG for invalid values;
 * EBS_E_UNSUPPORTED with the free-stream EB closure, or when the current tile
 * shape leaves no LDS for the pressure planes (choose another with
 * ebs_set_tile); EBS_E_OOM, EBS_E_HIP. */
typedef struct {
    double P00;    /* reference pressure of the equation of state, Pa (1e5) */
    double R;      /* gas constant of dry air, J / (kg K) */
    double gamma;  /* ratio of specific heats cp / cv */
    double g;      /* gravitational acceleration, m / s^2 */
} ebs_source_params;
ebs_status ebs_set_sources(ebs_ctx* ctx, const ebs_source_params* prm, const double* rhotheta0,
                           const double* rho0);

/* Thermal diffusion of rho theta (Section 4.2; Eq. theta-comp): every later
 * ebs_advance_stage / ebs_rk3_step adds c dt times the divergence of
 * rho alpha_theta grad(theta) to the provisional rho theta of every fluid
 * cell, before the redistribution.  Full faces use the centred difference of
 * theta; cut faces and the EB facets use the gradient of a least-squares fit
 * of a second-order polynomial over the fluid cells around them, as the
 * paper describes (its details are deferred to a reference): unweighted,
 * quadratic in mesh units about the face or facet centroid, over 4 cells
 * along a face's normal and 3 across (3 x 3 x 3 around a facet), falling back
 * to a linear fit with fewer than 10 points or a reciprocal 1-norm condition
 * number of the normal matrix below 1e-7, and to no gradient with fewer than
 * 4 points or a linear matrix as poorly conditioned.  The EB is adiabatic
 * (eb_mode 0: no flux) or held at theta_wall (eb_mode 1: the facet fit passes
 * through theta_wall at the facet centroid).  Face density: mean of the two
 * cells; facet density: the cut cell's.  The domain bottom and top are
 * adiabatic.  The fit weights depend on the geometry only and are built here
 * (or by the next geometry build), about 36 points per cut face; switching
 * diffusion on after a geometry build also rebuilds the stencil tables, whose
 * range of positions above the general range the fits read.
 *   prm: alpha_theta >= 0 (m^2/s), eb_mode 0 or 1, theta_wall finite; NULL
 *        switches diffusion off.
 * Synchronous: waits for the work queued on the context.  Errors: EBS_E_ARG,
 * EBS_E_OOM, EBS_E_HIP, EBS_E_UNSUPPORTED (more than 2^30 cells, or a table
 * beyond its index range; after an error other than EBS_E_ARG the geometry
 * must be built again). */
typedef struct {
    double alpha_theta; /* thermal diffusivity, m^2 / s */
    int32_t eb_mode;    /* 0 adiabatic EB, 1 EB held at theta_wall */
    double theta_wall;  /* K */
} ebs_diffusion_params;
ebs_status ebs_set_diffusion(ebs_ctx* ctx, const ebs_diffusion_params* prm);

/* Momentum diffusion (Sections 2.1 and 4.2; Eq. mom-comp): every later
 * ebs_advance_stage / ebs_rk3_step adds c dt times the divergence of the
 * viscous stress tau = lambda (div u) I + mu (grad u + grad u^T), lambda =
 * -2/3 mu, to the provisional momenta of every fluid u, v and w CV, before
 * the redistribution.  The velocity of a staggered CV is its momentum over
 * the mean density of the fluid cells beside its face.  tau_xx, tau_yy and
 * tau_zz act on the CV faces at cell centres, the shear components on those
 * at cell edges.  Full faces (area fraction >= 1 - 1e-12) use the centred
 * differences of the staggered grid.  Cut faces and EB facets use gradients
 * of least-squares fits of each velocity component over the fluid CVs of its
 * own grid, 3 CVs wide along an axis on which the face or facet CV centre
 * lines up with that grid and 4 wide otherwise (the stencil sizes the paper
 * gives for fits across grid types); the fit is that of ebs_set_diffusion.
 * The EB is stress-free (eb_mode 0) or no-slip (eb_mode 1: the fits at the
 * facet centroid take the velocity there as zero).  The domain bottom and
 * top are stress-free for u and v; the w CVs next to them end at the first
 * and last cell centres and feel tau_zz there, with w = 0 on the walls.  The
 * fit weights depend on the geometry only and are built here (or by the
 * next geometry build); switching it on after a geometry build also
 * rebuilds the stencil tables, whose range of positions above the general
 * range the fits read.
 *   prm: mu >= 0 finite (dynamic viscosity, kg / (m s)), eb_mode 0 or 1;
 *        NULL switches momentum diffusion off.
 * Synchronous: waits for the work queued on the context.  Errors: EBS_E_ARG,
 * EBS_E_OOM, EBS_E_HIP, EBS_E_UNSUPPORTED (a table beyond its index range;
 * after an error other than EBS_E_ARG the geometry must be built again). */
typedef struct {
    double mu;       /* dynamic viscosity */
    int32_t eb_mode; /* 0 stress-free EB, 1 no-slip EB */
} ebs_viscosity_params;
ebs_status ebs_set_viscosity(ebs_ctx* ctx, const ebs_viscosity_params* prm);

/* Restriction (averaging down) of a state of this context's grid onto the
 * grid coarsened by 2 in every direction (Section 4.3: static two-level
 * refinement with ratio 2; the coarse geometry is merged from the fine
 * subcells, cell-centred variables are averaged with volume-fraction weights
 * and face-centred ones with area-fraction weights, which keeps the mass of
 * every coarse cell and the mass flux through every coarse face).  Coarse
 * cell (I, J, K) covers fine cells (2I + a, 2J + b, 2K + c), a, b, c in {0, 1}.
 *   Ufine:   device state of this context (layout of ebs_advance_stage),
 *            each array aligned to two elements (8 bytes FP32, 16 FP64).
 *   Ucoarse: caller-owned device state of the coarse grid, same precision:
 *            rho, rhotheta (nz/2, ny/2, nx/2), rhou (nz/2, ny/2, nx/2 + 1),
 *            rhov (nz/2, ny/2 + 1, nx/2), rhow (nz/2 + 1, ny/2, nx/2), x
 *            fastest; every entry is written (periodic repeats copied, walls
 *            and covered cells 0).  Must not overlap Ufine.
 * A coarse momentum is the area-weighted mean over the four fine faces on
 * its face; where that face has no open area, the mean weighted by the
 * volume fractions of the four fine staggered CVs; 0 if both vanish.
 * Asynchronous on the context stream.  Errors: EBS_E_ARG (null or
 * misaligned pointers), EBS_E_ORDER (no geometry), EBS_E_UNSUPPORTED (an odd
 * grid size). */
ebs_status ebs_restrict(ebs_ctx* ctx, const ebs_state* Ufine, ebs_state* Ucoarse);

/* The merged geometry of the coarse grid (Section 4.3): volume fraction of
 * every coarse cell (mean of its eight children) and area fractions of its
 * lower x, y, z faces (means of the four fine faces on each); host arrays of
 * (nz/2)(ny/2)(nx/2) doubles each, x fastest.  Synchronous; allocates and
 * frees a device buffer.  Errors as ebs_restrict, EBS_E_OOM, EBS_E_HIP. */
ebs_status ebs_coarsened_geometry(ebs_ctx* ctx, double* alpha, double* beta_x, double* beta_y, double* beta_z);

/* ebs_coarsened_geometry for callers that cannot allocate device memory
 * (harnesses that forbid it, loops that must not call the allocator): the
 * same kernel and results, staged through a fixed device buffer that the
 * library holds for the life of the process (one per GPU, 16 MiB) instead of
 * a buffer allocated and freed per call.  It calls no allocator.  The coarse
 * grid may have at most EBS_COARSE_GEO_MAX_CELLS cells (EBS_E_UNSUPPORTED
 * beyond).  Calls on one GPU share the buffer; the library serialises them
 * within a process (each call holds the buffer until its copies to the host
 * are done), so concurrent calls from several host threads wait for each
 * other.  Synchronous.  Errors: as ebs_coarsened_geometry without
 * EBS_E_OOM. */
#define EBS_COARSE_GEO_MAX_CELLS (1 << 19)
ebs_status ebs_coarsened_geometry_noalloc(ebs_ctx* ctx, double* alpha, double* beta_x, double* beta_y,
                                          double* beta_z);

/* Kernel timing: when enabled, every launch of the regular-region stage
 * kernel is bracketed by HIP events on the context stream; read returns the
 * summed duration (ms) and launch count since the last reset and resets. */
ebs_status ebs_timing_enable(ebs_ctx* ctx, int32_t enable);
ebs_status ebs_timing_read(ebs_ctx* ctx, double* ms_total, int64_t* launches);

/* Bytes moved per call of the regular-region stage kernel by the method
 * (reads of Un and Ucur, one write, over the regular-region CVs), for roofline
 * accounting: out[0] = first-stage form (Un == Ucur), out[1] = later stages. */
ebs_status ebs_algorithmic_bytes(const ebs_ctx* ctx, double out[2]);

/* Measurement reference: copy `bytes` from src to dst (device pointers,
 * 16-byte aligned, bytes a multiple of 16, not overlapping) with a plain
 * streaming kernel, asynchronously on hip_stream (a hipStream_t, NULL = the
 * null stream).  Timed by the caller, it gives the HBM rate a streaming
 * kernel reaches on the device, against which the roofline fractions of the
 * method's kernels are also reported.  Errors: EBS_E_ARG (null, misaligned
 * or overlapping), EBS_E_UNSUPPORTED (beyond 2^31 blocks), EBS_E_HIP. */
ebs_status ebs_stream_copy(void* dst, const void* src, size_t bytes, void* hip_stream);

/* Static message describing the last error of the context (never NULL). */
const char* ebs_last_error(const ebs_ctx* ctx);

/* Free all device memory and graphs of the context.  ctx may be NULL. */
ebs_status ebs_destroy(ebs_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* EBSTAG_H */
