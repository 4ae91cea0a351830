/*
 * FP64 CPU oracle for the staggered embedded-boundary (cut-cell) update with
 * weighted state redistribution.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it.  It shares no source with the HIP library.
 *
 * It is deliberately plain and slow: dense triple loops over every control
 * volume, generic Sutherland-Hodgman polygon clipping with exact quadrature for
 * the geometry, explicit neighbourhood sets for the redistribution.
 *
 * Storage convention used throughout the oracle: every instance (0 = cell
 * centred, 1 = x-face, 2 = y-face, 3 = z-face control volumes) is held as a
 * dense array of (nz+1) x ny x nx entries, x fastest.  Entry (i,j,k) of the
 * x-face instance is the control volume around the x-face at node i, etc.
 * Planes that are not control volumes (k = nz for instances 0-2; k = 0 and
 * k = nz for the z-face instance) have volume fraction 0; their lower z-face
 * data are still filled where the face exists (the domain top).
 */
#ifndef EBS_ORACLE_H
#define EBS_ORACLE_H

#include <stdint.h>

/* geometry quantities per control volume (first index of the geometry array) */
enum {
    OQ_ALPHA = 0,         /* volume fraction                                       */
    OQ_BX, OQ_BY, OQ_BZ,  /* area fractions of the lower x, y, z faces             */
    OQ_FX1, OQ_FX2,       /* lower x-face centroid offset (y, z) / (dy, dz)        */
    OQ_FY1, OQ_FY2,       /* lower y-face centroid offset (x, z) / (dx, dz)        */
    OQ_FZ1, OQ_FZ2,       /* lower z-face centroid offset (x, y) / (dx, dy)        */
    OQ_VCX, OQ_VCY, OQ_VCZ, /* volume centroid offset from the CV centre / dx_d    */
    OQ_AX, OQ_AY, OQ_AZ,  /* EB area vector (into the fluid) / face area of dir d  */
    OQ_AREA,              /* EB facet area / (dx*dy)                               */
    OQ_EBX, OQ_EBY, OQ_EBZ, /* EB centroid offset from the CV centre / dx_d        */
    OQ_N
};

/* redistribution quantities per control volume */
enum {
    OW_SMALL = 0,  /* 1 if the CV is small (0 < alpha < small_vfrac)            */
    OW_TIER,       /* merge tier 1..3 for small CVs, 0 otherwise                 */
    OW_MASK,       /* members of M as a 27-bit mask over offsets in {-1,0,1}^3   */
    OW_NCOUNT,     /* N = |W| (number of neighbourhoods containing the CV)       */
    OW_KAPPA, OW_OMEGA,
    OW_VHAT,       /* neighbourhood volume / (dx dy dz)                          */
    OW_XHX, OW_XHY, OW_XHZ, /* neighbourhood centroid offset from CV centre / dx_d */
    OW_N
};

typedef struct {
    int32_t n[3];
    double dx[3];
    double lo[3];
    double small_vfrac;  /* V_target / (dx dy dz), 0.5 in the paper      */
    int32_t limiter;     /* 0 component-wise BJ, 1 scalar BJ, 2 none      */
    int32_t eb_flux;     /* 0 no-flux wall, 1 free-stream closure mode    */
} orc_grid;

/* geometry: geo[inst] points at OQ_N * (nz+1)*ny*nx doubles; ctype[inst] at
 * (nz+1)*ny*nx bytes (0 covered or not a CV, 1 regular, 2 cut) */
int orc_geometry(const orc_grid* g, const double* h_nodes, double* const geo[4],
                 int8_t* const ctype[4]);

/* Geometry of a general level set phi (Section 3.2), layout as orc_geometry.
 * phi_nodes: (nz+1) x (ny+1) x (nx+1) nodal values, x fastest; fluid is
 * {phi > 0} for the piecewise linear interpolant over the six Kuhn
 * tetrahedra of every cell.  phi must be nondecreasing along z at every node
 * column; returns 1 (and writes nothing) otherwise. */
int orc_geometry_levelset(const orc_grid* g, const double* phi_nodes, double* const geo[4],
                          int8_t* const ctype[4]);

/* Moments of box piece `part` (0 whole cell, 1/2 lower/upper half in x, 3/4
 * in y, 5/6 in z) of cell (i,j,k) for a level set, relative to the cell's
 * lower node: out = [vol, mx, my, mz, EB area vector x,y,z, EB area, 6 face
 * areas, type (0 covered, 1 regular, 2 cut)].  Exposed for tests. */
int orc_levelset_piece(const orc_grid* g, const double* phi_nodes, int i, int j, int k, int part,
                       double* out);

/* Geometry of the coarse grid g of a two-level hierarchy with refinement
 * ratio 2, merged from the fine cells (Section 4.3): fine_nodes are the
 * nodal terrain heights (kind 0, (2ny+1) x (2nx+1)) or level set (kind 1,
 * (2nz+1) x (2ny+1) x (2nx+1)) of the fine grid (2n cells of dx/2, same
 * origin).  Layout as orc_geometry; returns 1 for a level set that
 * decreases along z. */
int orc_geometry_merged(const orc_grid* g, const double* fine_nodes, int kind, double* const geo[4],
                        int8_t* const ctype[4]);

/* redistribution tables: w[inst] points at OW_N * (nz+1)*ny*nx doubles */
int orc_wsrd_setup(const orc_grid* g, double* const geo[4], double* const w[4]);

/* One explicit stage: Uhat = Un + cdt * dU(Ucur).  Each state is five dense
 * fields in instance storage: rho, rhotheta (inst 0), rhou (1), rhov (2),
 * rhow (3).  Entries that are not fluid CVs are written as 0. */
int orc_advance(const orc_grid* g, double* const geo[4], const double* const Un[5],
                const double* const Ucur[5], double* const Uhat[5], double cdt);

/* Redistribution of one provisional state, Uout = R(Uhat), field by field. */
int orc_redistribute(const orc_grid* g, double* const geo[4], double* const w[4],
                     const double* const Uhat[5], double* const Uout[5]);

/* Same, also returning the limited gradient of every CV: sig[f] points at
 * 3 * (nz+1)*ny*nx doubles (x, y, z interleaved per CV), physical units. */
int orc_redistribute_sig(const orc_grid* g, double* const geo[4], double* const w[4],
                         const double* const Uhat[5], double* const Uout[5],
                         double* const sig[5]);

/* Same, also returning Q-hat of every CV (Eq. qhat_omega; U-hat where the
 * neighbourhood is the CV alone): qhat[f] points at (nz+1)*ny*nx doubles. */
int orc_redistribute_diag(const orc_grid* g, double* const geo[4], double* const w[4],
                          const double* const Uhat[5], double* const Uout[5], double* const sig[5],
                          double* const qhat[5]);

/* Raw face fluxes, exposed for the telescoping and polynomial-exactness pins:
 * F[d] receives the flux used in the divergence on the lower d-face of every
 * CV of instance inst for field f (0 rho, 1 rhotheta, 2 rhou, 3 rhov, 4 rhow). */
int orc_face_fluxes(const orc_grid* g, double* const geo[4], const double* const U[5],
                    int field, double* const F[3], double* const Fhat[3]);

/* Constants of the equation of state p = P00 (R rho theta / P00)^gamma and
 * gravity (acting along -z), Section 2.1. */
typedef struct {
    double P00, R, gamma, g;
} orc_src;

/* Momentum sources of Ucur (perturbation pressure gradient, buoyancy on the
 * z-face CVs), intensive, per CV: S[d] receives instance d+1 in dense storage,
 * zero where not a fluid CV.  rt0, rho0: reference rho theta and density at
 * the cell-centre height of each level (nz entries); the reference pressure is
 * their equation-of-state value. */
int orc_sources(const orc_grid* g, double* const geo[4], const double* const U[5], const orc_src* s,
                const double* rt0, const double* rho0, double* const S[3]);

/* Geometry of the grid coarsened by 2 (Section 4.3, merged subcells):
 * alpha and the area fractions of the lower x, y, z faces of every coarse
 * cell, (nz/2) x (ny/2) x (nx/2) arrays, x fastest.  1 if a size is odd. */
int orc_coarsen_geometry(const orc_grid* g, double* const geo[4], double* alpha, double* const beta[3]);

/* Restriction of a fine state (dense instance storage) onto the grid coarsened
 * by 2 (dense instance storage with nz/2 + 1 planes).  1 if a size is odd. */
int orc_restrict(const orc_grid* g, double* const geo[4], const double* const Uf[5], double* const Uc[5]);

/* Moments of the fluid part {z > terrain} of an axis-aligned box inside the
 * xy-cell (ci,cj): exposed so tests can check the clipper against closed forms.
 * out: [vol, mx, my, mz, area vector x,y,z, eb area, 6 face areas] with moments
 * relative to the box corner. */
int orc_box_moments(const orc_grid* g, const double* h_nodes, int ci, int cj,
                    const double rect[4], double za, double zb, int bottom, double* out);

/* Thermal diffusion of rho theta (Section 4.2): thermal diffusivity
 * alpha_theta (>= 0); the EB is adiabatic (eb_mode 0) or held at theta_wall
 * (eb_mode 1). */
typedef struct {
    double alpha_theta;
    int32_t eb_mode;
    double theta_wall;
} orc_diff;

/* Intensive diffusive update of rho theta on the cell-centred CVs, D (dense
 * instance storage; 0 where not fluid): (1/V) times the sum of
 * rho alpha_theta grad(theta) . n_out over the open face areas and the EB
 * facet.  Optional outputs (NULL to skip): Fd[d] the flux density
 * rho alpha_theta d(theta)/dx_d on the lower d-face of every cell (0 on
 * closed faces and walls), Feb the EB term (rho alpha_theta grad(theta) .
 * n_out times the facet area) of every cell. */
int orc_diffusion(const orc_grid* g, double* const geo[4], const double* const U[5], const orc_diff* p,
                  double* D, double* const Fd[3], double* Feb);

/* Momentum diffusion (Sections 2.1 and 4.2): dynamic viscosity mu (>= 0);
 * the EB is stress-free (eb_mode 0) or no-slip (eb_mode 1). */
typedef struct {
    double mu;
    int32_t eb_mode;
} orc_visc;

/* Intensive viscous update of the three momenta, D[c] (dense storage of
 * instance c + 1; 0 where not fluid): (1/V) times the sum of tau_c . n_out
 * over the open face areas and the EB facet.  Optional outputs (NULL to
 * skip): F[3 c + d] the stress tau_{c d} on the lower d-face of every CV of
 * instance c + 1 (0 where the face is closed or a wall), E[c] the facet term
 * of every CV. */
int orc_viscous(const orc_grid* g, double* const geo[4], const double* const U[5], const orc_visc* p,
                double* const D[3], double* const F[9], double* const E[3]);

/* Threads used by the plane loops of the geometry, stage and redistribution
 * (n > 0 sets the count; returns the count in use).  Each loop iteration
 * writes only its own plane's entries, so results are bitwise independent
 * of the count. */
int orc_set_threads(int n);

#endif
