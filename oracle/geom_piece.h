/*
 * Shared by the oracle's two geometry builders, the terrain one (geom.c) and
 * the general level-set one (levelset.c).  TEST INFRASTRUCTURE ONLY (see
 * oracle.h).
 *
 * Both produce the moments of the fluid part of axis-aligned box pieces of a
 * cell; the assembly of the four control-volume instances from those pieces
 * (Section 3.2: a staggered control volume is the union of two half-cells of
 * neighbouring cells, volumes and areas summed, centroids volume- or
 * area-weighted) is common and lives in geom.c.
 */
#ifndef EBS_ORACLE_GEOM_PIECE_H
#define EBS_ORACLE_GEOM_PIECE_H

#include "oracle.h"

/* Result for one axis-aligned box; all moments relative to the cell's lower
 * corner node (X_i, Y_j, Z_k).  Faces: 0 x-lo, 1 x-hi, 2 y-lo, 3 y-hi, 4 z-lo,
 * 5 z-hi; fm holds the first moments of every face in all three coordinates. */
typedef struct {
    double vol, mv[3];
    double fa[6], fm[6][3];
    double av[3], area, em[3];
} BoxOut;

/* A geometry source.  piece(): moments of box piece `part` of cell (i, j, k)
 * (0 the whole cell; 1 / 2 the lower / upper half in x; 3 / 4 in y; 5 / 6 in
 * z); i and j may lie one outside [0, n) and wrap periodically.  type(): 0
 * covered, 1 regular, 2 cut for the same piece. */
typedef struct PieceSrc {
    const orc_grid* g;
    const void* data;
    void (*piece)(const struct PieceSrc* s, int i, int j, int k, int part, BoxOut* o);
    int (*type)(const struct PieceSrc* s, int i, int j, int k, int part);
} PieceSrc;

/* Nodal data of a source: terrain heights ((ny+1) x (nx+1)) or a level set
 * ((nz+1) x (ny+1) x (nx+1)), x fastest; it must outlive the source. */
typedef struct {
    const orc_grid* g;
    const double* v;
} NodeData;

/* The terrain builder's and the level-set builder's sources. */
void orc_terrain_src(const NodeData* d, PieceSrc* s);
void orc_levelset_src(const NodeData* d, PieceSrc* s);

/* Fill geo / ctype (layout of orc_geometry) from a geometry source. */
int orc_assemble(const PieceSrc* src, double* const geo[4], int8_t* const ctype[4]);

#endif
