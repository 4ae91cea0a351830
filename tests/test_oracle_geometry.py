"""Pins of the oracle geometry builder (Section 3.2 of the paper) against
closed forms, invariants and brute force.  CPU only."""
import numpy as np
import pytest

import oracle
import synth
from tests.helpers import (halfspace_box_volume, sample_cv, sample_facet, sample_vface,
                           sample_vface_moments, sample_zface_moments)

OQ = oracle.OQ


def cv_box(grid, inst, i, j, k):
    """Axis-aligned extent of CV (i,j,k) of an instance (x0,x1,y0,y1,z0,z1)."""
    dx, dy, dz = grid.dx
    x0 = grid.lo[0] + i * dx
    y0 = grid.lo[1] + j * dy
    z0 = grid.lo[2] + k * dz
    box = [x0, x0 + dx, y0, y0 + dy, z0, z0 + dz]
    if inst in (1, 2, 3):
        d = inst - 1
        box[2 * d] -= 0.5 * grid.dx[d]
        box[2 * d + 1] -= 0.5 * grid.dx[d]
    return box


@pytest.mark.parametrize("plane", [
    (0.37, 0.21, -0.13),     # generic slopes
    (0.40, 0.0, 0.33),       # zero x-slope
    (0.55, -0.6, 0.0),       # zero y-slope
    (0.2, 1.7, 0.9),         # steep: crosses several layers per cell
])
def test_plane_volume_fractions_closed_form(plane):
    """alpha of every CV of all four instances equals the exact volume of the
    box above the plane z = a + bx + cy (inclusion-exclusion over vertices);
    the piecewise-linear facets reproduce a plane exactly."""
    a, b, c = plane
    g = synth.Grid((8, 8, 8), (0.125, 0.125, 0.125))
    h = synth.terrain_plane(g, a, b, c)
    o = oracle.Oracle(g, h)
    dv = 0.125 ** 3
    nx, ny, nz = g.n
    worst = 0.0
    for inst in range(4):
        al = o.alpha(inst)
        for k in range(nz + 1):
            if inst == 3 and not (1 <= k <= nz - 1):
                continue
            if inst != 3 and k == nz:
                continue
            for j in range(ny):
                for i in range(nx):
                    # staggered CVs straddling the periodic seam join cells from
                    # both ends of a non-periodic plane: skip them
                    if (inst == 1 and i == 0) or (inst == 2 and j == 0):
                        continue
                    x0, x1, y0, y1, z0, z1 = cv_box(g, inst, i, j, k)
                    solid = halfspace_box_volume((x0, y0, z0), (x1, y1, z1), (-b, -c, 1.0), a)
                    exact = 1.0 - solid / dv
                    worst = max(worst, abs(al[k, j, i] - exact))
    assert worst < 2e-14


def test_column_identity_and_total_volume():
    """sum_k V_ijk = dx dy Lz - integral of the interpolated terrain over the
    xy-cell (mean of the two triangles' vertex means), for terrain inside the
    domain; the x-, y- and z-face instances tile the same fluid region."""
    w = synth.make_workload(2)
    g = w.grid
    o = oracle.Oracle(g, w.h_nodes)
    h = w.h_nodes
    dx, dy, dz = g.dx
    nx, ny, nz = g.n
    ha, hb, hc, hd = h[:-1, :-1], h[:-1, 1:], h[1:, 1:], h[1:, :-1]
    integral = dx * dy * ((ha + hb + hc) / 3.0 + (ha + hc + hd) / 3.0) / 2.0
    expect = dx * dy * nz * dz - integral
    col = o.volume(0)[:nz].sum(axis=0)
    assert np.max(np.abs(col - expect) / (dx * dy * nz * dz)) < 1e-13
    total = o.volume(0).sum()
    assert abs(o.volume(1).sum() - total) / total < 1e-13
    assert abs(o.volume(2).sum() - total) / total < 1e-13
    # z-face CVs miss the lower half of layer 0 and the (fully fluid) upper
    # half of layer nz-1
    missing = total - o.volume(3).sum() - nx * ny * dx * dy * dz / 2
    assert -1e-9 * total <= missing <= nx * ny * dx * dy * dz / 2 * (1 + 1e-13)


@pytest.mark.parametrize("cfg", [1, 2])
def test_closure_every_cv(cfg):
    """Divergence theorem per CV: beta_hi - beta_lo = a_d (area vector of the EB
    facet, into the fluid, normalised by the d-face area), all four instances."""
    w = synth.make_workload(cfg)
    o = oracle.Oracle(w.grid, w.h_nodes)
    nx, ny, nz = w.grid.n
    for inst in range(4):
        G = o.geo[inst]
        cv = np.zeros((nz + 1, ny, nx), bool)
        if inst == 3:
            cv[1:nz] = True
        else:
            cv[:nz] = True
        for d, (qb, qa) in enumerate([(OQ["BX"], OQ["AX"]), (OQ["BY"], OQ["AY"]), (OQ["BZ"], OQ["AZ"])]):
            lo = G[qb]
            if d == 0:
                hi = np.roll(lo, -1, axis=2)
            elif d == 1:
                hi = np.roll(lo, -1, axis=1)
            else:
                hi = np.concatenate([lo[1:], np.zeros_like(lo[:1])], axis=0)
            err = np.abs((hi - lo) - G[qa])[cv]
            assert err.max() < 1e-13, (inst, d, err.max())


def test_shared_face_from_both_sides_and_covered_faces():
    """The x-face between cells i-1 and i computed as the upper face of cell i-1
    equals the lower face of cell i (different triangles of different cells);
    covered CVs carry no fluid on any face."""
    w = synth.make_workload(1)
    g = w.grid
    dx, dy, dz = g.dx
    rng = np.random.default_rng(7)
    for _ in range(40):
        i = int(rng.integers(1, 32)); j = int(rng.integers(0, 32)); k = int(rng.integers(0, 12))
        za, zb = k * dz, (k + 1) * dz
        left = oracle.box_moments(g, w.h_nodes, i - 1, j, [0, dx, 0, dy], za, zb, k == 0)
        right = oracle.box_moments(g, w.h_nodes, i, j, [0, dx, 0, dy], za, zb, k == 0)
        assert abs(left[8 + 1] - right[8 + 0]) <= 1e-16 * dy * dz
        below = oracle.box_moments(g, w.h_nodes, i, j - 1, [0, dx, 0, dy], za, zb, k == 0)
        assert abs(below[8 + 3] - right[8 + 2]) <= 1e-16 * dx * dz
    o = oracle.Oracle(g, w.h_nodes)
    for inst in range(4):
        G = o.geo[inst]
        cov = (o.ctype[inst] == 0)
        if inst == 3:
            cov[0] = False
        cov[g.n[2]] = False
        for q in (OQ["BX"], OQ["BY"], OQ["BZ"]):
            assert np.all(G[q][cov] == 0.0)
        assert np.all(G[OQ["ALPHA"]][cov] == 0.0)


def test_brute_force_sampling_all_instances():
    """alpha, volume centroid, face fractions and EB area vector of every CV of
    all four instances against brute-force sampling of the definition, on a
    small grid with a bump that crosses several layers."""
    g = synth.Grid((6, 6, 4), (1.0, 1.0, 0.5))
    x, y = synth.node_coords(g)
    X, Y = np.meshgrid(x, y)
    h = 0.2 + 1.1 * np.exp(-((X - 3.1) ** 2 + (Y - 2.7) ** 2) / 2.0) + 0.05 * np.sin(X + 2 * Y)
    h = synth._periodic_fix(h)
    o = oracle.Oracle(g, h)
    dv = 0.5
    nx, ny, nz = g.n
    cnt = 0
    for inst in range(4):
        G = o.geo[inst]
        for k in range(nz + 1):
            if inst == 3 and not (1 <= k <= nz - 1):
                continue
            if inst != 3 and k == nz:
                continue
            for j in range(ny):
                for i in range(nx):
                    if (inst == 1 and i == 0) or (inst == 2 and j == 0):
                        continue
                    box = cv_box(g, inst, i, j, k)
                    V, cen, av = sample_cv(h, g, box, M=200)
                    assert abs(G[OQ["ALPHA"], k, j, i] - V / dv) < 1e-4
                    if V > 0.05 * dv:
                        ctr = np.array([(box[0] + box[1]) / 2, (box[2] + box[3]) / 2,
                                        (box[4] + box[5]) / 2])
                        vc = np.array([G[OQ["VCX"] + d, k, j, i] for d in range(3)])
                        assert np.allclose(vc * np.array(g.dx), cen - ctr, atol=2e-4)
                    farea = np.array([0.5, 0.5, 1.0])
                    ahat = np.array([G[OQ["AX"] + d, k, j, i] for d in range(3)])
                    assert np.allclose(ahat, av / farea, atol=2e-2)
                    # lower x and y faces by a 1-D sampler
                    bx = sample_vface(h, g, 0, box[0], box[2], box[3], box[4], box[5])
                    by = sample_vface(h, g, 1, box[2], box[0], box[1], box[4], box[5])
                    assert abs(G[OQ["BX"], k, j, i] - bx) < 1e-5
                    assert abs(G[OQ["BY"], k, j, i] - by) < 1e-5
                    cnt += 1
    assert cnt > 400


def test_terrain_on_grid_planes():
    """Terrain exactly on an interior grid plane: the face on the terrain carries
    no fluid, the facet belongs to the cell above (alpha = 1, full EB area,
    normal +z); the cell below is covered.  Terrain on the domain bottom:
    regular bottom cells (the wall takes precedence)."""
    g = synth.Grid((8, 8, 6), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 2.0))
    G = o.geo[0]
    assert np.all(G[OQ["ALPHA"], 1] == 0.0) and np.all(o.ctype[0][1] == 0)
    assert np.all(G[OQ["ALPHA"], 2] == 1.0)
    assert np.all(G[OQ["BZ"], 2] == 0.0)
    assert np.all(G[OQ["AREA"], 2] == 1.0) and np.all(G[OQ["AZ"], 2] == 1.0)
    assert np.all(o.ctype[0][2] == 2)
    assert np.all(o.ctype[0][3] == 1)
    # z-face instance: CV 2 spans [1.5, 2.5]: lower half solid
    assert np.allclose(o.geo[3][OQ["ALPHA"], 2], 0.5)
    o0 = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    assert np.all(o0.ctype[0][:6] == 1)
    assert np.all(o0.geo[0][OQ["BZ"], 0] == 1.0)
    assert np.all(o0.geo[0][OQ["AREA"]] == 0.0)


def test_flat_terrain_fractions():
    """Flat terrain at 0.73 dz: cc and x/y-face CVs of layer 0 have alpha = 0.27,
    face fractions 0.27 on the vertical faces, volume centroid at the middle of
    the fluid slab; the z-face CV at k = 1 has alpha = 0.77."""
    g = synth.Grid((8, 8, 6), (2.0, 3.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.73))
    for inst in range(3):
        G = o.geo[inst]
        assert np.allclose(G[OQ["ALPHA"], 0], 0.27, rtol=0, atol=1e-15)
        assert np.allclose(G[OQ["BX"], 0], 0.27, atol=1e-15)
        assert np.allclose(G[OQ["BY"], 0], 0.27, atol=1e-15)
        assert np.allclose(G[OQ["BZ"], 0], 0.0)
        assert np.allclose(G[OQ["VCZ"], 0], (0.73 + 1.0) / 2 - 0.5, atol=1e-15)
        assert np.allclose(G[OQ["FX2"], 0], (0.73 + 1.0) / 2 - 0.5, atol=1e-15)
        assert np.allclose(G[OQ["AZ"], 0], 1.0) and np.allclose(G[OQ["AREA"], 0], 1.0)
    assert np.allclose(o.geo[3][OQ["ALPHA"], 1], 0.77, atol=1e-15)


def test_mirror_symmetry():
    """x <-> y symmetric terrain on a square grid: the diagonal split maps the
    two triangles onto each other, so the cell-centred data are symmetric and
    the x- and y-face instances are mirror images."""
    g = synth.Grid((16, 16, 8), (1.0, 1.0, 0.4))
    x, y = synth.node_coords(g)
    X, Y = np.meshgrid(x, y)
    h = 1.3 * np.exp(-((X - 7.3) ** 2 + (Y - 7.3) ** 2) / 9.0) + 0.1 * np.cos(0.3 * (X * Y))
    h = 0.5 * (h + h.T)
    h = synth._periodic_fix(h)
    o = oracle.Oracle(g, h)
    T = lambda a: np.swapaxes(a, -1, -2)
    Gc, Gu, Gv = o.geo[0], o.geo[1], o.geo[2]
    assert np.allclose(Gc[OQ["ALPHA"]], T(Gc[OQ["ALPHA"]]), rtol=0, atol=1e-14)
    assert np.allclose(Gc[OQ["BX"]], T(Gc[OQ["BY"]]), rtol=0, atol=1e-14)
    assert np.allclose(Gc[OQ["AX"]], T(Gc[OQ["AY"]]), rtol=0, atol=1e-14)
    assert np.allclose(Gu[OQ["ALPHA"]], T(Gv[OQ["ALPHA"]]), rtol=0, atol=1e-14)
    assert np.allclose(Gu[OQ["BZ"]], T(Gv[OQ["BZ"]]), rtol=0, atol=1e-14)
    assert np.array_equal(o.ctype[1], T(o.ctype[2]))


def test_brute_force_face_centroids_and_facets_all_instances():
    """Face centroid offsets (FX1 .. FZ2), EB facet area and EB centroid of
    every CV of all four instances on the bump terrain (facets of two
    different slopes per xy-cell) against brute-force sampling of the
    definitions; offsets compared as moments (fraction x offset).  Catches
    swapped or mis-signed offsets, offsets from the wrong face centre and a
    staggered face or facet assembled from the wrong halves."""
    g = synth.Grid((6, 6, 4), (1.0, 1.0, 0.5))
    x, y = synth.node_coords(g)
    X, Y = np.meshgrid(x, y)
    h = 0.2 + 1.1 * np.exp(-((X - 3.1) ** 2 + (Y - 2.7) ** 2) / 2.0) + 0.05 * np.sin(X + 2 * Y)
    h = synth._periodic_fix(h)
    o = oracle.Oracle(g, h)
    nx, ny, nz = g.n
    dx = np.array(g.dx)
    worst = np.zeros(3)
    cut_faces = 0
    for inst in range(4):
        G = o.geo[inst]
        for k in range(nz + 1):
            if inst == 3 and not (1 <= k <= nz - 1):
                continue
            if inst != 3 and k == nz:
                continue
            for j in range(ny):
                for i in range(nx):
                    if (inst == 1 and i == 0) or (inst == 2 and j == 0):
                        continue
                    box = cv_box(g, inst, i, j, k)
                    ctr = np.array([(box[0] + box[1]) / 2, (box[2] + box[3]) / 2, (box[4] + box[5]) / 2])
                    # vertical lower faces
                    for d, (e1, e2) in ((0, (1, 2)), (1, (0, 2))):
                        lo_s, hi_s = (box[2], box[3]) if d == 0 else (box[0], box[1])
                        b, (cs, cz) = sample_vface_moments(h, g, d, box[2 * d], lo_s, hi_s, box[4], box[5])
                        q = OQ["FX1"] + 2 * d
                        e_s = abs(b * (cs - ctr[e1]) / dx[e1] - G[OQ["BX"] + d, k, j, i] * G[q, k, j, i])
                        e_z = abs(b * (cz - ctr[2]) / dx[2] - G[OQ["BX"] + d, k, j, i] * G[q + 1, k, j, i])
                        worst[0] = max(worst[0], e_s, e_z)
                        assert e_s < 1e-7 and e_z < 1e-7, (inst, d, i, j, k, e_s, e_z)
                        cut_faces += 0.01 < b < 0.99
                    # horizontal lower face
                    b, (cx, cy) = sample_zface_moments(h, g, box[4], box[0], box[1], box[2], box[3])
                    e_x = abs(b * (cx - ctr[0]) / dx[0] - G[OQ["BZ"], k, j, i] * G[OQ["FZ1"], k, j, i])
                    e_y = abs(b * (cy - ctr[1]) / dx[1] - G[OQ["BZ"], k, j, i] * G[OQ["FZ2"], k, j, i])
                    worst[1] = max(worst[1], e_x, e_y)
                    assert e_x < 2e-4 and e_y < 2e-4, (inst, i, j, k, e_x, e_y)
                    # EB facet: area and centroid
                    A, c = sample_facet(h, g, box)
                    a_or = G[OQ["AREA"], k, j, i] * dx[0] * dx[1]
                    assert abs(A - a_or) < 2e-3 * dx[0] * dx[1], (inst, i, j, k, A, a_or)
                    if A > 0.05 * dx[0] * dx[1]:
                        ebc = np.array([G[OQ["EBX"] + q, k, j, i] for q in range(3)])
                        err = np.abs(a_or * ebc - A * (c - ctr) / dx).max()
                        worst[2] = max(worst[2], err)
                        assert err < 1e-3, (inst, i, j, k, err)
    assert cut_faces > 100
    print("worst face-centroid moment errors (vertical, horizontal, facet)", worst)
