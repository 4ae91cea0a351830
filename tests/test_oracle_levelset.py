"""Pins of the oracle's level-set geometry builder (Section 3.2: the EB is the
zero set of an implicit function sampled at the nodes; reading: the piecewise
linear interpolant over the six Kuhn tetrahedra of every cell, fluid where it
is positive) against the terrain builder (a different algorithm on the same
geometry), closed forms and brute force.  CPU only.  Each test names the
mistakes it exists to catch."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import (clip_polygon, halfspace_box_volume, levelset_fluid_length,
                           polygon_area_centroid, rect)

OQ = oracle.OQ


def _comparable(o, inst):
    """Quantities of one instance in a form that is continuous in the
    geometry: centroid offsets times their fraction."""
    G = o.geo[inst]
    out = {q: G[OQ[q]] for q in ("ALPHA", "BX", "BY", "BZ", "AX", "AY", "AZ", "AREA")}
    for q, b in (("FX1", "BX"), ("FX2", "BX"), ("FY1", "BY"), ("FY2", "BY"), ("FZ1", "BZ"), ("FZ2", "BZ")):
        out[q] = G[OQ[q]] * G[OQ[b]]
    for q in ("VCX", "VCY", "VCZ"):
        out[q] = G[OQ[q]] * G[OQ["ALPHA"]]
    for q in ("EBX", "EBY", "EBZ"):
        out[q] = G[OQ[q]] * G[OQ["AREA"]]
    return out


def _bumpy_terrain(g, seed):
    rng = np.random.default_rng(seed)
    x, y = synth.node_coords(g)
    X, Y = np.meshgrid(x, y)
    Lz = g.n[2] * g.dx[2]
    h = 0.1 * Lz + 0.35 * Lz * np.exp(-((X - 0.45 * x[-1]) ** 2 + (Y - 0.55 * y[-1]) ** 2) / (0.1 * x[-1] ** 2))
    h = h + 0.03 * Lz * rng.standard_normal(h.shape)
    return synth._periodic_fix(h)


@pytest.mark.parametrize("case", ["c1", "bumpy", "plane", "hills"])
def test_terrain_as_level_set_matches_terrain_builder(case):
    """phi = z - h at the nodes describes the terrain geometry (the Kuhn
    interpolant of z - h is z minus the two-triangle terrain interpolant), so
    the level-set builder (3-D tetrahedra, polygons clipped in their own
    planes, divergence theorem) and the terrain builder (2-D triangles,
    column integrals) must agree on every quantity of all four instances, and
    on every type.  Catches a wrong tetrahedron set or diagonal, a box face
    booked on the wrong side, a wrong EB orientation, a half-cell clipped on
    the wrong side and a wrong domain-bottom rule (c1 has bottom slivers,
    the truncated hills exactly flat ground at h = 0)."""
    if case == "c1":
        w = synth.make_workload(1)
        g, h = w.grid, w.h_nodes
    elif case == "bumpy":
        g = synth.Grid((12, 10, 8), (1.0, 1.5, 0.75))
        h = _bumpy_terrain(g, 3)
    elif case == "plane":
        g = synth.Grid((8, 8, 8), (0.125, 0.125, 0.125))
        h = synth.terrain_plane(g, 0.37, 0.21, -0.13)
    else:
        g = synth.Grid((24, 24, 12), (78.125, 78.125, 23.4375))
        h = synth.terrain_gaussian_hills(g, 7, 3, hrange=(60.0, 200.0), wrange=(120.0, 250.0))
        assert (h == 0.0).mean() > 0.1
    ot = oracle.Oracle(g, h)
    ol = oracle.Oracle(g, phi_nodes=synth.levelset_terrain(g, h))
    for inst in range(4):
        assert np.array_equal(ot.ctype[inst], ol.ctype[inst]), inst
        a, b = _comparable(ot, inst), _comparable(ol, inst)
        for q in a:
            err = np.abs(a[q] - b[q]).max()
            assert err <= 1e-12, (case, inst, q, err)


@pytest.mark.parametrize("normal", [
    (0.6, 0.3, 0.74),    # tilted, crosses several cells
    (0.8, -0.6, 0.0),    # vertical: no terrain can describe it
    (0.0, 0.97, 0.243),  # steep in y
])
def test_plane_level_sets_exact(normal):
    """A plane phi = n . x - d (n_z >= 0) is reproduced exactly by the
    interpolant: alpha of every CV of all four instances equals the exact
    volume of the box on the fluid side (rational inclusion-exclusion), and
    the lower x- and y-face fractions of the cell-centred CVs equal the exact
    polygon areas.  Catches clipping on the wrong side, a dropped polygon in
    the divergence theorem and wrong face areas on vertical facets."""
    g = synth.Grid((8, 8, 8), (0.125, 0.125, 0.125))
    x, y, z = synth.node_coords3(g)
    n = np.array(normal)
    d0 = 0.51
    phi = n[0] * x[None, None, :] + n[1] * y[None, :, None] + n[2] * z[:, None, None] - d0
    o = oracle.Oracle(g, phi_nodes=np.ascontiguousarray(phi))
    dv = 0.125 ** 3
    nx, ny, nz = g.n
    checked = 0
    for inst in range(4):
        al = o.alpha(inst)
        for k in range(nz + 1):
            if (inst == 3 and not 1 <= k <= nz - 1) or (inst != 3 and k == nz):
                continue
            for j in range(ny):
                for i in range(nx):
                    if (inst == 1 and i == 0) or (inst == 2 and j == 0):
                        continue
                    lo = [i * 0.125, j * 0.125, k * 0.125]
                    hi = [v + 0.125 for v in lo]
                    if inst:
                        lo[inst - 1] -= 0.0625
                        hi[inst - 1] -= 0.0625
                    solid = halfspace_box_volume(lo, hi, tuple(n), d0)
                    assert abs(al[k, j, i] - (1.0 - solid / dv)) <= 1e-13, (inst, i, j, k)
                    checked += 1
    G = o.geo[0]
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                x0, y0, z0 = i * 0.125, j * 0.125, k * 0.125
                # x-face at x0: fluid where n1 y + n2 z + (n0 x0 - d0) > 0
                A, _ = polygon_area_centroid(clip_polygon(rect(y0, y0 + 0.125, z0, z0 + 0.125),
                                                          n[1], n[2], n[0] * x0 - d0))
                assert abs(G[OQ["BX"], k, j, i] - A / 0.125 ** 2) <= 1e-13
                A, _ = polygon_area_centroid(clip_polygon(rect(x0, x0 + 0.125, z0, z0 + 0.125),
                                                          n[0], n[2], n[1] * y0 - d0))
                assert abs(G[OQ["BY"], k, j, i] - A / 0.125 ** 2) <= 1e-13
    assert checked > 1500


@pytest.mark.parametrize("name", ["hemisphere", "cylinder"])
def test_closure_every_cv_levelset(name):
    """Divergence theorem per CV on the paper's two level-set geometries:
    beta_hi - beta_lo = a_d (EB area vector into the fluid over the d-face
    area), all four instances; the EB area is at least the length of its
    vector.  Catches an EB facet booked twice or not at all (vertical walls,
    the cylinder's top face lying on a grid plane) and a mis-signed facet."""
    w = synth.make_levelset_workload(name)
    o = oracle.Oracle(w.grid, phi_nodes=w.phi_nodes)
    nx, ny, nz = w.grid.n
    dx, dy, dz = w.grid.dx
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
        vec = np.sqrt((G[OQ["AX"]] * dy * dz) ** 2 + (G[OQ["AY"]] * dx * dz) ** 2 + (G[OQ["AZ"]] * dx * dy) ** 2)
        assert np.all(G[OQ["AREA"]] * dx * dy >= vec * (1 - 1e-12) - 1e-15)
    # the cylinder's top lies on the node plane z = 3: the facet belongs to
    # the cells above it, whose bottom faces carry no fluid
    if name == "cylinder":
        k = int(round(3.0 / dz))
        G = o.geo[0]
        top = (o.ctype[0][k - 1] == 0) & (G[OQ["AREA"], k] > 0.99)
        assert top.sum() > 20
        assert np.all(G[OQ["BZ"], k][top] == 0.0) and np.all(G[OQ["ALPHA"], k][top] == 1.0)
        assert np.allclose(G[OQ["AZ"], k][top], 1.0, atol=1e-14)


def test_pieces_add_up():
    """The two halves of a cell along each axis add up to the whole cell
    (volume, EB area vector and area, the faces they share with it), and the
    mid-plane face is the same from both sides.  Catches a mid-plane
    half-space on the wrong side and a cross-section missing from the
    divergence theorem."""
    w = synth.make_levelset_workload("hemisphere")
    g, phi = w.grid, w.phi_nodes
    rng = np.random.default_rng(11)
    n = 0
    for _ in range(1500):
        i, j, k = int(rng.integers(18, 46)), int(rng.integers(18, 46)), int(rng.integers(0, 14))
        P = [oracle.levelset_piece(g, phi, i, j, k, p) for p in range(7)]
        if P[0][14] != 2:
            continue
        n += 1
        for d in range(3):
            a, b = P[1 + 2 * d], P[2 + 2 * d]
            s = P[0][0]
            assert abs(a[0] + b[0] - s) <= 1e-15 + 1e-12 * s
            assert np.allclose(a[4:8] + b[4:8], P[0][4:8], rtol=0, atol=1e-15)
            assert abs(a[8 + 2 * d + 1] - b[8 + 2 * d]) <= 1e-16
            assert abs(a[8 + 2 * d] - P[0][8 + 2 * d]) <= 1e-16
            assert abs(b[8 + 2 * d + 1] - P[0][8 + 2 * d + 1]) <= 1e-16
            for e in range(3):
                if e != d:
                    for side in range(2):
                        f = 8 + 2 * e + side
                        assert abs(a[f] + b[f] - P[0][f]) <= 1e-15
    assert n > 40


def test_brute_force_sampling_non_terrain_level_set():
    """A level set that is not a terrain (its zero set bends across the
    tetrahedra of a cell): alpha of every CV of all four instances and the
    lower x- and y-face fractions of the cell-centred CVs against sampling of
    the interpolant written from its definition (sorted unit coordinates),
    exact along z.  Catches a wrong tetrahedron vertex order, a wrong linear
    function inside a tetrahedron and a staggered CV assembled from the wrong
    halves."""
    g = synth.Grid((6, 6, 4), (1.0, 1.0, 0.5))
    x, y, z = synth.node_coords3(g)
    X, Y = np.meshgrid(x, y)
    h = 0.2 + 1.1 * np.exp(-((X - 3.1) ** 2 + (Y - 2.7) ** 2) / 2.0)
    Z = z[:, None, None]
    phi = (Z - h[None]) * (1.0 + 0.3 * np.sin(X) * np.cos(Y))[None] + 0.15 * np.sin(2.0 * Z + X[None])
    phi = synth._periodic_fix3(np.ascontiguousarray(phi))
    assert np.all(np.diff(phi, axis=0) >= 0)
    o = oracle.Oracle(g, phi_nodes=phi)
    nx, ny, nz = g.n
    M = 96
    cnt = 0
    for inst in range(4):
        al = o.alpha(inst)
        for k in range(nz + 1):
            if (inst == 3 and not 1 <= k <= nz - 1) or (inst != 3 and k == nz):
                continue
            for j in range(ny):
                for i in range(nx):
                    if (inst == 1 and i == 0) or (inst == 2 and j == 0):
                        continue
                    lo = [i * 1.0, j * 1.0, k * 0.5]
                    hi = [lo[0] + 1.0, lo[1] + 1.0, lo[2] + 0.5]
                    if inst:
                        lo[inst - 1] -= 0.5 * g.dx[inst - 1]
                        hi[inst - 1] -= 0.5 * g.dx[inst - 1]
                    xs = lo[0] + (np.arange(M) + 0.5) / M
                    ys = lo[1] + (np.arange(M) + 0.5) / M
                    PX, PY = np.meshgrid(xs, ys)
                    L = levelset_fluid_length(phi, g, PX, PY, lo[2], hi[2])
                    assert abs(al[k, j, i] - L.mean() / 0.5) < 2e-3, (inst, i, j, k, al[k, j, i], L.mean() / 0.5)
                    cnt += 1
    G = o.geo[0]
    s = (np.arange(4 * M) + 0.5) / (4 * M)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                bx = levelset_fluid_length(phi, g, np.full(s.shape, i * 1.0), j + s, k * 0.5, k * 0.5 + 0.5)
                assert abs(G[OQ["BX"], k, j, i] - bx.mean() / 0.5) < 1e-3
    assert cnt > 400


def test_hemisphere_volume_second_order():
    """The solid volume of the reconstructed hemisphere approaches 2/3 pi a^3
    from below (the interpolant of a convex distance lies above it) at second
    order: halving the mesh spacing divides the error by about 4.  Catches
    facets placed off the interpolated zero set."""
    errs = []
    for n in (16, 32):
        d = 1.25 / n
        g = synth.Grid((2 * n, 2 * n, n), (d, d, d))
        o = oracle.Oracle(g, phi_nodes=synth.levelset_hemisphere(g, 0.5))
        solid = math.fsum(((1.0 - o.alpha(0)[:n]) * d ** 3).ravel().tolist())
        exact = 2.0 / 3.0 * math.pi * 0.5 ** 3
        errs.append((exact - solid) / exact)
    assert 0 < errs[1] < errs[0] < 0.05, errs
    assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_level_set_must_be_monotone_in_z():
    """A level set that decreases along z somewhere (an overhang) is refused:
    the column structure (covered, cut, regular from the bottom up) would not
    hold."""
    g = synth.Grid((6, 6, 4), (1.0, 1.0, 1.0))
    x, y, z = synth.node_coords3(g)
    phi = np.broadcast_to(z[:, None, None] - 1.5, (5, 7, 7)).copy()
    phi[2, 3, 3] = -5.0
    with pytest.raises(ValueError):
        oracle.Oracle(g, phi_nodes=phi)
