"""Closed-form pins of the oracle geometry and cut-face interpolation on a
sloped planar terrain z = a + bx x + by y (Section 3.2: face area fractions,
face centroids, EB facet area, normal and centroid for all four instances;
Section 4.1: bilinear interpolation of provisional fluxes to the centroid of
a cut face, with neighbours chosen by the signs of the centroid offsets).
On a plane every one of these is a polygon of a face or box clipped by a
straight line, computed here by an independent clipper.  CPU only.  Each
test names the mistake it exists to catch."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import clip_polygon, polygon_area_centroid, rect

OQ = oracle.OQ
PLANE = (2.3, 0.21, 0.13)
N = (12, 12, 8)
DX = (1.0, 1.25, 0.9)


def _setup():
    g = synth.Grid(N, DX)
    a, bx, by = PLANE
    return g, oracle.Oracle(g, synth.terrain_plane(g, a, bx, by))


def _h(x, y):
    a, bx, by = PLANE
    return a + bx * x + by * y


def cv_box(inst, i, j, k):
    x0, y0, z0 = i * DX[0], j * DX[1], k * DX[2]
    box = [x0, x0 + DX[0], y0, y0 + DX[1], z0, z0 + DX[2]]
    if inst:
        d = inst - 1
        box[2 * d] -= 0.5 * DX[d]
        box[2 * d + 1] -= 0.5 * DX[d]
    return box


def face_fluid(box, d):
    """Fluid part of the lower d-face of a box: (area, centroid in the two
    tangential coordinates).  The polygon is clipped in coordinates relative
    to the face's lower corner (u0, v0), so a sliver's centroid keeps its
    digits."""
    a, bx, by = PLANE
    x0, x1, y0, y1, z0, z1 = box
    if d == 0:  # x = x0: fluid z > a + bx x0 + by y  <=>  z - by y - (a + bx x0) > 0
        u0, v0 = y0, z0
        poly = clip_polygon(rect(0, y1 - y0, 0, z1 - z0), -by, 1.0, z0 - (a + bx * x0 + by * y0))
    elif d == 1:
        u0, v0 = x0, z0
        poly = clip_polygon(rect(0, x1 - x0, 0, z1 - z0), -bx, 1.0, z0 - (a + by * y0 + bx * x0))
    else:  # z = z0: fluid where h(x, y) < z0
        u0, v0 = x0, y0
        poly = clip_polygon(rect(0, x1 - x0, 0, y1 - y0), -bx, -by, z0 - (a + bx * x0 + by * y0))
    A, (cu, cv) = polygon_area_centroid(poly)
    return A, (u0 + cu, v0 + cv)


def facet(box):
    """EB facet of the plane inside a box: projected area, area vector (into
    the fluid), true area and centroid."""
    a, bx, by = PLANE
    x0, x1, y0, y1, z0, z1 = box
    c0 = a + bx * x0 + by * y0  # h at the box's lower corner
    poly = rect(0, x1 - x0, 0, y1 - y0)
    poly = clip_polygon(poly, bx, by, c0 - z0)      # h >= z0
    poly = clip_polygon(poly, -bx, -by, z1 - c0)    # h <= z1
    Ap, (cx, cy) = polygon_area_centroid(poly)
    cx, cy = x0 + cx, y0 + cy
    n = np.array([-bx, -by, 1.0])
    return Ap, Ap * n, Ap * math.sqrt(1 + bx * bx + by * by), np.array([cx, cy, _h(cx, cy)])


def _cvs(inst):
    nx, ny, nz = N
    ks = range(1, nz) if inst == 3 else range(nz)
    for k in ks:
        for j in range(2, ny - 2):
            for i in range(2, nx - 2):
                yield i, j, k


def test_face_centroids_and_fractions_all_instances():
    """Lower-face area fractions and centroid offsets (FX1 .. FZ2) of every
    CV of the four instances away from the seams.  Catches swapped
    tangential offsets, offsets measured from the wrong face centre, and a
    staggered face assembled from the wrong half-faces."""
    g, o = _setup()
    farea = [DX[1] * DX[2], DX[0] * DX[2], DX[0] * DX[1]]
    tang = [(1, 2), (0, 2), (0, 1)]
    checked = 0
    for inst in range(4):
        G = o.geo[inst]
        for (i, j, k) in _cvs(inst):
            box = cv_box(inst, i, j, k)
            ctr = [(box[0] + box[1]) / 2, (box[2] + box[3]) / 2, (box[4] + box[5]) / 2]
            for d in range(3):
                A, (cu, cv) = face_fluid(box, d)
                assert abs(G[OQ["BX"] + d, k, j, i] - A / farea[d]) <= 1e-13, (inst, d, i, j, k)
                if A <= 1e-9 * farea[d]:
                    continue
                e1, e2 = tang[d]
                q = OQ["FX1"] + 2 * d
                # compared as moments (fraction x offset): a sliver's centroid
                # is a ratio of two small numbers
                b = A / farea[d]
                assert abs(b * (G[q, k, j, i] - (cu - ctr[e1]) / DX[e1])) <= 1e-13, (inst, d, i, j, k)
                assert abs(b * (G[q + 1, k, j, i] - (cv - ctr[e2]) / DX[e2])) <= 1e-13, (inst, d, i, j, k)
                checked += 0 < A < farea[d] * (1 - 1e-12)
    assert checked > 300, checked


def test_eb_facet_area_vector_and_centroid_all_instances():
    """EB area (per dx dy), area vector into the fluid (per face area) and
    facet centroid offsets of every CV of the four instances.  Catches a
    flipped normal, a centroid offset with the wrong sign or origin, and an
    area-weighted staggered centroid built from the wrong halves."""
    g, o = _setup()
    farea = [DX[1] * DX[2], DX[0] * DX[2], DX[0] * DX[1]]
    checked = 0
    for inst in range(4):
        G = o.geo[inst]
        for (i, j, k) in _cvs(inst):
            box = cv_box(inst, i, j, k)
            ctr = np.array([(box[0] + box[1]) / 2, (box[2] + box[3]) / 2, (box[4] + box[5]) / 2])
            Ap, av, A, c = facet(box)
            assert abs(G[OQ["AREA"], k, j, i] - A / (DX[0] * DX[1])) <= 1e-12
            for d in range(3):
                assert abs(G[OQ["AX"] + d, k, j, i] - av[d] / farea[d]) <= 1e-12, (inst, d)
            if Ap > 1e-9:
                w = A / (DX[0] * DX[1])
                for d in range(3):
                    assert abs(w * (G[OQ["EBX"] + d, k, j, i] - (c[d] - ctr[d]) / DX[d])) <= 1e-13, (inst, d)
                checked += 1
    assert checked > 300, checked


def _has_fluid(box, d):
    A, _ = face_fluid(box, d)
    return A > 0.0


@pytest.mark.parametrize("d", [0, 1, 2])
def test_cut_face_interpolation_two_offsets_bilinear_exact(d):
    """A mass flux bilinear in the face's two tangential coordinates and a
    uniform theta: on every cut d-face of the cell-centred instance whose
    three interpolation neighbours hold fluid, the flux used in the
    divergence equals theta times the mass flux at the face's fluid centroid
    (both offsets are non-zero on this plane).  Catches a dropped diagonal
    weight, a neighbour chosen against the sign of an offset, and weights
    that are not the absolute offsets."""
    g, o = _setup()
    nx, ny, nz = N
    th = 2.0
    A0, B, C, D = 3.0, 0.25, -0.4, 0.15
    U = synth.state_uniform(g, rho=1.0, theta=th, u=0.0)
    names = ("rhou", "rhov", "rhow")
    tang = [(1, 2), (0, 2), (0, 1)]
    e1, e2 = tang[d]
    sh = U[names[d]].shape
    k_, j_, i_ = np.meshgrid(*[np.arange(s, dtype=float) for s in sh], indexing="ij")
    pos = [(i_ + 0.5) * DX[0], (j_ + 0.5) * DX[1], (k_ + 0.5) * DX[2]]
    pos[d] = [i_, j_, k_][d] * DX[d]
    U[names[d]] = A0 + B * pos[e1] + C * pos[e2] + D * pos[e1] * pos[e2]
    if d == 2:
        U["rhow"][0] = U["rhow"][-1] = 0.0
    F, Fh = o.face_fluxes(U, 1)
    checked = 0
    for k in range(1 if d == 2 else 0, nz):
        for j in range(2, ny - 2):
            for i in range(2, nx - 2):
                box = cv_box(0, i, j, k)
                A, (cu, cv) = face_fluid(box, d)
                full = DX[e1] * DX[e2]
                if not (0.0 < A < full * (1 - 1e-12)):
                    continue
                ctr = [(box[0] + box[1]) / 2, (box[2] + box[3]) / 2, (box[4] + box[5]) / 2]
                su = int(np.sign(cu - ctr[e1]))
                sv = int(np.sign(cv - ctr[e2]))
                assert su != 0 and sv != 0
                idx = [i, j, k]
                ok = True
                for (a1, a2) in ((su, 0), (0, sv), (su, sv)):
                    n = list(idx)
                    n[e1] += a1
                    n[e2] += a2
                    if not (0 <= n[2] <= nz - 1):
                        ok = False
                        break
                    ok = ok and _has_fluid(cv_box(0, *n), d)
                if not ok:
                    continue
                expect = th * (A0 + B * cu + C * cv + D * cu * cv)
                assert abs(F[d][k, j, i] - expect) <= 1e-12 * abs(expect), (d, i, j, k)
                checked += 1
    assert checked > 20, checked
