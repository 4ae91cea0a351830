"""Pins of the oracle's thermal diffusion of rho theta (Section 4.2: flux
rho alpha_theta grad(theta), gradients on cut faces and at EB facets from a
least-squares fit of a second-order polynomial over a local neighbourhood,
3 wide on the variable's own grid and 4 wide along the direction in which a
face centroid sits between two cells) against closed forms.  CPU only.  Each
test names the mistake it exists to catch."""
import math
from dataclasses import dataclass

import numpy as np
import pytest

import oracle
import synth
from tests.helpers import clip_polygon, polygon_area_centroid, rect

OQ = oracle.OQ


@dataclass
class Diff:
    alpha_theta: float = 2.5
    eb_mode: int = 0
    theta_wall: float = 0.0


def _centroids(o, g):
    """Physical volume centroid of every cell (dense instance-0 storage)."""
    nx, ny, nz = g.n
    k, j, i = np.meshgrid(np.arange(nz + 1.0), np.arange(ny * 1.0), np.arange(nx * 1.0), indexing="ij")
    G = o.geo[0]
    return [g.lo[0] + (i + 0.5 + G[OQ["VCX"]]) * g.dx[0], g.lo[1] + (j + 0.5 + G[OQ["VCY"]]) * g.dx[1],
            g.lo[2] + (k + 0.5 + G[OQ["VCZ"]]) * g.dx[2]]


def _state_from_theta(g, theta_dense, rho=1.0):
    U = synth.state_uniform(g, rho=rho, theta=1.0, u=0.0)
    nz = g.n[2]
    U["rhotheta"] = rho * theta_dense[:nz].copy()
    return U


def test_constant_theta_has_no_diffusive_flux():
    """Uniform theta with random densities, the EB held at the same theta:
    every face and facet gradient vanishes (fits reproduce constants).
    Catches a fit or a difference that does not annihilate constants and an
    EB term with the wrong reference value."""
    w = synth.make_workload(1)
    o = oracle.Oracle(w.grid, w.h_nodes)
    rng = np.random.default_rng(5)
    U = synth.state_uniform(w.grid, rho=1.0, theta=300.0, u=0.0)
    rho = 1.0 + rng.random(U["rho"].shape)
    U["rho"] = rho
    U["rhotheta"] = rho * 300.0
    D = o.diffusion(U, Diff(eb_mode=1, theta_wall=300.0))
    scale = 2.5 * 300.0 * 2.0 / min(w.grid.dx) ** 2
    a = o.alpha(0)
    assert np.abs(a * D)[a > 0].max() <= 1e-10 * scale


def test_regular_cells_quadratic_exact():
    """No terrain: with point values of a quadratic at the cell centres and
    rho = 1, the centred face differences are the exact derivatives at the
    face centres, so D = alpha_theta (2 a + 2 b + 2 c) for
    theta = a x^2 + b y^2 + c z^2 + (linear and cross terms) away from the
    seams and the adiabatic walls.  Catches a wrong spacing or sign in the
    face difference and a wrong face density."""
    g = synth.Grid((12, 10, 8), (1.0, 1.5, 0.75))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    X, Y, Z = _centroids(o, g)
    a, b, c = 0.3, -0.2, 0.45
    th = a * X * X + b * Y * Y + c * Z * Z + 0.7 * X - 0.1 * Z + 0.05 * X * Y + 0.02 * Y * Z
    U = _state_from_theta(g, th)
    p = Diff(alpha_theta=1.7)
    D = o.diffusion(U, p)
    want = p.alpha_theta * 2 * (a + b + c)
    inner = D[1:g.n[2] - 1, 1:-1, 1:-1]
    assert np.allclose(inner, want, rtol=1e-10, atol=0)


PLANE = (2.3, 0.21, 0.13)


def _plane_setup():
    g = synth.Grid((12, 12, 8), (1.0, 1.25, 0.9))
    a, bx, by = PLANE
    return g, oracle.Oracle(g, synth.terrain_plane(g, a, bx, by))


def _face_centroid(g, d, i, j, k):
    """Fluid centroid of the lower d-face of cell (i, j, k) on the plane
    (independent clipper), and its area fraction."""
    a, bx, by = PLANE
    dx = g.dx
    x0, y0, z0 = i * dx[0], j * dx[1], k * dx[2]
    if d == 0:
        poly = clip_polygon(rect(0, dx[1], 0, dx[2]), -by, 1.0, z0 - (a + bx * x0 + by * y0))
        A, (u, v) = polygon_area_centroid(poly)
        return A / (dx[1] * dx[2]), np.array([x0, y0 + u, z0 + v])
    if d == 1:
        poly = clip_polygon(rect(0, dx[0], 0, dx[2]), -bx, 1.0, z0 - (a + bx * x0 + by * y0))
        A, (u, v) = polygon_area_centroid(poly)
        return A / (dx[0] * dx[2]), np.array([x0 + u, y0, z0 + v])
    poly = clip_polygon(rect(0, dx[0], 0, dx[1]), -bx, -by, z0 - (a + bx * x0 + by * y0))
    A, (u, v) = polygon_area_centroid(poly)
    return A / (dx[0] * dx[1]), np.array([x0 + u, y0 + v, z0])


def test_cut_face_gradient_exact_for_quadratics():
    """Sloped plane, theta given as point values of a quadratic at the cell
    centroids (rho = 1): the fitted gradient at the centroid of every cut
    face whose 4 x 3 x 3 stencil holds at least 10 fluid cells is the exact
    derivative there, from an independent polygon clipper.  Catches a fit at
    the face centre instead of the centroid and a linear-only fit."""
    g, o = _plane_setup()
    X, Y, Z = _centroids(o, g)
    q = lambda x, y, z: 0.4 * x * x - 0.3 * y * y + 0.25 * z * z + 0.2 * x * y - 0.15 * x * z + 0.1 * y * z + x - 2 * z
    grad = lambda x, y, z: np.array([0.8 * x + 0.2 * y - 0.15 * z + 1.0, -0.6 * y + 0.2 * x + 0.1 * z,
                                     0.5 * z - 0.15 * x + 0.1 * y - 2.0])
    U = _state_from_theta(g, q(X, Y, Z))
    p = Diff(alpha_theta=1.3)
    D, F, E = o.diffusion(U, p, fluxes=True)
    nx, ny, nz = g.n
    a = o.alpha(0)
    checked = 0
    for d in range(3):
        lo = [-1, -1, -1]
        hi = [1, 1, 1]
        lo[d] = -2
        for k in range(1, nz):
            for j in range(2, ny - 3):
                for i in range(2, nx - 3):
                    beta, c = _face_centroid(g, d, i, j, k)
                    if not (0.0 < beta < 1.0 - 1e-12):
                        continue
                    n = 0
                    for oz in range(lo[2], hi[2] + 1):
                        for oy in range(lo[1], hi[1] + 1):
                            for ox in range(lo[0], hi[0] + 1):
                                kk = k + oz
                                n += 0 <= kk <= nz - 1 and a[kk, j + oy, i + ox] > 0
                    if n < 10:
                        continue
                    want = p.alpha_theta * grad(*c)[d]
                    assert abs(F[d][k, j, i] - want) <= 1e-9 * (1 + abs(want)), (d, i, j, k, F[d][k, j, i], want)
                    checked += 1
    assert checked > 100, checked


def test_isothermal_eb_flux_exact():
    """Sloped plane with phi = z - h(x, y): theta = theta_w + a1 phi + a2 phi^2
    takes the wall value on the terrain, and the constrained quadratic fit
    reproduces it, so the EB term of every cut cell is
    -rho alpha_theta a1 |grad phi|^2 times the projected facet area (the
    facet normal is parallel to grad phi).  Catches a flipped facet normal,
    a fit that ignores the wall value, and an evaluation point other than
    the facet centroid."""
    g, o = _plane_setup()
    a0, bx, by = PLANE
    X, Y, Z = _centroids(o, g)
    phi = Z - (a0 + bx * X + by * Y)
    tw, a1, a2 = 290.0, 0.8, 0.05
    U = _state_from_theta(g, tw + a1 * phi + a2 * phi * phi, rho=1.2)
    p = Diff(alpha_theta=2.0, eb_mode=1, theta_wall=tw)
    D, F, E = o.diffusion(U, p, fluxes=True)
    nx, ny, nz = g.n
    dx = g.dx
    al = o.alpha(0)
    checked = 0
    for k in range(nz):
        for j in range(2, ny - 3):
            for i in range(2, nx - 3):
                if not al[k, j, i] > 0:
                    continue
                x0, y0, z0, z1 = i * dx[0], j * dx[1], k * dx[2], (k + 1) * dx[2]
                c0 = a0 + bx * x0 + by * y0
                poly = clip_polygon(rect(0, dx[0], 0, dx[1]), bx, by, c0 - z0)
                poly = clip_polygon(poly, -bx, -by, z1 - c0)
                Ap, _ = polygon_area_centroid(poly)
                if Ap <= 1e-9:
                    continue
                want = -1.2 * p.alpha_theta * a1 * (1 + bx * bx + by * by) * Ap
                assert abs(E[k, j, i] - want) <= 1e-9 * abs(want), (i, j, k, E[k, j, i], want)
                checked += 1
    assert checked > 50, checked


@pytest.mark.parametrize("cfg", [1, 2])
def test_conservation_with_adiabatic_eb(cfg):
    """Adiabatic EB and walls: every face flux enters the two cells on its
    sides with opposite signs, so sum V D = 0 for any state.  Catches a face
    flux computed differently by the two cells that share it."""
    w = synth.make_workload(cfg)
    o = oracle.Oracle(w.grid, w.h_nodes)
    U = synth.state_random(w.grid, 13, amp=1.0)
    D = o.diffusion(U, Diff(alpha_theta=3.0))
    V = o.volume(0)
    tot = math.fsum((V * D).ravel().tolist())
    scale = math.fsum(np.abs(V * D).ravel().tolist())
    assert abs(tot) <= 1e-13 * scale, (tot, scale)


def test_diffusion_enters_the_stage():
    """With a diffusion setting the provisional rho theta gains cdt D and no
    other field changes."""
    w = synth.make_workload(1)
    o = oracle.Oracle(w.grid, w.h_nodes)
    U = synth.make_state(w)
    p = Diff(alpha_theta=1e-3, eb_mode=1, theta_wall=299.0)
    cdt = w.dt / 3
    a = o.advance(U, U, cdt)
    b = o.advance(U, U, cdt, diff=p)
    D = oracle.from_dense([np.zeros_like(o.alpha(0)), o.diffusion(U, p)] + [np.zeros_like(o.alpha(0))] * 3, o.n)
    assert np.allclose(b["rhotheta"] - a["rhotheta"], cdt * D["rhotheta"], rtol=0, atol=1e-12)
    for f in ("rho", "rhou", "rhov", "rhow"):
        assert np.array_equal(a[f], b[f])


@pytest.mark.parametrize("d", [0, 1])
def test_cut_face_stencil_symmetric_about_the_face(d):
    """Flat terrain at 0.73 dz cuts the faces of the bottom layer.  theta an
    even function of the distance to one face plane (fourth power, not
    reproduced by the fit): with the stencil two cells deep on each side of
    the face the fitted normal gradient there is zero by symmetry.  Catches
    a stencil shifted along the face normal (one cell on one side, three on
    the other)."""
    g = synth.Grid((12, 12, 6), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.73))
    X, Y, Z = _centroids(o, g)
    f0 = 6.0
    r = (X if d == 0 else Y) - f0
    U = _state_from_theta(g, r ** 4 + 0.3 * Z * Z)
    _, F, _ = o.diffusion(U, Diff(alpha_theta=1.0), fluxes=True)
    plane = F[d][0, :, 6] if d == 0 else F[d][0, 6, :]
    assert np.all(o.geo[0][OQ["BX"] + d][0] < 1.0)
    assert np.abs(plane).max() <= 1e-12, plane
    # one cell further the same field has a non-zero gradient
    off = F[d][0, :, 7] if d == 0 else F[d][0, 7, :]
    assert np.abs(off).min() > 1e-3
