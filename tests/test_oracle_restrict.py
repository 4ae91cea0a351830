"""Pins of the oracle restriction between two levels (refinement ratio 2,
Section 4.3): merged geometry and conservative averaging.  CPU only.

- terrains that both resolutions represent exactly (flat, tilted plane): the
  merged fine geometry equals the geometry built directly on the coarse grid;
- the mass (and rho theta) of every coarse cell equals that of its children;
- the mass flux through every coarse face equals that through its four fine
  faces;
- a uniform field stays uniform; a linear field on fully regular cells gives
  its value at the coarse cell centre; covered coarse cells and the wall faces
  of the z momentum are zero."""
import numpy as np
import pytest

import oracle
import synth


def _fine_case():
    g = synth.Grid((24, 20, 16), (78.125, 78.125, 31.25))
    return g, synth.terrain_agnesi(g, h0=200.0, a=400.0)


def _coarse(g):
    return synth.Grid((g.n[0] // 2, g.n[1] // 2, g.n[2] // 2), tuple(2 * d for d in g.dx), g.lo)


@pytest.fixture(scope="module")
def hill():
    g, h = _fine_case()
    return g, h, oracle.Oracle(g, h)


@pytest.mark.parametrize("kind", ["flat", "plane"])
def test_merged_geometry_equals_coarse_geometry(kind):
    """Flat ground and a tilted plane are exact on both grids, so merging the
    fine subcells must reproduce the coarse grid's own volume and lower-face
    area fractions (the coarse geometry is built independently)."""
    g = synth.Grid((16, 12, 12), (50.0, 50.0, 25.0))
    gc = _coarse(g)
    if kind == "flat":
        hf, hc = synth.terrain_flat(g, 37.0), synth.terrain_flat(gc, 37.0)
    else:
        # a periodic tent in x, linear between its kinks at x = 0 and x = 400 m,
        # which are coarse nodes: both grids' interpolants reproduce it exactly
        xf = np.arange(g.n[0] + 1) * g.dx[0]
        hf = np.broadcast_to(40.0 + 0.08 * np.minimum(xf, 800.0 - xf), (g.n[1] + 1, g.n[0] + 1)).copy()
        hc = hf[::2, ::2].copy()
    fo, co = oracle.Oracle(g, hf), oracle.Oracle(gc, hc)
    a, b = fo.coarsened_geometry()
    nzc = gc.n[2]
    np.testing.assert_allclose(a, co.alpha(0)[:nzc], rtol=0, atol=1e-14)
    for d in range(3):
        np.testing.assert_allclose(b[d], co.geo[0][oracle.OQ["BX"] + d][:nzc], rtol=0, atol=1e-14)
    assert ((a > 0.0) & (a < 1.0)).any()  # cut coarse cells are present


def test_mass_of_every_coarse_cell(hill):
    g, h, o = hill
    U = synth.state_random(g, 3)
    Uc = o.restrict(U)
    a, _ = o.coarsened_geometry()
    nx, ny, nz = g.n
    af = o.alpha(0)[:nz]
    for f in ("rho", "rhotheta"):
        fine = (af * U[f]).reshape(nz // 2, 2, ny // 2, 2, nx // 2, 2).sum(axis=(1, 3, 5))
        coarse = 8.0 * a * Uc[f]
        np.testing.assert_allclose(coarse, fine, rtol=1e-13, atol=1e-13 * np.abs(fine).max())
    assert np.all(Uc["rho"][a == 0.0] == 0.0) and (a == 0.0).any()


def test_mass_flux_through_every_coarse_face(hill):
    g, h, o = hill
    U = synth.state_random(g, 4)
    Uc = o.restrict(U)
    _, b = o.coarsened_geometry()
    nx, ny, nz = g.n
    D = oracle.to_dense(U, o.n)
    Dc = oracle.to_dense(Uc, (nx // 2, ny // 2, nz // 2))
    for d, f in enumerate(("rhou", "rhov", "rhow")):
        beta = o.geo[0][oracle.OQ["BX"] + d][:nz]
        flux = beta * D[2 + d][:nz]
        # keep the fine faces that lie on coarse faces (even index along d)
        sl = [slice(None)] * 3
        sl[2 - d] = slice(0, None, 2)
        flux = flux[tuple(sl)]
        sh = list(flux.shape)
        # sum the four fine faces of each coarse face (pairs along the other axes)
        axes = [ax for ax in range(3) if ax != 2 - d]
        shp = []
        for ax in range(3):
            shp += [sh[ax] // 2, 2] if ax in axes else [sh[ax], 1]
        fine = flux.reshape(shp).sum(axis=(1, 3, 5))
        coarse = 4.0 * b[d] * Dc[2 + d][:nz // 2]
        if d == 2:
            fine[0] = 0.0  # the bottom wall face is not restricted
        np.testing.assert_allclose(coarse, fine, rtol=1e-13, atol=1e-13 * np.abs(fine).max())


def test_uniform_and_linear_fields(hill):
    g, h, o = hill
    nx, ny, nz = g.n
    Uu = synth.state_uniform(g, rho=1.1, theta=300.0, u=7.0, v=-2.0, w=0.5)
    Uc = o.restrict(Uu)
    a, _ = o.coarsened_geometry()
    m = a > 0
    assert np.allclose(Uc["rho"][m], 1.1, rtol=1e-15) and np.allclose(Uc["rhotheta"][m], 330.0, rtol=1e-15)
    Dc = oracle.to_dense(Uc, (nx // 2, ny // 2, nz // 2))
    for d, val in enumerate((7.7, -2.2, 0.55)):
        x = Dc[2 + d][:nz // 2]
        nzv = x != 0.0
        if d == 2:
            nzv[0] = False
        np.testing.assert_allclose(x[nzv], val, rtol=1e-14)
    assert np.all(Uc["rhow"][0] == 0.0) and np.all(Uc["rhow"][-1] == 0.0)
    # linear in x on coarse cells whose children are all regular
    xc = (np.arange(nx) + 0.5) * g.dx[0]
    Ul = dict(Uu)
    Ul["rho"] = np.broadcast_to(1.0 + 1e-4 * xc[None, None, :], (nz, ny, nx)).copy()
    Uc = o.restrict(Ul)
    full = a == 1.0
    assert full.sum() > 100
    want = 1.0 + 1e-4 * ((np.arange(nx // 2) + 0.5) * 2 * g.dx[0])
    np.testing.assert_allclose(Uc["rho"][full], np.broadcast_to(want, a.shape)[full], rtol=1e-14)
