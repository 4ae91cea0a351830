"""Pins of the oracle flux divergence and stage update (Sections 3.1 and 4.1 of
the paper, Eqs. update-cc / update-fc) against invariants and closed forms.
CPU only."""
import math

import numpy as np
import pytest

import oracle
import synth

FIELDS = oracle.FIELDS


def _rel_change(o, U, cdt, flux_scale):
    Uh = o.advance(U, U, cdt)
    D0 = oracle.to_dense(U, o.n)
    D1 = oracle.to_dense(Uh, o.n)
    out = []
    for f in range(5):
        a = o.alpha(oracle.FIELD_INST[f])
        m = a > 0
        # extensive form alpha * dU: the closure residual is not amplified by
        # the 1/alpha of sliver cells
        out.append(np.abs(a * (D1[f] - D0[f]))[m].max() / flux_scale[f])
    return out


@pytest.mark.parametrize("cfg,vel", [(1, (10.0, 0.0)), (1, (0.0, 10.0)), (2, (10.0, 0.0)),
                                     (1, (-4.0, 7.0)), (2, (10.0, -3.0))])
def test_free_stream_closure_mode(cfg, vel):
    """With the EB flux set to -(area vector . mean provisional flux), uniform
    flow is an exact steady state on every CV of the four instances (closure of
    the cut-cell geometry; the interpolation weights sum to one; the reduced
    stencils are exact for constants).  With two non-zero velocity
    components this also needs the mass flux through a staggered face to be
    the mean over the fluid momentum CVs next to it: a covered one read as 0
    would halve the flux through a face whose area fraction already counts
    only the open half."""
    w = synth.make_workload(cfg)
    g = w.grid
    o = oracle.Oracle(g, w.h_nodes, eb_flux=1)
    U = synth.state_uniform(g, rho=1.2, theta=300.0, u=vel[0], v=vel[1])
    sp = max(abs(vel[0]), abs(vel[1]))
    scale = [1.2 * sp / min(g.dx), 360 * sp / min(g.dx)] + [1.2 * sp * sp / min(g.dx)] * 3
    ch = _rel_change(o, U, 1.0, scale)
    assert max(ch) < 1e-12, ch
    # the no-flux wall closes the EB for mass, so the same flow is not steady
    o.set_mode(eb_flux=0)
    ch0 = _rel_change(o, U, 1.0, scale)
    assert max(ch0) > 1e-3


def test_flat_terrain_uniform_flow_is_steady_with_wsrd():
    """Flat terrain at 0.73 dz (a layer of small cut cells), uniform wind along
    x: one full stage (update + redistribution) leaves the state unchanged."""
    g = synth.Grid((12, 10, 6), (78.125, 78.125, 31.25))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.73 * 31.25))
    U = synth.state_uniform(g, rho=1.1, theta=301.0, u=10.0)
    U1 = o.stage(U, U, 0.5)
    for f in FIELDS:
        inst = oracle.FIELD_INST[FIELDS.index(f)]
        m = o.export(inst, oracle.OQ["ALPHA"]) > 0
        ref = np.abs(U[f]).max() or 1.0
        assert np.abs(U1[f] - U[f])[m].max() / ref < 1e-14, f


def _quad_cell_avg(c2, c1, c0, a, b):
    """Average of c2 x^2 + c1 x + c0 over [a, b]."""
    F = lambda x: c2 * x ** 3 / 3 + c1 * x ** 2 / 2 + c0 * x
    return (F(b) - F(a)) / (b - a)


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("d", [0, 1, 2])
def test_upwind_reproduces_quadratics(sign, d):
    """Third-order upwind (fourth-order centred plus hyperviscosity) is exact
    for cell averages of quadratics: on uncut cells the provisional rho-theta
    flux divided by the mass flux equals the quadratic at the face."""
    g = synth.Grid((12, 12, 12), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    U = synth.state_uniform(g, rho=1.0, theta=0.0, u=0.0)
    q = (0.37, -1.3, 2.0)
    idx = np.arange(12, dtype=float)
    avg = np.array([_quad_cell_avg(*q, x, x + 1) for x in idx])
    shape = [1, 1, 1]
    shape[2 - d] = 12
    U["rhotheta"] = np.broadcast_to(avg.reshape(shape), (12, 12, 12)).copy()
    name = ("rhou", "rhov", "rhow")[d]
    U[name][...] = 2.5 * sign
    U["rhow"][0] = 0.0
    U["rhow"][-1] = 0.0
    F, Fh = o.face_fluxes(U, 1)
    Fd = np.moveaxis(Fh[d], 2 - d, 0)  # face index along d first
    for f in range(3, 10):  # faces whose 4-point stencil stays inside
        exact = q[0] * f * f + q[1] * f + q[2]
        plane = Fd[f] if d == 2 else Fd[f][:12]  # drop the pseudo plane above the top
        got = plane.ravel() / (2.5 * sign)
        assert np.allclose(got, exact, rtol=0, atol=1e-12), (d, f)


def test_order_reduction_when_upstream_cell_covered():
    """Flat terrain at 1.5 dz: layer 0 is covered.  Upward mass flux through
    the face between layers 1 and 2 has its upwind end in layer 0, so the face
    value is the second-order centred mean; one face higher it is third order."""
    g = synth.Grid((8, 8, 8), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 1.5))
    U = synth.state_uniform(g, rho=1.0, theta=0.0, u=0.0)
    th = np.array([0.0, 3.0, 5.0, 11.0, 13.0, 17.0, 19.0, 23.0])
    U["rhotheta"] = np.broadcast_to(th[:, None, None], (8, 8, 8)).copy()
    U["rhow"][1:-1] = 1.0
    _, Fh = o.face_fluxes(U, 1)
    assert np.allclose(Fh[2][2], (3.0 + 5.0) / 2)
    assert np.allclose(Fh[2][3], (-3.0 + 5 * 5.0 + 2 * 11.0) / 6)
    U["rhow"][1:-1] = -1.0
    _, Fh = o.face_fluxes(U, 1)
    assert np.allclose(Fh[2][2], -(2 * 3.0 + 5 * 5.0 - 11.0) / 6)


def test_cut_face_centroid_interpolation_is_bilinear_exact():
    """On the cut x-faces of the flat-terrain layer (fluid from 0.73 dz to dz,
    centroid 0.365 dz above the face centre) the flux is moved to the centroid:
    a mass flux linear in y and z gives the exact value at the centroid."""
    g = synth.Grid((10, 10, 6), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.73))
    U = synth.state_uniform(g, rho=1.0, theta=2.0, u=0.0)
    nz, ny, nx1 = U["rhou"].shape
    yc = np.arange(ny) + 0.5
    zc = np.arange(nz) + 0.5
    U["rhou"] = (3.0 + 0.25 * yc[None, :, None] + 0.5 * zc[:, None, None]) * np.ones((nz, ny, nx1))
    F, Fh = o.face_fluxes(U, 1)
    zcent = 0.73 + (1.0 - 0.73) / 2
    expect = 2.0 * (3.0 + 0.25 * yc[:, None] + 0.5 * zcent) * np.ones((1, nx1 - 1))
    assert np.allclose(F[0][0], expect, rtol=0, atol=1e-12)
    assert not np.allclose(Fh[0][0], expect)


@pytest.mark.parametrize("cfg", [1, 2])
def test_telescoping_conservation_random_state(cfg):
    """Every interior face flux enters two CVs with opposite signs and walls
    carry none, so sum V U-hat = sum V U^n for any state (all five fields)."""
    w = synth.make_workload(cfg)
    o = oracle.Oracle(w.grid, w.h_nodes)
    U = synth.state_random(w.grid, 11, amp=3.0)
    Uh = o.advance(U, U, 0.3 * w.dt)
    s0 = o.conserved_sums(U)
    s1 = o.conserved_sums(Uh)
    D0 = oracle.to_dense(U, o.n)
    D1 = oracle.to_dense(Uh, o.n)
    for f in range(5):
        V = o.volume(oracle.FIELD_INST[f])
        scale = math.fsum((V * (np.abs(D0[f]) + np.abs(D1[f] - D0[f]))).ravel().tolist())
        assert abs(s1[f] - s0[f]) <= 1e-14 * scale, (f, s1[f] - s0[f], scale)


def test_third_order_convergence_smooth_advection():
    """Without terrain the rho-theta update for a sine wave advected along x
    converges at third order (operator truncation error on cell averages)."""
    errs = []
    for n in (16, 32, 64):
        g = synth.Grid((n, 8, 4), (1.0 / n, 1.0 / 8, 1.0 / 4))
        o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
        U = synth.state_uniform(g, rho=1.0, theta=0.0, u=1.0)
        x = np.arange(n + 1) / n
        avg = (np.cos(2 * np.pi * x[:-1]) - np.cos(2 * np.pi * x[1:])) / (2 * np.pi / n)
        U["rhotheta"] = np.broadcast_to(avg[None, None, :], (4, 8, n)).copy()
        Uh = o.advance(U, U, 1.0)
        dU = Uh["rhotheta"] - U["rhotheta"]
        exact = -(np.sin(2 * np.pi * x[1:]) - np.sin(2 * np.pi * x[:-1])) * n
        errs.append(np.abs(dU - exact[None, None, :]).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert r1 > 7.0 and r2 > 7.5, errs
