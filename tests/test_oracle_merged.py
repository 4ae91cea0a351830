"""Pins of the oracle's merged coarse geometry (Section 4.3: the coarse level
of a two-level hierarchy takes its geometry from the fine one by merging
subcells, so that volumes and areas agree between the levels).  CPU only.
Each test names the mistakes it exists to catch."""
import math

import numpy as np
import pytest

import oracle
import synth

OQ = oracle.OQ


def _coarse(g):
    return synth.Grid(tuple(n // 2 for n in g.n), tuple(2 * d for d in g.dx), g.lo, g.small_vfrac)


def _cases():
    w = synth.make_workload(1)
    yield "c1", w.grid, dict(h_nodes=w.h_nodes)
    w = synth.make_levelset_workload("hemisphere")
    yield "hemisphere", w.grid, dict(phi_nodes=w.phi_nodes)


@pytest.mark.parametrize("case", ["c1", "hemisphere"])
def test_merged_alpha_beta_match_the_merged_fine_arrays(case):
    """The volume and lower-face fractions of the merged cell-centred CVs
    equal the means of the fine oracle's own fractions over the children
    (a different route: averaging the fine geometry arrays).  Catches fine
    cells gathered from the wrong offsets and faces taken from the wrong
    side of a coarse cell."""
    name, g, kw = next(c for c in _cases() if c[0] == case)
    of = oracle.Oracle(g, **kw)
    a, b = of.coarsened_geometry()
    oc = oracle.Oracle(_coarse(g), merged=True, **kw)
    nzc = g.n[2] // 2
    G = oc.geo[0]
    assert np.abs(G[OQ["ALPHA"], :nzc] - a).max() <= 1e-14
    for d, q in enumerate(("BX", "BY", "BZ")):
        assert np.abs(G[OQ[q], :nzc] - b[d]).max() <= 1e-14, q


@pytest.mark.parametrize("which", ["terrain_plane", "levelset_plane"])
def test_merged_equals_direct_coarse_build_on_planes(which):
    """A plane is represented exactly on both grids, so the geometry merged
    from the fine cells equals the geometry built directly on the coarse
    grid: all twenty quantities of all four instances, and every type.
    Catches a wrong shift of the children's moments, staggered CVs assembled
    from the wrong fine cells and centroids normalised on the fine spacing."""
    gf = synth.Grid((16, 16, 12), (0.5, 0.5, 0.25))
    gc = _coarse(gf)
    if which == "terrain_plane":
        hf = synth.terrain_plane(gf, 0.93, 0.11, -0.07)
        hc = synth.terrain_plane(gc, 0.93, 0.11, -0.07)
        om = oracle.Oracle(gc, h_nodes=hf, merged=True)
        od = oracle.Oracle(gc, hc)
    else:
        n = (0.3517, -0.2049, 0.9131)
        mk = lambda g: np.ascontiguousarray(
            n[0] * synth.node_coords3(g)[0][None, None, :] + n[1] * synth.node_coords3(g)[1][None, :, None]
            + n[2] * synth.node_coords3(g)[2][:, None, None] - 1.0537)
        om = oracle.Oracle(gc, phi_nodes=mk(gf), merged=True)
        od = oracle.Oracle(gc, phi_nodes=mk(gc))
    nx, ny, _ = gc.n
    for inst in range(4):
        # staggered CVs that straddle the periodic seam join the two ends of
        # a non-periodic plane
        keep = np.ones(od.ctype[inst].shape, bool)
        if inst == 1:
            keep[:, :, 0] = False
        if inst == 2:
            keep[:, 0, :] = False
        if which == "levelset_plane" or inst == 0:
            keep[:, :, -1] = False
            keep[:, -1, :] = False
        assert np.array_equal(om.ctype[inst][keep], od.ctype[inst][keep]), inst
        for q in range(oracle.OQ_N):
            # centroids as moments (their weight times the offset)
            w = {4: 1, 5: 1, 6: 2, 7: 2, 8: 3, 9: 3, 10: 0, 11: 0, 12: 0, 17: 16, 18: 16, 19: 16}.get(q)
            a, b = om.geo[inst][q], od.geo[inst][q]
            if w is not None:
                a, b = a * om.geo[inst][w], b * od.geo[inst][w]
            e = np.abs(a - b)[keep].max()
            assert e <= 1e-12, (inst, q, e)


def test_merged_closure_and_volume():
    """Every merged CV of all four instances is closed (the EB area vector
    equals the difference of its face fractions), and each instance holds
    the fluid volume of the fine cells it is made of.  Catches EB data or
    faces lost in the merge and staggered CVs made of the wrong cells."""
    w = synth.make_levelset_workload("hemisphere")
    gf = w.grid
    gc = _coarse(gf)
    of = oracle.Oracle(gf, phi_nodes=w.phi_nodes)
    oc = oracle.Oracle(gc, phi_nodes=w.phi_nodes, merged=True)
    nx, ny, nz = gc.n
    for inst in range(4):
        G = oc.geo[inst]
        cv = np.zeros((nz + 1, ny, nx), bool)
        cv[1:nz] = True
        if inst != 3:
            cv[0] = True
        for d, (qb, qa) in enumerate([("BX", "AX"), ("BY", "AY"), ("BZ", "AZ")]):
            lo = G[OQ[qb]]
            hi = (np.roll(lo, -1, axis=2) if d == 0 else np.roll(lo, -1, axis=1) if d == 1
                  else np.concatenate([lo[1:], np.zeros_like(lo[:1])], axis=0))
            assert np.abs((hi - lo) - G[OQ[qa]])[cv].max() < 1e-13, (inst, d)
    vf = of.alpha(0)[:gf.n[2]] * np.prod(gf.dx)
    vc = [oc.alpha(s) * np.prod(gc.dx) for s in range(4)]
    tot = math.fsum(vf.ravel().tolist())
    for s in range(3):
        assert abs(math.fsum(vc[s].ravel().tolist()) - tot) <= 1e-13 * tot, s
    inner = math.fsum(vf[1:-1].ravel().tolist())
    assert abs(math.fsum(vc[3].ravel().tolist()) - inner) <= 1e-13 * inner


def test_merged_free_stream():
    """On the merged coarse hemisphere, the closure test mode of the EB flux
    keeps a uniform flow in two directions steady to rounding: the merged
    face fractions, centroids and EB vectors are mutually consistent.
    Catches an EB vector merged without its faces."""
    w = synth.make_levelset_workload("hemisphere")
    gc = _coarse(w.grid)
    oc = oracle.Oracle(gc, phi_nodes=w.phi_nodes, merged=True, eb_flux=1)
    U = synth.state_uniform(gc, rho=1.2, theta=300.0, u=10.0, v=3.0, w=0.0)
    uh = oc.advance(U, U, 2 * w.dt / 3)
    for f, inst in zip(oracle.FIELDS, oracle.FIELD_INST):
        m = oc.export(inst, OQ["ALPHA"]) > 0
        if f == "rhow":
            m[0] = m[-1] = False
        scale = max(np.abs(U[f]).max(), 1.0)
        assert np.abs(uh[f] - U[f])[m].max() <= 1e-13 * scale, f
