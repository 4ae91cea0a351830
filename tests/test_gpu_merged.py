"""GPU parity of the two-level pieces (Section 4.3): the coarse level's
geometry merged from the fine cells, its redistribution tables, a coarse
stage, and the two-level sequence (fine stage, coarse stage, restriction of
the fine state onto the coarse level) against the FP64 oracle.

Bars: types and redistribution flags bit for bit; geometry <= 1e-13
(centroids as moments); weights <= 1e-12; FP64 states <= 1e-12 relative per
field on CVs with alpha > 1e-3 and within the sliver bound elsewhere; the
merged volume and face fractions equal those the restriction uses; after the
restriction the coarse mass and rho theta equal the fine ones to 1e-13."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_11959_amd as ebs  # noqa: E402

FIELDS = ebs.FIELDS
_WEIGHT = {4: 1, 5: 1, 6: 2, 7: 2, 8: 3, 9: 3, 10: 0, 11: 0, 12: 0, 17: 16, 18: 16, 19: 16}
_cache = {}


def _case(name):
    """(fine workload, fine nodes, keyword for the oracle, coarse grid)"""
    if name not in _cache:
        if name == "hemisphere":
            w = synth.make_levelset_workload("hemisphere")
            nodes, kw = w.phi_nodes, "phi_nodes"
        else:
            w = synth.make_workload({"c1": 1, "c2": 2}[name])
            nodes, kw = w.h_nodes, "h_nodes"
        g = w.grid
        gc = synth.Grid(tuple(n // 2 for n in g.n), tuple(2 * d for d in g.dx), g.lo, g.small_vfrac)
        of = oracle.Oracle(g, **{kw: nodes})
        oc = oracle.Oracle(gc, merged=True, **{kw: nodes})
        _cache[name] = (w, nodes, gc, of, oc)
    return _cache[name]


def _fine_ctx(w, nodes):
    c = ebs.Context(w.grid.n, w.grid.dx, w.grid.lo)
    if nodes.ndim == 2:
        c.build_geometry(nodes)
    else:
        c.build_geometry_levelset(nodes)
    return c


def _coarse_ctx(gc, nodes, name):
    print(f"[ctx] coarse of {name} {gc.n}", flush=True)
    c = ebs.Context(gc.n, gc.dx, gc.lo)
    c.build_geometry_merged(nodes)
    return c


def _host(U):
    return {k: v.double().cpu().numpy() for k, v in U.items()}


def _masks(o):
    m = {}
    for f, inst in zip(FIELDS, oracle.FIELD_INST):
        a = o.export(inst, oracle.OQ["ALPHA"]) > 0
        if f == "rhow":
            a[0] = a[-1] = False
        m[f] = a
    return m


def _check_state(got, want, o, U0, cdt, dmin, tag):
    masks = _masks(o)
    eps = np.finfo(np.float64).eps
    mom = max(np.abs(want[f][masks[f]]).max() for f in ("rhou", "rhov", "rhow"))
    mmax = max(np.abs(U0[f]).max() for f in ("rhou", "rhov", "rhow"))
    pos = U0["rho"] > 0  # the restricted state holds 0 on covered coarse cells
    vmax = mmax / U0["rho"][pos].min()
    tmax = np.abs(U0["rhotheta"][pos] / U0["rho"][pos]).max()
    fscale = {"rho": mmax, "rhotheta": mmax * tmax, "rhou": mmax * vmax, "rhov": mmax * vmax,
              "rhow": mmax * vmax}
    worst = 0.0
    for f, inst in zip(FIELDS, oracle.FIELD_INST):
        a = o.export(inst, oracle.OQ["ALPHA"])
        scale = np.abs(want[f][masks[f]]).max() if f in ("rho", "rhotheta") else mom
        d = np.abs(got[f] - want[f])
        big = masks[f] & (a > 1e-3)
        assert d[big].max() <= 1e-12 * scale, (tag, f, d[big].max() / scale)
        bound = 1e-12 * scale + eps * 6 * fscale[f] * cdt / (np.where(a > 0, a, 1.0) * dmin)
        ratio = (d / bound)[masks[f]].max()
        worst = max(worst, ratio)
        assert ratio <= 1.0, (tag, f, ratio)
    return worst


@pytest.mark.parametrize("name", ["c1", "hemisphere", "c2"])
def test_merged_geometry_and_tables(name):
    w, nodes, gc, of, oc = _case(name)
    c = _coarse_ctx(gc, nodes, name)
    for inst in range(4):
        assert np.array_equal(c.export(inst, ebs.Q["TYPE"]), oc.export_type(inst)), inst
    bad = {}
    for inst in range(4):
        for q in range(20):
            a, b = c.export(inst, q), oc.export(inst, q)
            if q in _WEIGHT:
                a = a * c.export(inst, _WEIGHT[q])
                b = b * oc.export(inst, _WEIGHT[q])
            e = float(np.abs(a - b).max())
            if e > 1e-13:
                bad[(inst, q)] = e
    assert not bad, bad
    OW = oracle.OW
    for inst in range(4):
        fl = oc.export(inst, oracle.OQ["ALPHA"]) > 0
        for q in ("SMALL", "TIER", "MASK", "NCOUNT"):
            assert np.array_equal(c.export(inst, ebs.Q[q])[fl], oc.export_w(inst, OW[q])[fl]), (inst, q)
        for qe, qo in [("KAPPA", "KAPPA"), ("OMEGA", "OMEGA"), ("VHAT", "VHAT"),
                       ("XHAT_X", "XHX"), ("XHAT_Y", "XHY"), ("XHAT_Z", "XHZ")]:
            e = np.abs(c.export(inst, ebs.Q[qe]) - oc.export_w(inst, OW[qo]))[fl].max()
            assert e <= 1e-12, (inst, qe, e)
    # the fractions the restriction uses (fine context) are the merged ones
    cf = _fine_ctx(w, nodes)
    a, b = cf.coarsened_geometry()
    assert np.abs(c.export(0, ebs.Q["ALPHA"]) - a).max() <= 1e-15
    for d, q in enumerate(("BETA_X", "BETA_Y", "BETA_Z")):
        got = c.export(0, ebs.Q[q])
        assert np.abs(got[:, :, :] - b[d]).max() <= 1e-15, q


@pytest.mark.parametrize("name", ["c1", "hemisphere"])
def test_two_level_stages(name):
    """Three stages of the two-level sequence: fine stage, coarse stage from
    the coarse state, restriction of the fine result onto the coarse level;
    the coarse stage result and the restricted state against the oracle,
    and the coarse mass and rho theta equal to the fine ones."""
    w, nodes, gc, of, oc = _case(name)
    cf = _fine_ctx(w, nodes)
    cc = _coarse_ctx(gc, nodes, name)
    Uf0 = synth.make_state(w)
    Uc0 = of.restrict(Uf0)
    dt_f = w.dt
    Fn, Cn = cf.new_state(Uf0), cc.new_state(Uc0)
    Fs, Cs = cf.new_state(Uf0), cc.new_state(Uc0)
    Fh, Ch = cf.new_state(), cc.new_state()
    of_n, oc_n = dict(Uf0), dict(Uc0)
    of_s, oc_s = dict(Uf0), dict(Uc0)
    worst = 0.0
    for s, cs in enumerate((1.0 / 3.0, 0.5, 1.0)):
        # fine stage
        cf.advance(Fn, Fs, Fh, cs * dt_f)
        cf.redistribute(Fh, Fs)
        # coarse stage (the same time step on both levels)
        cc.advance(Cn, Cs, Ch, cs * dt_f)
        cc.redistribute(Ch, Ch)
        torch.cuda.synchronize()
        want_f = of.stage(of_n, of_s, cs * dt_f)
        want_c = oc.stage(oc_n, oc_s, cs * dt_f)
        worst = max(worst, _check_state(_host(Ch), want_c, oc, Uc0, cs * dt_f, min(gc.dx), f"coarse stage {s}"))
        # the restriction overwrites the coarse state
        cf.restrict(Fs, Cs)
        torch.cuda.synchronize()
        of_s = want_f
        oc_s = of.restrict(want_f)
        worst = max(worst, _check_state(_host(Fs), want_f, of, Uf0, cs * dt_f, min(w.grid.dx), f"fine {s}"))
        worst = max(worst, _check_state(_host(Cs), oc_s, oc, Uc0, cs * dt_f, min(gc.dx), f"restricted {s}"))
        hf, lf = cf.conserved_sums(Fs)
        hc, lc = cc.conserved_sums(Cs)
        for f in range(2):
            ref = hf[f] + lf[f]
            assert abs(hc[f] + lc[f] - ref) <= 1e-13 * abs(ref), (s, f)
    print("worst fraction of the sliver bound", worst)
