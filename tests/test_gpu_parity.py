"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on
the same seeded inputs.  Discrete decisions must match bit for bit; floating
results within the stated tolerances:
  geometry moments <= 1e-13 (absolute, normalised quantities);
  FP64 state <= 1e-12 relative per field (max |dU| over fluid entries divided
  by max |U_ref| of the field; one joint scale for the three momenta);
  FP32-bulk state <= 2e-5 relative, same norm;
  conservation (FP64) <= 1e-13 relative drift of sum V U per stage."""
import math

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
GEO_Q = list(range(20))
_cache = {}


def _oracle(cfg):
    key = ("o", cfg)
    if key not in _cache:
        w = synth.make_workload(cfg)
        _cache[key] = (w, oracle.Oracle(w.grid, w.h_nodes))
    return _cache[key]


def _ctx(w, precision=ebs.EBS_F64, boxes=None, **kw):
    print(f"[ctx] {w.name} precision={precision}", flush=True)
    c = ebs.Context(w.grid.n, w.grid.dx, w.grid.lo, boxes=boxes, precision=precision, **kw)
    c.build_geometry(w.h_nodes)
    return c


def _host(U):
    return {k: v.double().cpu().numpy() for k, v in U.items()}


def _fluid_masks(o):
    m = {}
    for f, inst in zip(FIELDS, oracle.FIELD_INST):
        a = o.export(inst, oracle.OQ["ALPHA"]) > 0
        if f == "rhow":
            a[0] = a[-1] = False
        m[f] = a
    return m


def rel_err(got: dict, ref: dict, masks: dict) -> dict:
    """Per-field relative error (max abs difference over fluid entries / scale)."""
    out = {}
    mom = max(np.abs(ref[f][masks[f]]).max() if masks[f].any() else 0.0
              for f in ("rhou", "rhov", "rhow"))
    for f in FIELDS:
        S = np.abs(ref[f][masks[f]]).max() if f in ("rho", "rhotheta") else mom
        S = S if S > 0 else 1.0
        out[f] = float(np.abs(got[f] - ref[f])[masks[f]].max() / S) if masks[f].any() else 0.0
    return out


# centroid quantities are compared as moments (weight x offset): a centroid of
# a sliver face or facet is a ratio of two tiny numbers and carries no
# information beyond its moment
_WEIGHT = {4: 1, 5: 1, 6: 2, 7: 2, 8: 3, 9: 3, 10: 0, 11: 0, 12: 0, 17: 16, 18: 16, 19: 16}


def _geo_errors(c, o):
    errs = {}
    for inst in range(4):
        for q in GEO_Q:
            got = c.export(inst, q)
            ref = o.export(inst, q)
            if q in _WEIGHT:
                got = got * c.export(inst, _WEIGHT[q])
                ref = ref * o.export(inst, _WEIGHT[q])
            errs[(inst, q)] = float(np.abs(got - ref).max())
    return errs


@pytest.mark.parametrize("cfg", [1, 2])
def test_geometry_parity(cfg):
    """Four instances: classification bitwise, moments <= 1e-13."""
    w, o = _oracle(cfg)
    c = _ctx(w)
    for inst in range(4):
        ty = c.export(inst, ebs.Q["TYPE"])
        assert np.array_equal(ty, o.export_type(inst)), inst
    errs = _geo_errors(c, o)
    bad = {k: v for k, v in errs.items() if v > 1e-13}
    print(sorted(errs.items(), key=lambda kv: -kv[1])[:6])
    assert not bad, bad


@pytest.mark.parametrize("plane", [(0.37, 0.21, -0.13), (0.2, 1.7, 0.9), (0.5, 0.0, 0.0)])
def test_geometry_parity_planes(plane):
    """Planar terrain (made periodic by a flat border) with steep and flat parts."""
    g = synth.Grid((16, 16, 12), (0.125, 0.125, 0.125))
    x, y = synth.node_coords(g)
    X, Y = np.meshgrid(x, y)
    a, b, cc = plane
    h = a + b * np.minimum(X, 2.0 - X) * 0.5 + cc * np.minimum(Y, 2.0 - Y) * 0.5
    h = synth._periodic_fix(np.clip(h, 0.0, 1.2))
    w = synth.Workload("plane", g, h, 1e-3, 0)
    o = oracle.Oracle(g, h)
    c = _ctx(w)
    for inst in range(4):
        assert np.array_equal(c.export(inst, ebs.Q["TYPE"]), o.export_type(inst))
    bad = {k: v for k, v in _geo_errors(c, o).items() if v > 1e-13}
    assert not bad, bad


@pytest.mark.parametrize("cfg", [1, 2])
def test_wsrd_tables_parity(cfg):
    """Small flags, tiers, member masks and N bitwise; weights <= 1e-12."""
    w, o = _oracle(cfg)
    c = _ctx(w)
    OW = oracle.OW
    pairs = [("SMALL", "SMALL"), ("TIER", "TIER"), ("MASK", "MASK"), ("NCOUNT", "NCOUNT")]
    for inst in range(4):
        fl = o.export(inst, oracle.OQ["ALPHA"]) > 0
        for qe, qo in pairs:
            got = c.export(inst, ebs.Q[qe])
            ref = o.export_w(inst, OW[qo])
            assert np.array_equal(got[fl], ref[fl]), (inst, qe)
        for qe, qo in [("KAPPA", "KAPPA"), ("OMEGA", "OMEGA"), ("VHAT", "VHAT"),
                       ("XHAT_X", "XHX"), ("XHAT_Y", "XHY"), ("XHAT_Z", "XHZ")]:
            got = c.export(inst, ebs.Q[qe])
            ref = o.export_w(inst, OW[qo])
            assert np.abs(got - ref)[fl].max() <= 1e-12, (inst, qe)


@pytest.mark.parametrize("cfg", [1, 2])
def test_single_stage_parity_fp64(cfg):
    """One stage (advance + redistribute) from the same input, FP64."""
    w, o = _oracle(cfg)
    c = _ctx(w)
    U0 = synth.make_state(w)
    cdt = w.dt / 3
    ref = o.stage(U0, U0, cdt)
    Ud = c.new_state(U0)
    Uh = c.new_state()
    c.advance(Ud, Ud, Uh, cdt)
    c.redistribute(Uh, Uh)
    torch.cuda.synchronize()
    err = rel_err(_host(Uh), ref, _fluid_masks(o))
    print(err)
    assert max(err.values()) <= 1e-12, err
    # every entry written: walls and covered entries zero, periodic repeats equal
    h = _host(Uh)
    assert np.all(h["rhow"][0] == 0) and np.all(h["rhow"][-1] == 0)
    assert np.array_equal(h["rhou"][:, :, -1], h["rhou"][:, :, 0])
    assert np.array_equal(h["rhov"][:, -1, :], h["rhov"][:, 0, :])
    m = _fluid_masks(o)
    for f in FIELDS:
        assert np.all(h[f][~m[f]] == 0.0), f


def test_stage_parity_random_state_fp64():
    """A random state on the hill stresses every stencil branch (signs of the
    mass flux, order reduction, cut-face interpolation, all limiter paths)."""
    w, o = _oracle(1)
    c = _ctx(w)
    U0 = synth.state_random(w.grid, 21, amp=2.0)
    Un = synth.state_random(w.grid, 22, amp=2.0)
    cdt = 0.2 * w.dt
    uh_ref = o.advance(Un, U0, cdt)
    ref = o.redistribute(uh_ref)
    Ud, Ucur, Uh = c.new_state(Un), c.new_state(U0), c.new_state()
    c.advance(Ud, Ucur, Uh, cdt)
    torch.cuda.synchronize()
    # provisional state in extensive form (alpha * U-hat), not amplified by 1/alpha
    h = _host(Uh)
    for f, inst in zip(FIELDS, oracle.FIELD_INST):
        a = o.export(inst, oracle.OQ["ALPHA"])
        e = np.abs(a * (h[f] - uh_ref[f])).max() / max(np.abs(a * uh_ref[f]).max(), 1e-300)
        assert e <= 1e-12, (f, e)
    c.redistribute(Uh, Uh)
    torch.cuda.synchronize()
    err = rel_err(_host(Uh), ref, _fluid_masks(o))
    assert max(err.values()) <= 1e-12, err


@pytest.mark.parametrize("cfg", [1, 2])
def test_general_range_rules(cfg):
    """Each rule for the top of the general range (0 loose, 1 small-CV
    footprint, 2 the cells the redistribution touches) gives the oracle's
    stage within the FP64 bar; a stricter rule never keeps more general cells."""
    w, o = _oracle(cfg)
    U0 = synth.state_random(w.grid, 31, amp=1.0) if cfg == 1 else synth.make_state(w)
    cdt = w.dt / 3
    ref = o.stage(U0, U0, cdt)
    m = _fluid_masks(o)
    general = []
    for rule in (0, 1, 2):
        print(f"[range rule] cfg={cfg} rule={rule}", flush=True)
        c = ebs.Context(w.grid.n, w.grid.dx, w.grid.lo, precision=ebs.EBS_F64)
        c.set_range_rule(rule)
        c.build_geometry(w.h_nodes)
        general.append(int(c.stats()[0][6]))
        Ud, Uh = c.new_state(U0), c.new_state()
        c.advance(Ud, Ud, Uh, cdt)
        c.redistribute(Uh, Uh)
        torch.cuda.synchronize()
        err = rel_err(_host(Uh), ref, m)
        assert max(err.values()) <= 1e-12, (rule, err)
    print("general cells per rule", general)
    assert general[0] >= general[1] >= general[2] > 0, general
    with pytest.raises(ebs.EbsError):
        c.set_range_rule(3)


def _hills_with_flat_ground(nz=40):
    """Two small truncated hills: most columns are flat ground (h = 0), whose
    whole neighbourhood is regular down to the bottom wall."""
    g = synth.Grid((48, 40, nz), (78.125, 78.125, 31.25))
    h = synth.terrain_gaussian_hills(g, 5, 2, hrange=(80.0, 200.0), wrange=(150.0, 250.0))
    return synth.Workload("hills_flat48", g, h, synth.cfl_dt(g), 5, [((0, 0, 0), g.n)], "atmos")


@pytest.mark.parametrize("terrain", ["hills", "flat"])
@pytest.mark.parametrize("precision,tiles,tol", [
    (ebs.EBS_F64, ((16, 4, 16), (16, 8, 64)), 1e-12),
    (ebs.EBS_F32_BULK, ((16, 16, 16), (32, 8, 32), (32, 16, 16), (32, 8, 64, 1), (64, 16, 64, 1)), 2e-5),
])
def test_bottom_wall_and_flat_ground(terrain, precision, tiles, tol):
    """Columns with no cut CV nearby have an empty general range: the
    regular-region kernel updates them down to the bottom wall (zero flux
    through k = 0, order reduction of the z stencils next to it, no z-face CV
    at k = 0).  A random state makes every z flux live; one stage against the
    oracle, for several tile shapes (tiles starting at the bottom and above)."""
    w = _hills_with_flat_ground()
    if terrain == "flat":
        w = synth.Workload("flat48", w.grid, synth.terrain_flat(w.grid, 0.0), w.dt, 5,
                           [((0, 0, 0), w.grid.n)], "atmos")
    # the scenario: many columns whose 7 x 7 neighbourhood is flat ground
    hn = w.h_nodes
    hc = np.maximum(np.maximum(hn[:-1, :-1], hn[1:, :-1]), np.maximum(hn[:-1, 1:], hn[1:, 1:])) > 0
    win = np.zeros_like(hc)
    for dj in range(-3, 4):
        for di in range(-3, 4):
            win |= np.roll(np.roll(hc, dj, 0), di, 1)
    assert (~win).mean() > (0.3 if terrain == "hills" else 0.99)
    o = oracle.Oracle(w.grid, w.h_nodes)
    U0 = synth.state_random(w.grid, 31, amp=2.0)
    Un = synth.state_random(w.grid, 32, amp=2.0)
    cdt = 0.3 * w.dt
    ref = o.redistribute(o.advance(Un, U0, cdt))
    masks = _fluid_masks(o)
    boxes = synth.boxes_split(w.grid.n, 9, 12, block=16, unit=8)
    for tile in tiles:
        c = _ctx(w, precision=precision, boxes=boxes)
        c.set_tile(*tile)
        general = int(c.stats()[0][6])
        if terrain == "flat":
            assert general == 0, general
        Ud, Ucur, Uh = c.new_state(Un), c.new_state(U0), c.new_state()
        c.advance(Ud, Ucur, Uh, cdt)
        c.redistribute(Uh, Uh)
        torch.cuda.synchronize()
        h = _host(Uh)
        err = rel_err(h, ref, masks)
        print(terrain, precision, tile, err, flush=True)
        assert max(err.values()) <= tol, (tile, err)
        assert np.all(h["rhow"][0] == 0) and np.all(h["rhow"][-1] == 0)
        for f in FIELDS:
            assert np.all(h[f][~masks[f]] == 0.0), f



def _window_state(U, i0, j0, wx, wy):
    """The state of a window of columns, with the window's periodic face copies."""
    W = {
        "rho": U["rho"][:, j0:j0 + wy, i0:i0 + wx].copy(),
        "rhotheta": U["rhotheta"][:, j0:j0 + wy, i0:i0 + wx].copy(),
        "rhou": U["rhou"][:, j0:j0 + wy, i0:i0 + wx + 1].copy(),
        "rhov": U["rhov"][:, j0:j0 + wy + 1, i0:i0 + wx].copy(),
        "rhow": U["rhow"][:, j0:j0 + wy, i0:i0 + wx].copy(),
    }
    W["rhou"][:, :, -1] = W["rhou"][:, :, 0]
    W["rhov"][:, -1, :] = W["rhov"][:, 0, :]
    return W


def test_full_size_benchmark_configuration_sampled_windows():
    """The benchmark configuration at full size (512 x 512 x 128, 512 boxes,
    FP32 bulk, the tile the benchmark uses, RK3 step captured in a HIP graph)
    against the FP64 oracle on sampled windows.  One RK3 step reaches a few
    cells per stage (flux stencil and redistribution radius), so the oracle run
    on a 64 x 64-column window cut from the same terrain and state reproduces
    the interior of the window (24-column margin) exactly."""
    import json
    import os

    w = synth.make_workload(4)
    n = w.grid.n
    cache = os.path.join(os.path.dirname(ebs.__file__), "tiles_mi355x.json")
    key = f"f32bulk_{n[0]}x{n[1]}x{n[2]}_b{len(w.boxes)}"
    tile = json.load(open(cache))[key]
    c = _ctx(w, precision=ebs.EBS_F32_BULK, boxes=w.boxes)
    c.set_tile(*tile)
    U0 = synth.make_state(w)
    U = c.new_state(U0)
    S = [c.new_state(), c.new_state()]
    c.rk3_step(U, S, w.dt, use_graph=True)
    torch.cuda.synchronize()
    got = _host(U)
    del U, S
    # reference: one oracle RK3 step on each window
    wx = wy = 64
    m = 24
    hn = w.h_nodes
    centres = []
    hc = hn[:-1, :-1]
    for _ in range(2):  # the two highest hills, then a flat area
        jj, ii = np.unravel_index(np.argmax(hc), hc.shape)
        centres.append((ii, jj))
        hc = hc.copy()
        hc[max(jj - 64, 0):jj + 64, max(ii - 64, 0):ii + 64] = -1.0
    flat = np.argwhere(hn[:-1, :-1] == 0.0)
    centres.append((int(flat[len(flat) // 2][1]), int(flat[len(flat) // 2][0])))
    for (ci, cj) in centres:
        i0 = int(min(max(ci - wx // 2, 0), n[0] - wx - 1))
        j0 = int(min(max(cj - wy // 2, 0), n[1] - wy - 1))
        ww = synth.window(w, i0, j0, wx, wy, n[2])
        o = oracle.Oracle(ww.grid, ww.h_nodes)
        ref = o.rk3_step(_window_state(U0, i0, j0, wx, wy), w.dt)
        gw = _window_state(got, i0, j0, wx, wy)
        masks = _fluid_masks(o)
        for f in FIELDS:
            inner = np.zeros_like(masks[f])
            inner[:, m:-m, m:-m] = True
            masks[f] = masks[f] & inner
        err = rel_err(gw, ref, masks)
        print((i0, j0), err, flush=True)
        assert max(err.values()) <= 2e-5, ((i0, j0), err)



def test_ridges_1024x1024x192_sampled_windows():
    """The ridge workload at full size (1024 x 1024 x 192, 3072 boxes, steep
    hipped-roof ridges, FP32 bulk, domain tiles 64 x 16 x 64) against the FP64
    oracle on windows around the steepest ridges and on flat ground."""
    w = synth.make_workload(5)
    n = w.grid.n
    c = _ctx(w, precision=ebs.EBS_F32_BULK, boxes=w.boxes)
    c.set_tile(64, 16, 64, 1)
    U0 = synth.make_state(w)
    U = c.new_state(U0)
    S = [c.new_state(), c.new_state()]
    c.rk3_step(U, S, w.dt, use_graph=True)
    torch.cuda.synchronize()
    got = _host(U)
    del U, S
    wx = wy = 56
    m = 22
    hn = w.h_nodes
    # steepest node-to-node slope, the highest point, flat ground
    slope = np.abs(np.diff(hn, axis=1))[:-1, :] + np.abs(np.diff(hn, axis=0))[:, :-1]
    jj, ii = np.unravel_index(np.argmax(slope), slope.shape)
    centres = [(ii, jj)]
    jj, ii = np.unravel_index(np.argmax(hn[:-1, :-1]), (n[1], n[0]))
    centres.append((ii, jj))
    flat = np.argwhere(hn[:-1, :-1] == 0.0)
    centres.append((int(flat[len(flat) // 3][1]), int(flat[len(flat) // 3][0])))
    for (ci, cj) in centres:
        i0 = int(min(max(ci - wx // 2, 0), n[0] - wx - 1))
        j0 = int(min(max(cj - wy // 2, 0), n[1] - wy - 1))
        ww = synth.window(w, i0, j0, wx, wy, n[2])
        o = oracle.Oracle(ww.grid, ww.h_nodes)
        ref = o.rk3_step(_window_state(U0, i0, j0, wx, wy), w.dt)
        gw = _window_state(got, i0, j0, wx, wy)
        masks = _fluid_masks(o)
        for f in FIELDS:
            inner = np.zeros_like(masks[f])
            inner[:, m:-m, m:-m] = True
            masks[f] = masks[f] & inner
        err = rel_err(gw, ref, masks)
        print((i0, j0), err, flush=True)
        assert max(err.values()) <= 2e-5, ((i0, j0), err)

def test_terrain_on_a_grid_plane_stage_and_rk3():
    """Flat terrain exactly on the plane z = 2 dz (faces on the terrain carry no
    fluid; the first fluid layer is regular), plus the fully flat domain at
    z = 0 through the RK3 driver and its graph; FP64 against the oracle."""
    g = synth.Grid((24, 16, 12), (78.125, 78.125, 31.25))
    for h0 in (2 * 31.25, 0.0):
        w = synth.Workload("flat_on_plane", g, synth.terrain_flat(g, h0), synth.cfl_dt(g), 3,
                           [((0, 0, 0), g.n)], "atmos")
        o = oracle.Oracle(g, w.h_nodes)
        c = _ctx(w)
        U0 = synth.state_random(g, 41, amp=1.5)
        for inst in range(4):
            assert np.array_equal(c.export(inst, ebs.Q["TYPE"]), o.export_type(inst)), inst
        ref = o.rk3_step(U0, w.dt)
        for use_graph in (False, True, True):
            U = c.new_state(U0)
            S = [c.new_state(), c.new_state()]
            c.rk3_step(U, S, w.dt, use_graph=use_graph)
            torch.cuda.synchronize()
            err = rel_err(_host(U), ref, _fluid_masks(o))
            print(h0, use_graph, err, flush=True)
            assert max(err.values()) <= 1e-12, (h0, use_graph, err)

def test_trajectory_parity_c1_ten_stages():
    """Ten consecutive RK3 stages (three steps and the first stage of the
    fourth) on the hill, FP64, compared after every stage; conservation."""
    w, o = _oracle(1)
    c = _ctx(w)
    U0 = synth.make_state(w)
    dn = oracle.to_dense(U0, o.n)
    cur = dn
    Un_d = c.new_state(U0)
    bufs = [c.new_state(), c.new_state()]
    cur_d = Un_d
    masks = _fluid_masks(o)
    s_ref0 = o.conserved_sums(U0)
    for s in range(10):
        cs = oracle.RK3_C[s % 3]
        if s % 3 == 0 and s > 0:
            dn = cur
            Un_d = {k: v.clone() for k, v in cur_d.items()}
        cur = o.redistribute_dense(o.advance_dense(dn, cur, cs * w.dt))
        out = bufs[s % 2]
        c.advance(Un_d, cur_d, out, cs * w.dt)
        c.redistribute(out, out)
        cur_d = out
        torch.cuda.synchronize()
        err = rel_err(_host(cur_d), oracle.from_dense(cur, o.n), masks)
        print(s, err, flush=True)
        assert max(err.values()) <= 1e-12, (s, err)
        hi, lo = c.conserved_sums(cur_d)
        for f in range(5):
            ref = s_ref0[f]
            tot = hi[f] + lo[f]
            scale = abs(ref) if ref != 0 else 1.0
            assert abs(tot - ref) <= 1e-13 * scale + 1e-300, (s, f, tot, ref)


def test_rk3_step_matches_stages_and_graph():
    """ebs_rk3_step equals three explicit stages bit for bit; the captured graph
    replays give the same bits (replayed several times with eager work and
    synchronisation between replays)."""
    w, o = _oracle(1)
    c = _ctx(w)
    U0 = synth.make_state(w)
    A = c.new_state(U0)
    S = [c.new_state(), c.new_state()]
    c.rk3_step(A, S, w.dt, use_graph=False)
    # manual stages
    Un = c.new_state(U0)
    b0, b1, b2 = c.new_state(), c.new_state(), c.new_state()
    c.advance(Un, Un, b0, w.dt / 3); c.redistribute(b0, b0)
    c.advance(Un, b0, b1, w.dt / 2); c.redistribute(b1, b1)
    c.advance(Un, b1, b2, w.dt); c.redistribute(b2, b2)
    torch.cuda.synchronize()
    for f in FIELDS:
        assert torch.equal(A[f], b2[f]), f
    # graph replays
    G = c.new_state(U0)
    ref = {k: v.clone() for k, v in G.items()}
    for rep in range(3):
        for k in FIELDS:
            G[k].copy_(ref[k])
        torch.cuda.synchronize()
        c.rk3_step(G, S, w.dt, use_graph=True)
        torch.cuda.synchronize()
        junk = torch.ones(1000, device="cuda").sum()  # eager work between replays
        for f in FIELDS:
            assert torch.equal(G[f], A[f]), (rep, f)
    del junk


def test_free_stream_mode_c2():
    """With the closure test mode for the EB flux, uniform flow stays uniform on
    the C2 hill after a full RK3 step (all four instances)."""
    w = synth.make_workload(2)
    c = _ctx(w, eb_flux=ebs.EBS_EB_FREESTREAM)
    U0 = synth.state_uniform(w.grid, rho=1.2, theta=300.0, u=10.0)
    U = c.new_state(U0)
    S = [c.new_state(), c.new_state()]
    c.rk3_step(U, S, w.dt)
    torch.cuda.synchronize()
    o = _oracle(2)[1]
    h = _host(U)
    m = _fluid_masks(o)
    for f in FIELDS:
        ref = U0[f]
        scale = max(np.abs(ref).max(), 1.0)
        assert np.abs(h[f] - ref)[m[f]].max() <= 1e-12 * scale, f


@pytest.mark.parametrize("precision", [ebs.EBS_F64, ebs.EBS_F32_BULK])
def test_overlap_gives_identical_bits(precision):
    """The regular-region kernel on a second stream, concurrent with the
    general range and the redistribution, gives the same bits as the serial
    order, eagerly and through the captured graph (replayed three times)."""
    w = synth.make_workload(2)
    U0 = synth.make_state(w)
    boxes = synth.boxes_split(w.grid.n, 7, 40, block=32, unit=16)
    res = []
    for overlap, use_graph in ((False, False), (True, False), (True, True)):
        c = _ctx(w, precision=precision, boxes=boxes)
        c.set_overlap(overlap)
        U = c.new_state(U0)
        S = [c.new_state(), c.new_state()]
        for _ in range(3):
            c.rk3_step(U, S, w.dt, use_graph=use_graph)
            torch.cuda.synchronize()
        res.append(_host(U))
    for r in res[1:]:
        for f in FIELDS:
            assert np.array_equal(r[f], res[0][f]), f

@pytest.mark.parametrize("precision,tiles", [
    (ebs.EBS_F64, ((16, 4), (16, 8), (32, 8, 64, 1), (32, 16, 32, 1), (16, 8, 128, 1))),
    (ebs.EBS_F32_BULK, ((16, 4), (16, 16), (32, 8), (64, 2), (32, 8, 64, 1), (64, 4, 16, 1),
                        (64, 16, 64, 1), (64, 8, 32, 1), (32, 16, 16, 0), (64, 16, 128, 1),
                        (32, 8, 256, 0))),
])
def test_box_list_and_tiles_do_not_change_results(precision, tiles):
    """Uneven AMR-style boxes and different tile shapes give identical bits."""
    w = synth.make_workload(2)
    U0 = synth.make_state(w)
    boxes = synth.boxes_split(w.grid.n, 7, 40, block=32, unit=16)
    res = []
    for bx, tile in [(None, tiles[0])] + [(boxes, t) for t in tiles]:
        c = _ctx(w, precision=precision, boxes=bx)
        c.set_tile(*tile)
        U = c.new_state(U0)
        S = [c.new_state(), c.new_state()]
        c.rk3_step(U, S, w.dt)
        torch.cuda.synchronize()
        res.append(_host(U))
    for r in res[1:]:
        for f in FIELDS:
            assert np.array_equal(r[f], res[0][f]), f


def test_f32_bulk_parity_c2_ten_stages():
    """FP32-bulk state and regular-region arithmetic against the FP64 oracle
    over ten stages: per-field error <= 2e-5."""
    w, o = _oracle(2)
    c = _ctx(w, precision=ebs.EBS_F32_BULK)
    U0 = synth.make_state(w)
    U = c.new_state(U0)
    S = [c.new_state(), c.new_state()]
    ref = U0
    for step in range(3):
        c.rk3_step(U, S, w.dt)
        ref = o.rk3_step(ref, w.dt)
    torch.cuda.synchronize()
    err = rel_err(_host(U), ref, _fluid_masks(o))
    print(err)
    assert max(err.values()) <= 2e-5, err


def test_conservation_c2_fp64_many_stages():
    """sum V U of every field drifts by <= 1e-13 relative per stage over 30
    stages of the C2 case (double-double sums)."""
    w = synth.make_workload(2)
    c = _ctx(w)
    U = c.new_state(synth.make_state(w))
    S = [c.new_state(), c.new_state()]
    hi0, lo0 = c.conserved_sums(U)
    for step in range(10):
        c.rk3_step(U, S, w.dt, use_graph=True)
    hi, lo = c.conserved_sums(U)
    for f in range(5):
        ref = hi0[f] + lo0[f]
        if ref == 0.0:
            continue
        assert abs((hi[f] + lo[f]) - ref) / abs(ref) <= 30 * 1e-13, (f, hi[f], ref)


def test_api_errors_on_device():
    w = synth.make_workload(1)
    c = ebs.Context(w.grid.n, w.grid.dx)
    U = c.new_state(synth.make_state(w))
    V = c.new_state()
    with pytest.raises(ebs.EbsError) as e:
        c.advance(U, U, V, 1e-3)
    assert e.value.status == ebs.EBS_E_ORDER
    bad = w.h_nodes.copy()
    bad[3, 4] = np.nan
    with pytest.raises(ebs.EbsError) as e:
        c.build_geometry(bad)
    assert e.value.status == ebs.EBS_E_ARG
    tall = w.h_nodes.copy() * 10.0
    with pytest.raises(ebs.EbsError) as e:
        c.build_geometry(tall)
    assert e.value.status == ebs.EBS_E_ARG
    c.build_geometry(w.h_nodes)
    with pytest.raises(ebs.EbsError) as e:
        c.advance(U, U, U, 1e-3)  # output aliases the stencil input
    assert e.value.status == ebs.EBS_E_ARG
    with pytest.raises(ebs.EbsError):
        c.set_tile(48, 4)


def test_stage_parity_rough_vertical_momentum_c2():
    """A state with cell-scale random vertical momentum on the Agnesi hill.
    Away from slivers the FP64 bar holds; at a sliver CV the provisional value
    is the flux bracket divided by alpha (Eq. update-fc), so the rounding of
    the bracket -- summed in different orders by the two implementations -- is
    amplified by 1/alpha, and the redistributed value of the sliver keeps part
    of it.  Per CV the bound is 1e-12 of the field scale plus
    eps * 6 F_max * c dt / (alpha * min(dx)), with F_max the largest
    advective flux of the field (mass flux times advected quantity); the
    largest difference measured is about a tenth of it."""
    w, o = _oracle(2)
    ref_state = synth.reference_isentropic(w.grid)
    U0 = synth.state_reference(w.grid, ref_state, 42)
    cdt = w.dt / 3
    ref = o.stage(U0, U0, cdt)
    c = _ctx(w)
    Ud, Uh = c.new_state(U0), c.new_state()
    c.advance(Ud, Ud, Uh, cdt)
    c.redistribute(Uh, Uh)
    torch.cuda.synchronize()
    got = _host(Uh)
    masks = _fluid_masks(o)
    eps = np.finfo(np.float64).eps
    mmax = max(np.abs(U0[f]).max() for f in ("rhou", "rhov", "rhow"))
    vmax = mmax / U0["rho"].min()
    phi = {"rho": 1.0, "rhotheta": np.abs(U0["rhotheta"] / U0["rho"]).max(), "rhou": vmax, "rhov": vmax,
           "rhow": vmax}
    mom = max(np.abs(ref[f][masks[f]]).max() for f in ("rhou", "rhov", "rhow"))
    worst = 0.0
    for f, inst in zip(FIELDS, oracle.FIELD_INST):
        a = o.export(inst, oracle.OQ["ALPHA"])
        scale = np.abs(ref[f][masks[f]]).max() if f in ("rho", "rhotheta") else mom
        bound = 1e-12 * scale + eps * 6 * mmax * phi[f] * cdt / (np.where(a > 0, a, 1.0) * min(w.grid.dx))
        d = np.abs(got[f] - ref[f])
        ratio = (d / bound)[masks[f]]
        worst = max(worst, ratio.max())
        assert ratio.max() <= 1.0, (f, ratio.max())
        # the plain bar holds on every CV that is not a sliver
        big = masks[f] & (a > 1e-3)
        assert d[big].max() <= 1e-12 * scale, (f, d[big].max() / scale)
    print("worst fraction of the bound", worst)


@pytest.mark.parametrize("precision,tile", [(ebs.EBS_F64, (16, 8, 32, 0)), (ebs.EBS_F32_BULK, (64, 16, 64, 0)),
                                            (ebs.EBS_F32_BULK, (32, 8, 16, 0)), (ebs.EBS_F32_BULK, (32, 16, 16, 0))])
def test_persistent_schedule_gives_identical_bits(precision, tile):
    """Per-box tiles (many more tiles than resident blocks) run by a grid of
    resident blocks walking the tile list give the same bits as one block
    per tile, eagerly and through the captured graph."""
    w = synth.make_workload(2)
    U0 = synth.make_state(w)
    boxes = synth.boxes_split(w.grid.n, 7, 40, block=32, unit=16)
    res = []
    for persistent, use_graph in ((False, False), (True, False), (True, True)):
        c = _ctx(w, precision=precision, boxes=boxes)
        c.set_tile(*tile)
        c.set_persistent(persistent)
        U = c.new_state(U0)
        S = [c.new_state(), c.new_state()]
        for _ in range(2):
            c.rk3_step(U, S, w.dt, use_graph=use_graph)
        torch.cuda.synchronize()
        res.append(_host(U))
    for r in res[1:]:
        for f in FIELDS:
            assert np.array_equal(r[f], res[0][f]), f
