"""Error paths and contracts of the C ABI that need a device: overlap rules
of ebs_advance_stage / ebs_redistribute / ebs_rk3_step, the rule that
ebs_redistribute takes the output of the last advance, and a geometry
rebuild on a context that already holds geometry and a captured graph."""
import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2604_11959_amd as ebs  # noqa: E402

FIELDS = ebs.FIELDS


def _ctx(w):
    print(f"[ctx] {w.name}", flush=True)
    c = ebs.Context(w.grid.n, w.grid.dx, w.grid.lo)
    c.build_geometry(w.h_nodes)
    return c


def _raw_advance(c, Un, Ucur, Uhat):
    a, b, d = ebs.State(*Un), ebs.State(*Ucur), ebs.State(*Uhat)
    return c.lib.ebs_advance_stage(c.h, C.byref(a), C.byref(b), C.byref(d), 1e-3)


def _ptrs(U):
    return [U[f].data_ptr() for f in FIELDS]


def test_advance_rejects_every_overlap_with_the_stencil_input():
    w = synth.make_workload(1)
    c = _ctx(w)
    U = c.new_state(synth.make_state(w))
    V = c.new_state()
    ok = _raw_advance(c, _ptrs(U), _ptrs(U), _ptrs(V))
    assert ok == ebs.EBS_OK
    for f in range(5):  # each output array equal to the same input array
        out = _ptrs(V)
        out[f] = _ptrs(U)[f]
        assert _raw_advance(c, _ptrs(U), _ptrs(U), out) == ebs.EBS_E_ARG, FIELDS[f]
    # rhotheta output aliasing rho input (cross-field)
    out = _ptrs(V)
    out[1] = _ptrs(U)[0]
    assert _raw_advance(c, _ptrs(U), _ptrs(U), out) == ebs.EBS_E_ARG
    # rhov output starting one element into the rhov input
    out = _ptrs(V)
    out[3] = _ptrs(U)[3] + 8
    assert _raw_advance(c, _ptrs(U), _ptrs(U), out) == ebs.EBS_E_ARG
    # two output arrays overlapping each other
    out = _ptrs(V)
    out[4] = out[0]
    assert _raw_advance(c, _ptrs(U), _ptrs(U), out) == ebs.EBS_E_ARG
    # U^n separate from U_cur: output may equal U^n field by field, but not
    # overlap it partly
    W = c.new_state(synth.make_state(w))
    assert _raw_advance(c, _ptrs(W), _ptrs(U), _ptrs(W)) == ebs.EBS_OK
    out = _ptrs(W)
    out[2] = _ptrs(W)[2] + 8
    assert _raw_advance(c, _ptrs(W), _ptrs(U), out) == ebs.EBS_E_ARG
    assert b"overlap" in c.lib.ebs_last_error(c.h)
    torch.cuda.synchronize()
    c.close()


def test_redistribute_needs_the_last_advance_output():
    w = synth.make_workload(1)
    c = _ctx(w)
    U = c.new_state(synth.make_state(w))
    A, B = c.new_state(), c.new_state()
    with pytest.raises(ebs.EbsError) as e:  # no advance since the build
        c.redistribute(A, A)
    assert e.value.status == ebs.EBS_E_ORDER
    c.advance(U, U, A, w.dt / 3)
    with pytest.raises(ebs.EbsError) as e:  # another state
        c.redistribute(B, B)
    assert e.value.status == ebs.EBS_E_ORDER
    c.redistribute(A, B)  # the advance's output, separate result: fine
    c.redistribute(A, A)
    S = [c.new_state(), c.new_state()]
    c.rk3_step(U, S, w.dt)
    with pytest.raises(ebs.EbsError) as e:  # the step overwrote the copy
        c.redistribute(A, A)
    assert e.value.status == ebs.EBS_E_ORDER
    with pytest.raises(ebs.EbsError) as e:  # scratch overlapping U
        c.rk3_step(U, [U, S[1]], w.dt)
    assert e.value.status == ebs.EBS_E_ARG
    torch.cuda.synchronize()
    c.close()


def test_geometry_rebuild_drops_graph_and_matches_fresh_context():
    """Build on the hill, capture and replay an RK3 graph, rebuild on another
    terrain with the same state pointers: the next graph step must use the
    new tables (equal to a fresh context on the new terrain, bit for bit).  A
    rebuild rejected by argument checks keeps the previous geometry."""
    w = synth.make_workload(1)
    g = w.grid
    U0 = synth.make_state(w)
    h2 = synth.terrain_plane(g, 0.21, 0.0, 0.0) + 0.05 * np.cos(
        2 * np.pi * synth.node_coords(g)[0][None, :] / g.length[0])
    h2 = synth._periodic_fix(h2)
    c = _ctx(w)
    U = c.new_state(U0)
    S = [c.new_state(), c.new_state()]
    c.rk3_step(U, S, w.dt, use_graph=True)
    c.rk3_step(U, S, w.dt, use_graph=True)
    bad = w.h_nodes.copy()
    bad[2, 2] = np.inf
    with pytest.raises(ebs.EbsError) as e:
        c.build_geometry(bad)
    assert e.value.status == ebs.EBS_E_ARG
    c.rk3_step(U, S, w.dt, use_graph=True)  # previous geometry still in place
    c.build_geometry(h2)
    U1 = synth.state_uniform(g, rho=1.0, theta=300.0, u=10.0)
    U1["rhotheta"] = U0["rhotheta"].copy()
    for f in FIELDS:
        U[f].copy_(torch.as_tensor(U1[f]))
    c.rk3_step(U, S, w.dt, use_graph=True)
    torch.cuda.synchronize()
    f2 = ebs.Context(g.n, g.dx, g.lo)
    f2.build_geometry(h2)
    V = f2.new_state(U1)
    T = [f2.new_state(), f2.new_state()]
    f2.rk3_step(V, T, w.dt, use_graph=True)
    torch.cuda.synchronize()
    for f in FIELDS:
        assert torch.equal(U[f], V[f]), f
    c.close()
    f2.close()
