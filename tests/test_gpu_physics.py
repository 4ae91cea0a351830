"""GPU parity with every physics term on at once: the momentum sources
(perturbation pressure gradient, buoyancy), the thermal diffusion of rho
theta with an isothermal EB and the momentum diffusion with a no-slip EB
(Sections 2.1, 4.1, 4.2), through the three stage forms of the RK3 step of
Algorithm 1, against the FP64 oracle.

FP64: each stage starts from the oracle's state of the previous stage, so the
three forms (U^n = U_cur in the first stage, distinct states in the others)
are checked at the single-stage bars: the provisional state in extensive
form within 1e-12 of the field plus 1e7 eps times the CV's diffusive update
(the least-squares fits are accepted down to a reciprocal condition number
of 1e-7, and the two implementations solve them by different routes); after
the redistribution 1e-12 of the field plus the largest provisional bar and
the flux-bracket rounding amplified by 1/alpha.  FP32 bulk through the graph,
one whole RK3 step from FP32-representable inputs: 2e-5 plus the bound that
FP32 storage of rho theta puts on the pressure gradient (as in the sources
tests)."""
from dataclasses import dataclass

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
RK = (1.0 / 3.0, 0.5, 1.0)


@dataclass
class Diff:
    alpha_theta: float
    eb_mode: int = 1
    theta_wall: float = 299.0


@dataclass
class Visc:
    mu: float
    eb_mode: int = 1


def _setup():
    w = synth.make_workload(2)
    o = oracle.Oracle(w.grid, w.h_nodes)
    ref = synth.reference_isentropic(w.grid)
    h2 = min(w.grid.dx) ** 2
    # diffusion and viscous numbers 0.1 and 0.05 per step
    return w, o, ref, Diff(alpha_theta=0.1 * h2 / w.dt), Visc(mu=0.05 * float(ref.rho0.min()) * h2 / w.dt)


def _ctx(w, ref, d, v, precision=ebs.EBS_F64):
    print(f"[ctx] {w.name} precision={precision} sources, diffusion {d}, viscosity {v}", flush=True)
    c = ebs.Context(w.grid.n, w.grid.dx, w.grid.lo, precision=precision)
    c.build_geometry(w.h_nodes)
    c.set_sources(ref)
    c.set_diffusion(d)
    c.set_viscosity(v)
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


def test_all_physics_rk3_stages_fp64():
    w, o, ref, d, v = _setup()
    U0 = synth.state_reference(w.grid, ref, 71, theta_amp=2.0)
    c = _ctx(w, ref, d, v)
    ext = {f: o.export(inst, oracle.OQ["ALPHA"]) for f, inst in zip(FIELDS, oracle.FIELD_INST)}
    masks = _masks(o)
    eps = np.finfo(np.float64).eps
    Un = U0
    cur = U0
    worst = 0.0
    for s, cs in enumerate(RK):
        cdt = cs * w.dt
        uh = o.advance(Un, cur, cdt, ref, d, v)
        nofit = o.advance(Un, cur, cdt, ref)
        want = o.redistribute(uh)
        Gn, Gc, Gh = c.new_state(Un), c.new_state(cur), c.new_state()
        c.advance(Gn, Gc if s > 0 else Gn, Gh, cdt)
        torch.cuda.synchronize()
        h = _host(Gh)
        mscale = max(np.abs(ext[f] * uh[f]).max() for f in ("rhou", "rhov", "rhow"))
        bar = {}
        for f in FIELDS:
            fit = 1e7 * eps * np.abs(ext[f] * (uh[f] - nofit[f]))
            b = 1e-12 * (np.abs(ext[f] * uh[f]).max() if f in ("rho", "rhotheta") else mscale) + fit
            ratio = (np.abs(ext[f] * (h[f] - uh[f])) / b)[masks[f]].max()
            assert ratio <= 1.0, (s, f, ratio)
            bar[f] = b[masks[f]].max()
        # the diffusion terms moved rho theta and the momenta beyond the bar
        for f in ("rhotheta", "rhou", "rhov"):
            moved = np.abs(ext[f] * (uh[f] - nofit[f]))[masks[f]].max() / bar[f]
            assert moved > 1e3, (s, f, moved)
        c.redistribute(Gh, Gh)
        torch.cuda.synchronize()
        got = _host(Gh)
        mom = max(np.abs(want[f][masks[f]]).max() for f in ("rhou", "rhov", "rhow"))
        mmax = max(np.abs(cur[f]).max() for f in ("rhou", "rhov", "rhow"))
        pos = cur["rho"] > 0  # the oracle's states hold 0 on covered cells
        vmax = mmax / cur["rho"][pos].min()
        fscale = {"rho": mmax, "rhotheta": mmax * np.abs(cur["rhotheta"][pos] / cur["rho"][pos]).max(),
                  "rhou": mmax * vmax, "rhov": mmax * vmax, "rhow": mmax * vmax}
        for f in FIELDS:
            a = ext[f]
            scale = np.abs(want[f][masks[f]]).max() if f in ("rho", "rhotheta") else mom
            dd = np.abs(got[f] - want[f])
            prov = 8.0 * bar[f] + eps * 6 * fscale[f] * cdt / min(w.grid.dx)
            bound = 1e-12 * scale + prov / np.where(a > 0, a, 1.0)
            ratio = (dd / bound)[masks[f]].max()
            worst = max(worst, ratio)
            assert ratio <= 1.0, (s, f, ratio)
        cur = want
    print("worst fraction of the sliver bound", worst)


def test_all_physics_f32_rk3_graph():
    w, o, ref, d, v = _setup()
    U0 = {k: x.astype(np.float32).astype(np.float64)
          for k, x in synth.state_reference(w.grid, ref, 72, theta_amp=2.0).items()}
    want = o.rk3_step(U0, w.dt, ref, d, v)
    c = _ctx(w, ref, d, v, precision=ebs.EBS_F32_BULK)
    U = c.new_state(U0)
    S = [c.new_state(), c.new_state()]
    c.rk3_step(U, S, w.dt, use_graph=True)
    torch.cuda.synchronize()
    got = _host(U)
    masks = _masks(o)
    mom = max(np.abs(want[f][masks[f]]).max() for f in ("rhou", "rhov", "rhow"))
    storage = sum(RK) * w.dt * 2.0 * ref.gamma * float(ref.p0.max()) * 2.0 ** -24 / min(w.grid.dx) / mom
    for f in FIELDS:
        scale = np.abs(want[f][masks[f]]).max() if f in ("rho", "rhotheta") else mom
        e = np.abs(got[f] - want[f])[masks[f]].max() / scale
        bar = 2e-5 + (storage if f in ("rhou", "rhov", "rhow") else 0.0)
        assert e <= bar, (f, e, bar)
