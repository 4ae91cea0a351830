"""Pins of the oracle's limited least-squares reconstruction in the weighted
state redistribution (Section 5.1: gradient of Q-hat over the 3x3x3 stencil,
widened to 5 where the centroids lack spread, Barth-Jespersen-style
limiting, Eqs. qrecon and final_update_omega).  CPU only.

- A hand-derived case (tests/golden/wsrd_limiter_080.json) where the limiter
  is partly active, with and without the limiter.
- On random states: the limited gradient is the unlimited one scaled by a
  factor in [0, 1] (per component, or one factor with the scalar variant);
  the reconstruction at the centroids of the members of the neighbourhood
  stays inside [min, max] of Q-hat over the fit points and the CV; and the
  factor is the largest such one (1, or some member reaches a bound).
Each test names the mistake it exists to catch."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

OQ, OW = oracle.OQ, oracle.OW
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fr(s):
    return float(Fraction(s))


def _layer_state(g, values):
    U = synth.state_uniform(g, rho=1.0, theta=1.0, u=0.0)
    for k, v in enumerate(values):
        U["rho"][k] = v
    return U


@pytest.mark.parametrize("limiter", [0, 1, 2])
def test_hand_derived_limited_reconstruction(limiter):
    """Flat terrain at 0.8 of a unit cell, a layer-wise field: the weights,
    the neighbourhood centroid, Q-hat, the widened least-squares gradient,
    its Barth-Jespersen factor and the redistributed values equal the
    closed forms derived in the golden file.  Catches swapped min / max
    bounds, limiter evaluation at points other than the member centroids,
    and the final-update weights."""
    gd = json.load(open(os.path.join(GOLDEN, "wsrd_limiter_080.json")))
    g = synth.Grid((6, 6, 4), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, gd["terrain"]), limiter=limiter)
    W = o.w[0]
    assert np.allclose(W[OW["KAPPA"], 0], _fr(gd["kappa0"]), rtol=0, atol=1e-15)
    assert np.allclose(W[OW["OMEGA"], 1], _fr(gd["omega1"]), rtol=0, atol=1e-15)
    assert np.allclose(W[OW["VHAT"], 0], _fr(gd["vhat0"]), rtol=0, atol=1e-15)
    assert np.allclose(W[OW["XHZ"], 0], _fr(gd["xhat0_z"]), rtol=0, atol=1e-15)
    U = _layer_state(g, [_fr(v) for v in gd["layers"]])
    R, sig, qh = o.redistribute_diag(U)
    assert np.allclose(qh[0][0, :, :], _fr(gd["qhat0"]), rtol=0, atol=1e-15)
    s = sig[0][0]  # layer 0, (ny, nx, 3), physical units (dz = 1)
    key = "sigma_unlimited_z" if limiter == 2 else "sigma_limited_z"
    assert np.allclose(s[..., 2], _fr(gd[key]), rtol=0, atol=1e-13)
    assert np.all(np.abs(s[..., :2]) <= 1e-14)
    suffix = "unlimited" if limiter == 2 else "limited"
    assert np.allclose(R["rho"][0], _fr(gd["U0_" + suffix]), rtol=0, atol=1e-14)
    assert np.allclose(R["rho"][1], _fr(gd["U1_" + suffix]), rtol=0, atol=1e-14)
    assert np.array_equal(R["rho"][2], U["rho"][2])
    if limiter != 2:
        lam = s[..., 2] / _fr(gd["sigma_unlimited_z"])
        assert np.allclose(lam, _fr(gd["lambda_z"]), rtol=1e-12, atol=0)


def _fluid(o, inst, k, j, i):
    nx, ny, nz = o.n
    if inst == 3:
        if not (1 <= k <= nz - 1):
            return False
    elif not (0 <= k <= nz - 1):
        return False
    return o.geo[inst][OQ["ALPHA"], k, j % ny, i % nx] > 0.0


def _check_cv(o, inst, qh, su, sl, k, j, i, scalar):
    """Barth-Jespersen properties at the small CV (k, j, i).  Returns the
    factor(s) found."""
    nx, ny, nz = o.n
    W, G = o.w[inst], o.geo[inst]
    dx = np.array(o.dx)
    xh = lambda kk, jj, ii: np.array([W[OW["XHX"] + d, kk, jj % ny, ii % nx] for d in range(3)])
    vc = lambda kk, jj, ii: np.array([G[OQ["VCX"] + d, kk, jj % ny, ii % nx] for d in range(3)])
    x0 = xh(k, j, i)
    # fit points of the stencil (3 wide, 5 along directions lacking spread)
    def gather(wd):
        pts = []
        for oz in range(-wd[2], wd[2] + 1):
            for oy in range(-wd[1], wd[1] + 1):
                for ox in range(-wd[0], wd[0] + 1):
                    if (ox, oy, oz) != (0, 0, 0) and _fluid(o, inst, k + oz, j + oy, i + ox):
                        pts.append(((ox, oy, oz), qh[k + oz, (j + oy) % ny, (i + ox) % nx]))
        return pts
    pts = gather([1, 1, 1])
    spread = np.zeros(3)
    for (off, _) in pts:
        spread = np.maximum(spread, np.abs(np.array(off) + xh(k + off[2], j + off[1], i + off[0]) - x0))
    wd = [2 if spread[d] < 0.5 * (1 - 1e-12) else 1 for d in range(3)]
    if max(wd) == 2:
        pts = gather(wd)
    qi = qh[k, j % ny, i % nx]
    qs = [q for (_, q) in pts] + [qi]
    qmin, qmax = min(qs), max(qs)
    tol = 1e-12 * max(abs(qmin), abs(qmax), 1e-300)
    # evaluation points: centroids of the members of M_i, relative to x-hat_i
    mask = int(W[OW["MASK"], k, j % ny, i % nx])
    ev = []
    for oz in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for ox in (-1, 0, 1):
                if (mask >> ((oz + 1) * 9 + (oy + 1) * 3 + (ox + 1))) & 1:
                    ev.append(np.array([ox, oy, oz]) + vc(k + oz, j + oy, i + ox) - x0)
    gu = su * dx  # mesh units
    gl = sl * dx
    lams = []
    comps = [None] if scalar else [0, 1, 2]
    for d in comps:
        if scalar:
            nz_ = np.flatnonzero(gu != 0.0)
            if len(nz_) == 0:
                assert np.all(gl == 0.0)
                continue
            lam = gl[nz_[0]] / gu[nz_[0]]
            assert np.allclose(gl, lam * gu, rtol=1e-12, atol=1e-300)
            vals = [qi + lam * float(gu @ e) for e in ev]
            deltas = [float(gu @ e) for e in ev]
        else:
            if gu[d] == 0.0:
                assert gl[d] == 0.0
                continue
            lam = gl[d] / gu[d]
            vals = [qi + lam * gu[d] * e[d] for e in ev]
            deltas = [gu[d] * e[d] for e in ev]
        assert -1e-12 <= lam <= 1.0 + 1e-12, lam
        for v in vals:
            assert qmin - tol <= v <= qmax + tol, (v, qmin, qmax)
        if lam < 1.0 - 1e-12:
            tight = [abs(v - (qmax if dl > 0 else qmin)) <= tol for v, dl in zip(vals, deltas) if dl != 0]
            assert any(tight), (lam, vals, qmin, qmax)
        lams.append(lam)
    return lams


@pytest.mark.parametrize("cfg", [1, 2])
@pytest.mark.parametrize("scalar", [False, True])
def test_barth_jespersen_properties_random_state(cfg, scalar):
    """Random provisional states on the hill geometries, all four instances.
    Catches swapped bounds (negative or infeasible factors), bounds that
    leave out the CV itself or evaluation at the wrong points (a factor that
    is not the largest feasible one), and limiting the wrong component."""
    w = synth.make_workload(cfg)
    o = oracle.Oracle(w.grid, w.h_nodes, limiter=1 if scalar else 0)
    U = synth.state_random(w.grid, 23, amp=3.0)
    _, sl, qh = o.redistribute_diag(U)
    o.set_mode(limiter=2)
    _, su, qh2 = o.redistribute_diag(U)
    n_checked = n_limited = 0
    rng = np.random.default_rng(cfg)
    for f, inst in enumerate(oracle.FIELD_INST):
        assert np.array_equal(qh[f], qh2[f])
        W = o.w[inst]
        cand = np.argwhere((W[OW["SMALL"]] > 0) & (W[OW["TIER"]] > 0) & (W[OW["KAPPA"]] > 0))
        if len(cand) > 150:
            cand = cand[rng.choice(len(cand), 150, replace=False)]
        for (k, j, i) in cand:
            lams = _check_cv(o, inst, qh[f], su[f][k, j, i], sl[f][k, j, i], k, j, i, scalar)
            n_checked += 1
            n_limited += any(l < 1.0 - 1e-12 for l in lams)
    assert n_checked > 200 and n_limited > 50, (n_checked, n_limited)
