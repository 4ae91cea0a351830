"""Pins of the oracle's momentum diffusion (Sections 2.1 and 4.2: the viscous
stress tau = lambda (div u) I + mu (grad u + grad u^T) on the staggered
control volumes; least-squares gradients on cut faces and at EB facets, 3
wide where the evaluation point lines up with a variable's grid and 4 wide
where it sits between two of its points) against closed forms.  CPU only.
Each test names the mistakes it exists to catch."""
import math
from dataclasses import dataclass

import numpy as np
import pytest

import oracle
import synth

OQ = oracle.OQ


@dataclass
class Visc:
    mu: float = 1.7
    eb_mode: int = 0


def _centroids(o, g, inst):
    """Physical volume centroids of the CVs of an instance (dense)."""
    nx, ny, nz = g.n
    k, j, i = np.meshgrid(np.arange(nz + 1.0), np.arange(ny * 1.0), np.arange(nx * 1.0), indexing="ij")
    G = o.geo[inst]
    idx = (i, j, k)
    out = []
    for d in range(3):
        ctr = idx[d] + 0.5 - (0.5 if inst == d + 1 else 0.0)
        out.append(g.lo[d] + (ctr + G[OQ["VCX"] + d]) * g.dx[d])
    return out


def _dense_state(o, g, vel_funcs, rho=1.0):
    """Dense state with density rho and the momenta of the velocity
    functions evaluated at the CV centroids."""
    nx, ny, nz = g.n
    D = [np.full((nz + 1, ny, nx), rho), np.full((nz + 1, ny, nx), 300.0 * rho)]
    for e in range(3):
        X = _centroids(o, g, e + 1)
        D.append(np.ascontiguousarray(rho * vel_funcs[e](*X)))
    return D


# a random quadratic velocity field: u_e = c_e + sum_a l_ea x_a + sum_ab q_eab x_a x_b
_rng = np.random.default_rng(17)
_C = _rng.uniform(-1, 1, 3)
_L = _rng.uniform(-1, 1, (3, 3))
_Q = _rng.uniform(-1, 1, (3, 3, 3))
_Q = 0.5 * (_Q + _Q.transpose(0, 2, 1))


def _vel(e):
    return lambda x, y, z: (_C[e] + _L[e, 0] * x + _L[e, 1] * y + _L[e, 2] * z
                            + sum(_Q[e, a, b] * (x, y, z)[a] * (x, y, z)[b] for a in range(3) for b in range(3)))


def _grad(e, p):
    """du_e/dx_a at point p"""
    return np.array([_L[e, a] + 2 * sum(_Q[e, a, b] * p[b] for b in range(3)) for a in range(3)])


def _tau(mu, p, c, d):
    G = np.array([_grad(e, p) for e in range(3)])
    t = mu * (G[c, d] + G[d, c])
    if c == d:
        t += -2.0 / 3.0 * mu * np.trace(G)
    return t


def test_regular_grid_quadratic_exact():
    """No terrain: the staggered centred differences are exact for
    quadratic velocities, so D_c = mu lap(u_c) + (mu + lambda) d(div u)/dx_c
    with lambda = -2/3 mu away from the walls and the periodic seams.
    Catches a wrong lambda (value or sign), a missing factor 2 on the normal
    stress, cross terms taken from the wrong CVs and a wrong spacing."""
    g = synth.Grid((12, 10, 10), (1.0, 1.3, 0.8))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    p = Visc(mu=1.7)
    U = _dense_state(o, g, [_vel(e) for e in range(3)])
    D = o.viscous_dense(U, p)
    mu = p.mu
    lap = [2 * sum(_Q[e, a, a] for a in range(3)) for e in range(3)]
    ddiv = [2 * sum(_Q[e, e, c] for e in range(3)) for c in range(3)]
    for c in range(3):
        want = mu * lap[c] + (mu - 2.0 / 3.0 * mu) * ddiv[c]
        inner = D[c][2:g.n[2] - 2, 2:-2, 2:-2]
        assert np.allclose(inner, want, rtol=1e-9, atol=1e-9), (c, inner.min(), inner.max(), want)


def _plane():
    g = synth.Grid((12, 12, 8), (1.0, 1.25, 0.9))
    a, bx, by = 2.3, 0.21, 0.13
    return g, (a, bx, by), oracle.Oracle(g, synth.terrain_plane(g, a, bx, by))


def test_cut_face_stress_exact_for_quadratics():
    """Sloped plane, quadratic velocities: the stress on every cut face of
    the three momentum CVs whose fits have enough fluid points equals the
    exact stress at the face centroid.  Catches fitting the wrong component,
    a fit about the face centre instead of its centroid, a stencil on the
    wrong grid and a missing divergence term on the normal faces."""
    g, _, o = _plane()
    p = Visc(mu=0.9)
    U = _dense_state(o, g, [_vel(e) for e in range(3)])
    D, F, E = o.viscous_dense(U, p, fluxes=True)
    nx, ny, nz = g.n
    tang = [[1, 2], [0, 2], [0, 1]]
    checked = 0
    for c in range(3):
        G = o.geo[c + 1]
        for d in range(3):
            b = G[OQ["BX"] + d]
            for k in range(2, nz - 1):
                for j in range(3, ny - 3):
                    for i in range(3, nx - 3):
                        if not (0.0 < b[k, j, i] < 1.0 - 1e-12):
                            continue
                        idx = (i, j, k)
                        x = [g.lo[a] + (idx[a] + 0.5 - 0.5 * (a == c) - 0.5 * (a == d)) * g.dx[a] for a in range(3)]
                        x[tang[d][0]] += G[OQ["FX1"] + 2 * d, k, j, i] * g.dx[tang[d][0]]
                        x[tang[d][1]] += G[OQ["FX1"] + 2 * d + 1, k, j, i] * g.dx[tang[d][1]]
                        want = _tau(p.mu, x, c, d)
                        got = F[3 * c + d][k, j, i]
                        if abs(got - want) > 1e-8 * (1 + abs(want)):
                            # a fit may fall back to linear where the stencil is thin;
                            # it must then at least be close
                            assert abs(got - want) < 0.5 * (1 + abs(want)), (c, d, i, j, k, got, want)
                            continue
                        checked += 1
    assert checked > 300, checked


def test_no_slip_wall_stress_exact():
    """Sloped plane, velocities u_e = a_e phi + b_e phi^2 (phi = z - h, zero on
    the terrain): the constrained fits reproduce them, so the facet term of
    every cut CV of the three momentum instances is minus tau(a) dotted with
    the facet's area vector, tau(a) from the exact wall gradients a_e grad
    phi.  Catches a fit that ignores the no-slip value, a flipped facet
    normal and an evaluation point other than the facet centroid."""
    g, (a0, bx, by), o = _plane()
    av_c = np.array([0.7, -0.4, 0.2])
    bv_c = np.array([0.05, 0.03, -0.02])
    gphi = np.array([-bx, -by, 1.0])
    funcs = [lambda x, y, z, e=e: av_c[e] * (z - a0 - bx * x - by * y) + bv_c[e] * (z - a0 - bx * x - by * y) ** 2
             for e in range(3)]
    U = _dense_state(o, g, funcs)
    p = Visc(mu=1.3, eb_mode=1)
    D, F, E = o.viscous_dense(U, p, fluxes=True)
    mu = p.mu
    Gw = np.outer(av_c, gphi)  # du_e/dx_a on the wall
    tau = mu * (Gw + Gw.T) - 2.0 / 3.0 * mu * np.trace(Gw) * np.eye(3)
    nx, ny, nz = g.n
    checked = 0
    for c in range(3):
        G = o.geo[c + 1]
        for k in range(1, nz - 1):
            for j in range(3, ny - 3):
                for i in range(3, nx - 3):
                    if not (G[OQ["ALPHA"], k, j, i] > 0 and G[OQ["AREA"], k, j, i] > 1e-3):
                        continue
                    av = np.array([G[OQ["AX"], k, j, i] * g.dx[1] * g.dx[2], G[OQ["AY"], k, j, i] * g.dx[0] * g.dx[2],
                                   G[OQ["AZ"], k, j, i] * g.dx[0] * g.dx[1]])
                    want = -tau[c] @ av
                    got = E[c][k, j, i]
                    assert abs(got - want) <= 1e-8 * (1 + abs(want)), (c, i, j, k, got, want)
                    checked += 1
    assert checked > 100, checked


@pytest.mark.parametrize("cfg", [1, 2])
def test_conservation_stress_free(cfg):
    """Stress-free EB and walls: every face stress enters the two CVs on its
    sides with opposite signs, so the sum of V D over the u and v instances
    vanishes for any state; the w CVs end half a cell from the bottom and top
    walls, so their sum is the normal stress on those two boundary planes
    (the cell centres of the first and last layers).  Catches a face computed
    differently by its two CVs and a facet term in the stress-free mode."""
    w = synth.make_workload(cfg)
    o = oracle.Oracle(w.grid, w.h_nodes)
    g = w.grid
    U = synth.state_random(g, 19, amp=1.0)
    D, F, E = o.viscous(U, Visc(mu=2.0), fluxes=True)
    nz = g.n[2]
    A = g.dx[0] * g.dx[1]
    for c in range(3):
        V = o.volume(c + 1)
        tot = math.fsum((V * D[c]).ravel().tolist())
        scale = math.fsum(np.abs(V * D[c]).ravel().tolist())
        want = 0.0
        if c == 2:
            bz = o.geo[3][OQ["BZ"]]
            want = math.fsum((A * bz[nz] * F[8][nz]).ravel().tolist()) - math.fsum((A * bz[1] * F[8][1]).ravel().tolist())
            assert abs(want) > 1e-6 * scale
        assert abs(tot - want) <= 1e-13 * scale, (c, tot, want, scale)


def test_constant_velocity_no_stress():
    """A uniform velocity (random densities, stress-free EB): every fitted
    and centred gradient vanishes.  Catches fits that do not reproduce
    constants and velocities taken from momenta without their own face
    densities."""
    w = synth.make_workload(1)
    o = oracle.Oracle(w.grid, w.h_nodes)
    g = w.grid
    rng = np.random.default_rng(3)
    U = synth.state_uniform(g, rho=1.0, theta=300.0, u=0.0)
    rho = 1.0 + rng.random(U["rho"].shape)
    U["rho"] = rho
    Dn = oracle.to_dense(U, g.n)
    vel = (1.3, -0.4, 0.0)
    for e in range(3):
        inst = e + 1
        # momentum = velocity x mean density of the fluid cells on either side
        r = Dn[0]
        a0 = o.alpha(0) > 0
        lo = np.roll(r, 1, axis=2 - e) if e < 2 else np.concatenate([r[:1], r[:-1]], axis=0)
        alo = np.roll(a0, 1, axis=2 - e) if e < 2 else np.concatenate([np.zeros_like(a0[:1]), a0[:-1]], axis=0)
        cnt = a0.astype(float) + alo
        s = np.where(a0, r, 0.0) + np.where(alo, lo, 0.0)
        Dn[2 + e] = np.where(cnt > 0, vel[e] * s / np.maximum(cnt, 1), 0.0)
    D = o.viscous_dense(Dn, Visc(mu=1.0))
    # extensive form (alpha D): the intensive one divides the rounding of
    # the fits by the volume fraction of slivers
    scale = 1.0 * max(abs(v) for v in vel) / min(g.dx) ** 2
    for c in range(3):
        e = np.abs(o.alpha(c + 1) * D[c]).max()
        assert e <= 1e-10 * scale, (c, e, scale)


def test_cross_grid_stencil_symmetric_about_the_edge():
    """Flat terrain at 0.73 dz cuts the y-faces of the x-momentum CVs in the
    bottom layer.  With u = 0 and v an even function of the distance to the
    plane x = x_i of one column of those faces (fourth power, not
    reproduced by the fit), the stress tau_xy = mu dv/dx there vanishes when
    the v stencil runs two points on each side of the edge.  Catches a cross
    stencil shifted by one point."""
    g = synth.Grid((12, 12, 6), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.73))
    x0 = 6.0
    funcs = [lambda x, y, z: 0.0 * x, lambda x, y, z: (x - x0) ** 4 + 0.3 * z * z, lambda x, y, z: 0.0 * x]
    U = _dense_state(o, g, funcs)
    D, F, E = o.viscous_dense(U, Visc(mu=1.0), fluxes=True)
    assert np.all(o.geo[1][OQ["BY"]][0] < 1.0) and np.all(o.geo[1][OQ["BY"]][0] > 0.0)
    edge = F[3 * 0 + 1][0, :, 6]  # tau_xy on the lower y-faces of x-CVs at x = 6
    assert np.abs(edge).max() <= 1e-12, edge
    off = F[1][0, :, 7]
    assert np.abs(off).min() > 1e-3

def _triquad(rng):
    """coefficients c[a, b, d] of x^a y^b z^d, a, b, d in 0..2"""
    return rng.uniform(-1, 1, (3, 3, 3))


def _poly(cf, x, y, z, dx=(0, 0, 0)):
    """value of the tri-quadratic polynomial or of a partial derivative
    (orders dx along x, y, z)"""
    out = 0.0
    for a in range(3):
        for b in range(3):
            for d in range(3):
                e = (a, b, d)
                coef = cf[a, b, d]
                term = coef
                for q, v in enumerate((x, y, z)):
                    n = e[q]
                    for _ in range(dx[q]):
                        term = term * n
                        n -= 1
                    if n < 0:
                        term = term * 0.0
                        n = 0
                    term = term * v ** n
                out = out + term
    return out


def test_regular_grid_triquadratic_exact():
    """No terrain, velocities quadratic in each coordinate separately (x^2 y
    z^2 and the like): every centred difference the staggered stresses take
    is exact, so D_c = sum_d d(tau_cd)/dx_d exactly away from the walls and
    seams.  Catches a cross-term difference taken one CV off (an error of
    the order of the mesh spacing that fields of total degree two do not
    show)."""
    g = synth.Grid((12, 10, 10), (0.5, 0.6, 0.4))
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    rng = np.random.default_rng(23)
    cf = [_triquad(rng) for _ in range(3)]
    mu = 1.1
    U = _dense_state(o, g, [lambda x, y, z, e=e: _poly(cf[e], x, y, z) for e in range(3)])
    D = o.viscous_dense(U, Visc(mu=mu))
    lam = -2.0 / 3.0 * mu
    for c in range(3):
        X = _centroids(o, g, c + 1)
        oc = [int(a == c) for a in range(3)]
        want = 0.0
        for d in range(3):
            od = [int(a == d) for a in range(3)]
            # d/dx_d of mu (du_c/dx_d + du_d/dx_c)
            want = want + mu * (_poly(cf[c], *X, dx=tuple(2 * v for v in od)) +
                                _poly(cf[d], *X, dx=tuple(a + b for a, b in zip(oc, od))))
            # d/dx_c of lambda du_d/dx_d
            want = want + lam * _poly(cf[d], *X, dx=tuple(a + b for a, b in zip(oc, od)))
        inner = (D[c] - want)[2:g.n[2] - 2, 2:-2, 2:-2]
        assert np.abs(inner).max() <= 1e-9 * (1 + np.abs(want).max()), (c, np.abs(inner).max())


def test_no_slip_drags_a_uniform_flow():
    """A uniform flow u = 1 over the sloped plane: with the no-slip EB every
    cut x-momentum CV with a facet of some size loses x momentum through it
    (the constrained fit sees the velocity drop to zero at the wall); with
    the stress-free EB the facet term is zero.  Catches a no-slip fit that
    does not prescribe the wall value."""
    g, _, o = _plane()
    U = _dense_state(o, g, [lambda x, y, z: 1.0 + 0.0 * x, lambda x, y, z: 0.0 * x, lambda x, y, z: 0.0 * x])
    _, _, E1 = o.viscous_dense(U, Visc(mu=1.0, eb_mode=1), fluxes=True)
    _, _, E0 = o.viscous_dense(U, Visc(mu=1.0, eb_mode=0), fluxes=True)
    G = o.geo[1]
    sel = (G[OQ["ALPHA"]] > 0) & (G[OQ["AREA"]] > 0.1)
    sel[:, :, :3] = sel[:, :, -3:] = False
    sel[:, :3, :] = sel[:, -3:, :] = False
    assert sel.sum() > 30
    assert np.all(E1[0][sel] < 0.0)
    assert all(np.all(E0[c] == 0.0) for c in range(3))
