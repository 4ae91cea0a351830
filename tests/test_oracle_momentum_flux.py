"""Pins of the oracle's advective fluxes on the three staggered instances
(Section 4.1: the momentum flux rho u (x) u on the faces of the staggered
control volumes of Section 3.1, Eq. update-fc) against closed forms.  CPU
only.

Readings pinned here: the mass flux through a face of a staggered CV is the
mean of the two stored face momenta next to it over those whose CV holds
fluid (one such: its value); the advected
velocity is the stored momentum divided by the mean density of the fluid
cells on either side of its face; the upwind stencil runs over the CVs of
the instance itself.  Each test names the mistake it exists to catch."""
import numpy as np
import pytest

import oracle
import synth

DX = (1.0, 1.25, 0.8)
N = (10, 10, 8)
MOM = ("rhou", "rhov", "rhow")


def _grid():
    return synth.Grid(N, DX)


def _entry_xyz(name, shape):
    """Physical location (X, Y, Z) of every entry of a momentum array in the
    public layout: rhou at (i dx, (j+1/2) dy, (k+1/2) dz), etc."""
    k, j, i = np.meshgrid(*[np.arange(s, dtype=float) for s in shape], indexing="ij")
    X, Y, Z = (i + 0.5) * DX[0], (j + 0.5) * DX[1], (k + 0.5) * DX[2]
    if name == "rhou":
        X = i * DX[0]
    elif name == "rhov":
        Y = j * DX[1]
    else:
        Z = k * DX[2]
    return X, Y, Z


def _cv_centre(s, shape):
    """Centre of every CV (dense instance storage (nz+1, ny, nx)) of the
    staggered instance along axis s."""
    k, j, i = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    c = [(i + 0.5) * DX[0], (j + 0.5) * DX[1], (k + 0.5) * DX[2]]
    c[s] = [i, j, k][s] * DX[s]
    return c


def _base(g):
    U = synth.state_uniform(g, rho=1.0, theta=1.0, u=0.0)
    for m in MOM:
        U[m][...] = 0.0
    return U


def _interior(shape, s, d, stencil_axis=None, lo=2, hi=2):
    """Mask of CVs away from the periodic seams and walls (dense storage)."""
    nz1, ny, nx = shape
    nz = nz1 - 1
    m = np.zeros(shape, bool)
    m[:, lo:ny - hi, lo:nx - hi] = True
    k = np.arange(nz1)
    kmin, kmax = (1, nz - 1) if s == 2 else (0, nz - 1)
    if d == 2:  # lower z-face: not the bottom wall
        kmin = max(kmin, 1)
    if stencil_axis == 2:  # four-point z stencil inside the instance's CV planes
        kmin, kmax = kmin + 2, kmax - 1
    m &= ((k >= kmin) & (k <= kmax))[:, None, None]
    return m


@pytest.mark.parametrize("s", [0, 1, 2])
def test_mass_flux_pairing_on_staggered_faces(s):
    """Momentum of instance s uniform (so the advected velocity is one value
    and the upwind face value is exact), the momentum normal to face
    direction d linear in x, y, z: the provisional flux on the lower d-face of
    every s-CV must be C * L(face centre).  Catches pairing the face momentum
    with its neighbour on the wrong side along s (e.g. rho v[i] with
    rho v[i+1] on the x-CV y-face) or along the other axes."""
    g = _grid()
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    C0 = 1.7
    coef = (0.3, 0.11, -0.07, 0.05)
    for d in range(3):
        if d == s:
            continue
        U = _base(g)
        U[MOM[s]][...] = C0
        X, Y, Z = _entry_xyz(MOM[d], U[MOM[d]].shape)
        U[MOM[d]] = coef[0] + coef[1] * X + coef[2] * Y + coef[3] * Z
        U["rhow"][0] = U["rhow"][-1] = 0.0
        _, Fh = o.face_fluxes(U, 2 + s)
        shape = Fh[d].shape
        c = _cv_centre(s, shape)
        c[d] = c[d] - 0.5 * DX[d]
        expect = C0 * (coef[0] + coef[1] * c[0] + coef[2] * c[1] + coef[3] * c[2])
        m = _interior(shape, s, d)
        assert np.abs(Fh[d] - expect)[m].max() <= 1e-13 * np.abs(expect[m]).max(), (s, d)


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("s", [0, 1, 2])
def test_own_axis_stencil_reproduces_quadratic(s, sign):
    """Momentum of instance s = CV averages of a quadratic q along s (rho = 1):
    on the lower s-face of the s-CV at index i, at x_f = (i - 1/2) dx_s, the
    upwind value is q(x_f) exactly and the mass flux is the mean of the two
    CV averages, q(x_f) + q2 dx_s^2 / 3, so the provisional flux is
    (q(x_f) + q2 dx_s^2 / 3) q(x_f).  Catches an off-by-one of the stencil
    along the instance's own axis and a wrong own-axis mass-flux pairing."""
    g = _grid()
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    q2, q1, q0 = 0.013 * sign, -0.05 * sign, 2.0 * sign
    q = lambda x: q2 * x * x + q1 * x + q0
    Q = lambda x: q2 * x ** 3 / 3 + q1 * x * x / 2 + q0 * x
    D = DX[s]
    U = _base(g)
    X = _entry_xyz(MOM[s], U[MOM[s]].shape)[s]
    U[MOM[s]] = (Q(X + 0.5 * D) - Q(X - 0.5 * D)) / D  # average over the s-CV
    U["rhow"][0] = U["rhow"][-1] = 0.0
    _, Fh = o.face_fluxes(U, 2 + s)
    shape = Fh[s].shape
    xf = _cv_centre(s, shape)[s] - 0.5 * D
    expect = (q(xf) + q2 * D * D / 3.0) * q(xf)
    m = _interior(shape, s, s, stencil_axis=s if s == 2 else None, lo=2, hi=2)
    if s != 2:  # the four-point stencil i-2 .. i+1 must not cross the seam
        sl = [slice(None)] * 3
        sl[2 - s] = slice(None, 2)
        m[tuple(sl)] = False
    assert m.sum() > 50
    assert np.abs(Fh[s] - expect)[m].max() <= 1e-12 * np.abs(expect[m]).max(), s


@pytest.mark.parametrize("sign", [1.0, -1.0])
@pytest.mark.parametrize("s", [0, 1, 2])
def test_cross_axis_stencil_reproduces_quadratic(s, sign):
    """Momentum of instance s = averages over the s-CVs' extent along d != s
    of a quadratic q(x_d), the momentum normal to d uniform M: the provisional
    flux on the lower d-face is M q(face coordinate).  Catches a stencil
    shifted along the other axes of a staggered instance."""
    g = _grid()
    o = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    q2, q1, q0 = 0.02, -0.09, 1.5
    q = lambda x: q2 * x * x + q1 * x + q0
    Q = lambda x: q2 * x ** 3 / 3 + q1 * x * x / 2 + q0 * x
    M = 0.8 * sign
    for d in range(3):
        if d == s:
            continue
        U = _base(g)
        Xd = _entry_xyz(MOM[s], U[MOM[s]].shape)[d]
        D = DX[d]
        U[MOM[s]] = (Q(Xd + 0.5 * D) - Q(Xd - 0.5 * D)) / D
        U[MOM[d]][...] = M
        U["rhow"][0] = U["rhow"][-1] = 0.0
        _, Fh = o.face_fluxes(U, 2 + s)
        shape = Fh[d].shape
        xf = _cv_centre(s, shape)[d] - 0.5 * D
        expect = M * q(xf)
        m = _interior(shape, s, d, stencil_axis=2 if d == 2 else None)
        if d != 2:
            sl = [slice(None)] * 3
            sl[2 - d] = slice(None, 2)
            m[tuple(sl)] = False
        assert m.sum() > 50
        assert np.abs(Fh[d] - expect)[m].max() <= 1e-12 * np.abs(expect[m]).max(), (s, d)


def test_face_velocity_uses_mean_density_of_fluid_neighbours():
    """Random densities; each face momentum is C times the mean density of
    the fluid cells on either side of its face (one side only next to a
    covered cell: flat terrain at 1.3 dz covers layer 0, so the z-CV at k = 1
    sees only cell 1).  The advected velocity is then C on every CV, and the
    provisional flux divided by the mass flux is C.  Catches a face velocity
    taken from one cell's density, or from a mean that counts a covered
    cell; and a mass flux that reads the momentum of a covered CV as 0 in
    the mean (at k = 1 the flux must be the fluid neighbour's momentum)."""
    g = synth.Grid((8, 8, 6), (1.0, 1.0, 1.0))
    o = oracle.Oracle(g, synth.terrain_flat(g, 1.3))
    rng = np.random.default_rng(3)
    U = synth.state_uniform(g, rho=1.0, theta=1.0, u=0.0)
    rho = 1.0 + rng.random(U["rho"].shape)
    U["rho"] = rho
    U["rhotheta"] = rho.copy()
    Cw, Mu = 0.7, 1.1
    nz = g.n[2]
    w = np.zeros_like(U["rhow"])
    w[2:nz] = Cw * 0.5 * (rho[1:nz - 1] + rho[2:nz])
    w[1] = Cw * rho[1]  # cell 0 is covered
    U["rhow"] = w
    U["rhou"][...] = Mu
    _, Fh = o.face_fluxes(U, 4)
    # lower x-faces of the z-CVs: mass flux = mean of rho u at k-1, k over the
    # fluid x-CVs; at k = 1 the x-CV at k = 0 is covered, so rho u at k = 1
    m = np.full(Fh[0].shape, Mu)
    sel = np.zeros(Fh[0].shape, bool)
    sel[1:nz] = True
    assert np.allclose(Fh[0][sel] / m[sel], Cw, rtol=1e-14, atol=0)
    # x-CVs with the velocity C on every fluid CV: rho u = C mean(rho) over x
    U2 = synth.state_uniform(g, rho=1.0, theta=1.0, u=0.0)
    o2 = oracle.Oracle(g, synth.terrain_flat(g, 0.0))
    U2["rho"] = rho
    U2["rhotheta"] = rho.copy()
    Cu = 1.9
    ru = np.empty_like(U2["rhou"])
    ru[:, :, :g.n[0]] = Cu * 0.5 * (np.roll(rho, 1, axis=2) + rho)
    ru[:, :, -1] = ru[:, :, 0]
    U2["rhou"] = ru
    U2["rhov"][...] = 0.0
    U2["rhow"][...] = 0.0
    _, Fh2 = o2.face_fluxes(U2, 2)
    mass = 0.5 * (np.roll(ru[:, :, :g.n[0]], 1, axis=2) + ru[:, :, :g.n[0]])
    assert np.allclose(Fh2[0][:nz] / mass, Cu, rtol=1e-14, atol=0)
