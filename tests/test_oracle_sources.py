"""Pins of the oracle momentum sources (compressible model of Section 2.1:
perturbation pressure gradient from the equation of state, buoyancy -rho' g)
against closed forms and invariants.  CPU only.

The reference state comes from the textbook isentropic atmosphere (Exner
function), written independently of the oracle's equation of state; the
state at rest pins the level indexing of rho theta0 / rho0, and the
perturbation pressure of single cells is checked against the plain
difference of two EOS pressures in extended precision.
Linear perturbation pressures pin sign, index direction and spacing of the
gradient on every momentum instance; a uniform density excess pins the
buoyancy; CVs next to covered cells pin the treatment of the terrain."""
import numpy as np
import pytest

import oracle
import synth


def _terrain_case():
    """24 x 20 x 16 cells, 78.125 m x 78.125 m x 31.25 m, Agnesi hill of 200 m:
    cut cells, covered cells and regular cells in every instance."""
    g = synth.Grid((24, 20, 16), (78.125, 78.125, 31.25))
    h = synth.terrain_agnesi(g, h0=200.0, a=400.0)
    return g, h


def _rhotheta_for(ref, p):
    """rho theta whose EOS pressure is p (inverse of p = P00 (R rho theta / P00)^gamma)."""
    return ref.P00 / ref.R * (p / ref.P00) ** (1.0 / ref.gamma)


def _p0_eos(ref):
    return ref.P00 * (ref.R * ref.rhotheta0 / ref.P00) ** ref.gamma


def _fluid_cv(o, inst):
    a = o.alpha(inst) > 0
    nz = o.n[2]
    if inst == 3:
        a[0] = False
    a[nz] = False
    return a


def _cell_fluid_dense(o):
    return o.alpha(0) > 0


@pytest.fixture(scope="module")
def case():
    g, h = _terrain_case()
    return g, h, oracle.Oracle(g, h), synth.reference_isentropic(g)


def test_reference_state_at_rest_has_no_source(case):
    """The hydrostatic reference state at rest is an exact steady state of the
    sources: p' = 0 and rho' = 0 on every fluid cell (well-balanced form)."""
    g, h, o, ref = case
    U = synth.state_reference(g, ref, 0, rho_noise=0.0, theta_noise=0.0, theta_amp=0.0, u0=0.0, w_amp=0.0)
    S = o.sources_dense(oracle.to_dense(U, o.n), ref)
    scale = ref.g * ref.rho0.max()
    for d in range(3):
        assert np.abs(S[d]).max() <= 1e-12 * scale, d


def test_perturbation_pressure_against_extended_precision(case):
    """p' of single perturbed cells (their lower x-neighbours at rest, p' = 0
    there, so S = -p' / dx) against P00 (R rho theta / P00)^gamma - p0
    evaluated in x87 extended precision (absolute error about 1e-14 Pa).
    Departures of about 1e-6 give |p'| up to about 0.5 Pa; the plain FP64
    difference of two pressures near 1e5 Pa would be off by about 1e-11 Pa,
    the cancellation-free form by about 1e-16 |p'|: the bound is 1e-13 Pa."""
    g, h, o, ref = case
    nx, ny, nz = g.n
    U = synth.state_reference(g, ref, 0, rho_noise=0.0, theta_noise=0.0, theta_amp=0.0, u0=0.0, w_amp=0.0)
    rng = np.random.default_rng(7)
    pert = np.zeros((nz, ny, nx), dtype=bool)
    pert[:, :, 1::2] = True
    rt = U["rhotheta"].copy()
    rt[pert] *= 1.0 + 1e-6 * rng.standard_normal(int(pert.sum()))
    U["rhotheta"] = rt
    S = o.sources_dense(oracle.to_dense(U, o.n), ref)[0][:nz]
    fc = (o.alpha(0) > 0)[:nz]
    cv = (o.alpha(1) > 0)[:nz]
    sel = cv & fc & np.roll(fc, 1, axis=2) & pert
    assert sel.sum() > 1000
    L = np.longdouble
    P00, R, gam = L(ref.P00), L(ref.R), L(ref.gamma)
    p_ld = P00 * (R * rt.astype(L) / P00) ** gam
    p0_ld = P00 * (R * ref.rhotheta0.astype(L) / P00) ** gam
    pp_ld = p_ld - p0_ld[:, None, None]
    got = -S * g.dx[0]
    err = np.abs(got[sel] - pp_ld[sel].astype(np.float64))
    assert 0.05 < np.abs(pp_ld[sel]).max() < 1.0
    assert err.max() <= 1e-13, err.max()


@pytest.mark.parametrize("d", [0, 1, 2])
def test_linear_perturbation_pressure(case, d):
    """p' = a * (cell-centre coordinate along d): the source of a momentum CV
    whose two cells are fluid is -a, except across the periodic seam, where the
    difference spans the domain: -(x_0 - x_{n-1}) a / dx = a (n - 1).  CVs with
    a covered cell get no pressure force.  rho = rho0 keeps the buoyancy zero."""
    g, h, o, ref = case
    nx, ny, nz = g.n
    a = 0.37 if d < 2 else -0.8
    idx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    coord = (idx[2 - d] + 0.5) * g.dx[d]
    p = _p0_eos(ref)[:, None, None] + a * coord
    U = synth.state_reference(g, ref, 0, rho_noise=0.0, theta_noise=0.0, theta_amp=0.0, u0=0.0, w_amp=0.0)
    U["rhotheta"] = _rhotheta_for(ref, p)
    S = o.sources_dense(oracle.to_dense(U, o.n), ref)[d]
    fc = _cell_fluid_dense(o)
    fc[nz] = False
    lower = np.roll(fc, 1, axis=2 - d)
    if d == 2:
        lower[0] = False
    cv = _fluid_cv(o, d + 1)
    both = cv & fc & lower
    one = cv & ~(fc & lower)
    assert both.sum() > 100 and one.sum() > 10
    expect = np.full(S.shape, -a)
    if d < 2:
        seam = [slice(None)] * 3
        seam[2 - d] = 0
        expect[tuple(seam)] = a * (g.n[d] - 1)
    np.testing.assert_allclose(S[both], expect[both], rtol=1e-9, atol=1e-9)
    assert np.all(S[one] == 0.0)
    assert np.all(S[~cv] == 0.0)


def test_buoyancy_of_uniform_density_excess(case):
    """rho = rho0 + c with rho theta unchanged (p' = 0): every fluid z-face CV
    gets -g c, whether one or both of its cells are fluid; x and y sources vanish."""
    g, h, o, ref = case
    c = 0.013
    U = synth.state_reference(g, ref, 0, rho_noise=0.0, theta_noise=0.0, theta_amp=0.0, u0=0.0, w_amp=0.0)
    rt = U["rhotheta"].copy()
    U["rho"] = U["rho"] + c
    U["rhotheta"] = rt
    S = o.sources_dense(oracle.to_dense(U, o.n), ref)
    scale = ref.g * c
    assert np.abs(S[0]).max() <= 1e-9 * scale and np.abs(S[1]).max() <= 1e-9 * scale
    cv = _fluid_cv(o, 3)
    np.testing.assert_allclose(S[2][cv], -ref.g * c, rtol=1e-9)
    assert np.all(S[2][~cv] == 0.0)


def test_buoyancy_averages_the_two_cells(case):
    """rho' differing between levels: the z-face CV between two fluid cells
    gets -g times their mean; one whose lower cell is covered gets -g rho' of
    the upper cell."""
    g, h, o, ref = case
    nz = g.n[2]
    c = 0.01 * (1.0 + np.arange(nz, dtype=np.float64))
    U = synth.state_reference(g, ref, 0, rho_noise=0.0, theta_noise=0.0, theta_amp=0.0, u0=0.0, w_amp=0.0)
    rt = U["rhotheta"].copy()
    U["rho"] = U["rho"] + c[:, None, None]
    U["rhotheta"] = rt
    S = o.sources_dense(oracle.to_dense(U, o.n), ref)[2]
    fc = _cell_fluid_dense(o)
    cv = _fluid_cv(o, 3)
    k = np.arange(nz + 1)[:, None, None] * np.ones(S.shape)
    kk = np.clip(k.astype(int), 1, nz - 1)
    both = cv & fc & np.roll(fc, 1, axis=0)
    upper_only = cv & fc & ~np.roll(fc, 1, axis=0)
    assert both.sum() > 100 and upper_only.sum() > 10
    np.testing.assert_allclose(S[both], -ref.g * 0.5 * (c[kk[both] - 1] + c[kk[both]]), rtol=1e-9)
    np.testing.assert_allclose(S[upper_only], -ref.g * c[kk[upper_only]], rtol=1e-9)


def test_stage_adds_cdt_times_source(case):
    """The stage update with a reference state differs from the one without by
    c dt times the source, on the momenta only."""
    g, h, o, ref = case
    U = synth.state_reference(g, ref, 5)
    cdt = 0.3
    a = o.advance(U, U, cdt)
    b = o.advance(U, U, cdt, ref)
    S = o.sources(U, ref)
    for f in ("rho", "rhotheta"):
        assert np.array_equal(a[f], b[f])
    for f in ("rhou", "rhov", "rhow"):
        np.testing.assert_allclose(b[f] - a[f], cdt * S[f], rtol=0, atol=1e-12 * np.abs(a[f]).max())
        assert np.abs(S[f]).max() > 0
