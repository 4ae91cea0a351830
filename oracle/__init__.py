"""FP64 CPU oracle for the staggered cut-cell update with weighted state
redistribution.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use this package; the library and its Python binding
never import it.  It shares no code with the HIP path; the only common input
is the seeded generator module ``synth``.

The arithmetic lives in plain C (``geom.c``, ``flux.c``, ``wsrd.c``) compiled
with gcc; this module marshals numpy arrays through ctypes, converts between
the public staggered layout and the oracle's dense per-instance storage, runs
the three-stage Runge-Kutta loop (Algorithm 1 of the paper) and computes the
conserved sums with exactly rounded summation (``math.fsum``).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = ["geom.c", "levelset.c", "coarse.c", "flux.c", "wsrd.c", "source.c", "restrict.c", "diffusion.c", "viscous.c"]

# geometry quantity indices (mirror oracle.h)
OQ = dict(ALPHA=0, BX=1, BY=2, BZ=3, FX1=4, FX2=5, FY1=6, FY2=7, FZ1=8, FZ2=9,
          VCX=10, VCY=11, VCZ=12, AX=13, AY=14, AZ=15, AREA=16, EBX=17, EBY=18, EBZ=19)
OQ_N = 20
OW = dict(SMALL=0, TIER=1, MASK=2, NCOUNT=3, KAPPA=4, OMEGA=5, VHAT=6, XHX=7, XHY=8, XHZ=9)
OW_N = 10

FIELDS = ("rho", "rhotheta", "rhou", "rhov", "rhow")
FIELD_INST = (0, 0, 1, 2, 3)
RK3_C = (1.0 / 3.0, 0.5, 1.0)


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, no FMA contraction, OpenMP
    over the planes of every loop nest)."""
    srcs = [os.path.join(_HERE, s) for s in _SRC]
    if not force and os.path.exists(_SO):
        so_t = os.path.getmtime(_SO)
        hdrs = [os.path.join(_HERE, h) for h in ("oracle.h", "geom_piece.h", "lsq.h")]
        if all(os.path.getmtime(s) <= so_t for s in srcs + hdrs):
            return _SO
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp", "-Wall",
           "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class _Src(C.Structure):
    _fields_ = [("P00", C.c_double), ("R", C.c_double), ("gamma", C.c_double), ("g", C.c_double)]


class _Diff(C.Structure):
    _fields_ = [("alpha_theta", C.c_double), ("eb_mode", C.c_int32), ("theta_wall", C.c_double)]


class _Visc(C.Structure):
    _fields_ = [("mu", C.c_double), ("eb_mode", C.c_int32)]


class _Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dx", C.c_double * 3), ("lo", C.c_double * 3),
                ("small_vfrac", C.c_double), ("limiter", C.c_int32), ("eb_flux", C.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_SO)
        P = C.POINTER
        dp = P(C.c_double)
        dpp = P(dp)
        i8pp = P(P(C.c_int8))
        lib.orc_geometry.argtypes = [P(_Grid), dp, dpp, i8pp]
        lib.orc_geometry_levelset.argtypes = [P(_Grid), dp, dpp, i8pp]
        lib.orc_geometry_merged.argtypes = [P(_Grid), dp, C.c_int, dpp, i8pp]
        lib.orc_levelset_piece.argtypes = [P(_Grid), dp, C.c_int, C.c_int, C.c_int, C.c_int, dp]
        lib.orc_wsrd_setup.argtypes = [P(_Grid), dpp, dpp]
        lib.orc_advance.argtypes = [P(_Grid), dpp, dpp, dpp, dpp, C.c_double]
        lib.orc_redistribute.argtypes = [P(_Grid), dpp, dpp, dpp, dpp]
        lib.orc_redistribute_sig.argtypes = [P(_Grid), dpp, dpp, dpp, dpp, dpp]
        lib.orc_redistribute_diag.argtypes = [P(_Grid), dpp, dpp, dpp, dpp, dpp, dpp]
        lib.orc_face_fluxes.argtypes = [P(_Grid), dpp, dpp, C.c_int, dpp, dpp]
        lib.orc_sources.argtypes = [P(_Grid), dpp, dpp, P(_Src), dp, dp, dpp]
        lib.orc_coarsen_geometry.argtypes = [P(_Grid), dpp, dp, dpp]
        lib.orc_restrict.argtypes = [P(_Grid), dpp, dpp, dpp]
        lib.orc_box_moments.argtypes = [P(_Grid), dp, C.c_int, C.c_int, dp, C.c_double,
                                        C.c_double, C.c_int, dp]
        lib.orc_diffusion.argtypes = [P(_Grid), dpp, dpp, P(_Diff), dp, dpp, dp]
        lib.orc_viscous.argtypes = [P(_Grid), dpp, dpp, P(_Visc), dpp, dpp, dpp]
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_set_threads.restype = C.c_int
        _lib = lib
    return _lib


def set_threads(n: int = 0) -> int:
    """Threads of the oracle's plane loops (n > 0 sets them); returns the
    count in use.  Results do not depend on it."""
    return int(_load().orc_set_threads(int(n)))


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _dpp(arrs):
    arr = (C.POINTER(C.c_double) * len(arrs))(*[_dptr(a) for a in arrs])
    return arr


def to_dense(U: dict, n) -> list:
    """Public staggered layout -> oracle dense (nz+1, ny, nx) instance arrays."""
    nx, ny, nz = n
    out = []
    for name in FIELDS:
        a = np.zeros((nz + 1, ny, nx))
        src = np.asarray(U[name], dtype=np.float64)
        if name in ("rho", "rhotheta"):
            a[:nz] = src
        elif name == "rhou":
            a[:nz] = src[:, :, :nx]
        elif name == "rhov":
            a[:nz] = src[:, :ny, :]
        else:
            a[:] = src
            a[0] = 0.0
            a[nz] = 0.0
        out.append(np.ascontiguousarray(a))
    return out


def from_dense(D: list, n) -> dict:
    nx, ny, nz = n
    U = {}
    for name, a in zip(FIELDS, D):
        if name in ("rho", "rhotheta"):
            U[name] = a[:nz].copy()
        elif name == "rhou":
            b = np.empty((nz, ny, nx + 1))
            b[:, :, :nx] = a[:nz]
            b[:, :, nx] = a[:nz, :, 0]
            U[name] = b
        elif name == "rhov":
            b = np.empty((nz, ny + 1, nx))
            b[:, :ny, :] = a[:nz]
            b[:, ny, :] = a[:nz, 0, :]
            U[name] = b
        else:
            b = a.copy()
            b[0] = 0.0
            b[nz] = 0.0
            U[name] = b
    return U


class Oracle:
    """Dense FP64 reference for one grid and terrain.

    grid: object with attributes n (nx, ny, nz), dx, lo, small_vfrac.
    limiter: 0 component-wise Barth-Jespersen (default), 1 scalar, 2 none.
    eb_flux: 0 no-flux wall (default), 1 free-stream closure test mode.
    """

    def __init__(self, grid, h_nodes: np.ndarray = None, limiter: int = 0, eb_flux: int = 0,
                 phi_nodes: np.ndarray = None, merged: bool = False):
        """Exactly one of h_nodes (terrain heights, (ny+1, nx+1)) and
        phi_nodes (level set, (nz+1, ny+1, nx+1), nondecreasing in z).  With
        merged=True they are the nodes of the grid refined by 2, and the
        geometry of `grid` is merged from the fine cells (Section 4.3)."""
        lib = _load()
        if (h_nodes is None) == (phi_nodes is None):
            raise ValueError("give exactly one of h_nodes and phi_nodes")
        self.n = tuple(int(v) for v in grid.n)
        nx, ny, nz = self.n
        if min(nx, ny) < 6 or nz < 2:
            raise ValueError("grid too small")
        self.g = _Grid((C.c_int32 * 3)(*self.n), (C.c_double * 3)(*grid.dx),
                       (C.c_double * 3)(*grid.lo), float(grid.small_vfrac), limiter, eb_flux)
        self.dx = tuple(float(v) for v in grid.dx)
        self.NI = (nz + 1) * ny * nx
        shape = (OQ_N, nz + 1, ny, nx)
        self.geo = [np.zeros(shape) for _ in range(4)]
        self.ctype = [np.zeros((nz + 1, ny, nx), dtype=np.int8) for _ in range(4)]
        i8 = (C.POINTER(C.c_int8) * 4)(*[c.ctypes.data_as(C.POINTER(C.c_int8)) for c in self.ctype])
        if merged:
            self.h = None
            kind = 0 if h_nodes is not None else 1
            self.fine_nodes = np.ascontiguousarray(h_nodes if kind == 0 else phi_nodes, dtype=np.float64)
            want = (2 * ny + 1, 2 * nx + 1) if kind == 0 else (2 * nz + 1, 2 * ny + 1, 2 * nx + 1)
            assert self.fine_nodes.shape == want
            if lib.orc_geometry_merged(C.byref(self.g), _dptr(self.fine_nodes), kind, _dpp(self.geo), i8) != 0:
                raise ValueError("level set not nondecreasing along z")
        elif h_nodes is not None:
            self.h = np.ascontiguousarray(h_nodes, dtype=np.float64)
            assert self.h.shape == (ny + 1, nx + 1)
            lib.orc_geometry(C.byref(self.g), _dptr(self.h), _dpp(self.geo), i8)
        else:
            self.h = None
            self.phi = np.ascontiguousarray(phi_nodes, dtype=np.float64)
            assert self.phi.shape == (nz + 1, ny + 1, nx + 1)
            if lib.orc_geometry_levelset(C.byref(self.g), _dptr(self.phi), _dpp(self.geo), i8) != 0:
                raise ValueError("level set not nondecreasing along z")
        self.w = [np.zeros((OW_N, nz + 1, ny, nx)) for _ in range(4)]
        lib.orc_wsrd_setup(C.byref(self.g), _dpp(self.geo), _dpp(self.w))

    # --------------------------------------------------------------- helpers
    def alpha(self, inst: int) -> np.ndarray:
        return self.geo[inst][OQ["ALPHA"]]

    def volume(self, inst: int) -> np.ndarray:
        """Fluid volume of every CV (0 where not a CV)."""
        return self.alpha(inst) * (self.dx[0] * self.dx[1] * self.dx[2])

    def set_mode(self, limiter: int = None, eb_flux: int = None):
        if limiter is not None:
            self.g.limiter = limiter
        if eb_flux is not None:
            self.g.eb_flux = eb_flux

    # ------------------------------------------------------------- operators
    def sources_dense(self, Ucur: list, ref) -> list:
        """Momentum sources (perturbation pressure gradient, buoyancy) of a
        dense state for the reference state ``ref`` (attributes P00, R,
        gamma, g, rhotheta0[nz], rho0[nz]): three dense arrays, instances 1-3."""
        nz = self.n[2]
        p0 = np.ascontiguousarray(ref.rhotheta0, dtype=np.float64)
        r0 = np.ascontiguousarray(ref.rho0, dtype=np.float64)
        assert p0.shape == (nz,) and r0.shape == (nz,)
        S = [np.zeros_like(Ucur[0]) for _ in range(3)]
        prm = _Src(float(ref.P00), float(ref.R), float(ref.gamma), float(ref.g))
        _load().orc_sources(C.byref(self.g), _dpp(self.geo), _dpp(Ucur), C.byref(prm), _dptr(p0),
                            _dptr(r0), _dpp(S))
        return S

    def sources(self, U: dict, ref) -> dict:
        """Intensive momentum sources in the public layout (rhou, rhov, rhow)."""
        S = self.sources_dense(to_dense(U, self.n), ref)
        zero = [np.zeros_like(S[0]), np.zeros_like(S[0])]
        out = from_dense(zero + S, self.n)
        return {k: out[k] for k in ("rhou", "rhov", "rhow")}

    def diffusion_dense(self, Ucur: list, diff, fluxes: bool = False):
        """Intensive diffusive update of rho theta (dense, instance 0) for
        ``diff`` (attributes alpha_theta, eb_mode, theta_wall); with fluxes,
        also the lower-face flux densities [3] and the EB terms."""
        p = _Diff(float(diff.alpha_theta), int(diff.eb_mode), float(diff.theta_wall))
        D = np.zeros_like(Ucur[0])
        F = [np.zeros_like(Ucur[0]) for _ in range(3)]
        E = np.zeros_like(Ucur[0])
        _load().orc_diffusion(C.byref(self.g), _dpp(self.geo), _dpp(Ucur), C.byref(p), _dptr(D), _dpp(F),
                              _dptr(E))
        return (D, F, E) if fluxes else D

    def diffusion(self, U: dict, diff, fluxes: bool = False):
        return self.diffusion_dense(to_dense(U, self.n), diff, fluxes)

    def viscous_dense(self, Ucur: list, visc, fluxes: bool = False):
        """Intensive viscous update of the three momenta (dense, instances
        1-3) for ``visc`` (attributes mu, eb_mode); with fluxes, also the
        stresses on the lower faces [3 c + d] and the EB terms [c]."""
        p = _Visc(float(visc.mu), int(visc.eb_mode))
        D = [np.zeros_like(Ucur[0]) for _ in range(3)]
        F = [np.zeros_like(Ucur[0]) for _ in range(9)]
        E = [np.zeros_like(Ucur[0]) for _ in range(3)]
        _load().orc_viscous(C.byref(self.g), _dpp(self.geo), _dpp(Ucur), C.byref(p), _dpp(D), _dpp(F), _dpp(E))
        return (D, F, E) if fluxes else D

    def viscous(self, U: dict, visc, fluxes: bool = False):
        return self.viscous_dense(to_dense(U, self.n), visc, fluxes)

    def advance_dense(self, Un: list, Ucur: list, cdt: float, ref=None, diff=None, visc=None) -> list:
        """Uhat = Un + cdt dU(Ucur); with a reference state, plus cdt times the
        momentum sources of Ucur on every fluid CV; with a diffusion setting,
        plus cdt times the diffusive update of rho theta; with a viscosity
        setting, plus cdt times the viscous update of the momenta."""
        out = [np.zeros_like(Un[0]) for _ in range(5)]
        _load().orc_advance(C.byref(self.g), _dpp(self.geo), _dpp(Un), _dpp(Ucur), _dpp(out),
                            float(cdt))
        if ref is not None:
            S = self.sources_dense(Ucur, ref)
            for d in range(3):
                out[2 + d] = out[2 + d] + float(cdt) * S[d]
        if diff is not None:
            out[1] = out[1] + float(cdt) * self.diffusion_dense(Ucur, diff)
        if visc is not None:
            V = self.viscous_dense(Ucur, visc)
            for cc in range(3):
                out[2 + cc] = out[2 + cc] + float(cdt) * V[cc]
        return out

    def redistribute_dense(self, Uhat: list) -> list:
        out = [np.zeros_like(Uhat[0]) for _ in range(5)]
        _load().orc_redistribute(C.byref(self.g), _dpp(self.geo), _dpp(self.w), _dpp(Uhat),
                                 _dpp(out))
        return out

    def redistribute_sig(self, Uhat: dict):
        """Redistribution plus the limited gradient sigma of every CV
        (shape (nz+1, ny, nx, 3) per field, dense instance storage)."""
        D = to_dense(Uhat, self.n)
        out = [np.zeros_like(D[0]) for _ in range(5)]
        sig = [np.zeros(D[0].shape + (3,)) for _ in range(5)]
        _load().orc_redistribute_sig(C.byref(self.g), _dpp(self.geo), _dpp(self.w), _dpp(D),
                                     _dpp(out), _dpp(sig))
        return from_dense(out, self.n), sig

    def redistribute_diag(self, Uhat: dict):
        """Redistribution plus, per field in dense instance storage, the
        limited gradient sigma (nz+1, ny, nx, 3; physical units) and Q-hat
        (nz+1, ny, nx) of every CV."""
        D = to_dense(Uhat, self.n)
        out = [np.zeros_like(D[0]) for _ in range(5)]
        sig = [np.zeros(D[0].shape + (3,)) for _ in range(5)]
        qh = [np.zeros_like(D[0]) for _ in range(5)]
        _load().orc_redistribute_diag(C.byref(self.g), _dpp(self.geo), _dpp(self.w), _dpp(D),
                                      _dpp(out), _dpp(sig), _dpp(qh))
        return from_dense(out, self.n), sig, qh

    def advance(self, Un: dict, Ucur: dict, cdt: float, ref=None, diff=None, visc=None) -> dict:
        return from_dense(self.advance_dense(to_dense(Un, self.n), to_dense(Ucur, self.n), cdt, ref, diff, visc),
                          self.n)

    def redistribute(self, Uhat: dict) -> dict:
        return from_dense(self.redistribute_dense(to_dense(Uhat, self.n)), self.n)

    def stage(self, Un: dict, Ucur: dict, cdt: float, ref=None, diff=None, visc=None) -> dict:
        """Algorithm 1 steps (1)-(4) for one stage: U^s = R(U^n + c dt dU(U^{s-1}))."""
        d_n = to_dense(Un, self.n)
        d_c = d_n if Ucur is Un else to_dense(Ucur, self.n)
        return from_dense(self.redistribute_dense(self.advance_dense(d_n, d_c, cdt, ref, diff, visc)), self.n)

    def rk3_step(self, U: dict, dt: float, ref=None, diff=None, visc=None) -> dict:
        """Low-storage three-stage Runge-Kutta (Wicker-Skamarock form)."""
        d_n = to_dense(U, self.n)
        cur = d_n
        for c in RK3_C:
            cur = self.redistribute_dense(self.advance_dense(d_n, cur, c * dt, ref, diff, visc))
        return from_dense(cur, self.n)

    # ------------------------------------------------------------ two levels
    def coarsened_geometry(self):
        """alpha and lower-face area fractions (x, y, z) of the grid coarsened
        by 2, each (nz/2, ny/2, nx/2)."""
        nx, ny, nz = self.n
        sh = (nz // 2, ny // 2, nx // 2)
        a = np.zeros(sh)
        b = [np.zeros(sh) for _ in range(3)]
        if _load().orc_coarsen_geometry(C.byref(self.g), _dpp(self.geo), _dptr(a), _dpp(b)) != 0:
            raise ValueError("odd grid size")
        return a, b

    def restrict(self, U: dict) -> dict:
        """Restriction of a fine state onto the grid coarsened by 2 (public layout)."""
        nx, ny, nz = self.n
        D = to_dense(U, self.n)
        cn = (nx // 2, ny // 2, nz // 2)
        out = [np.zeros((cn[2] + 1, cn[1], cn[0])) for _ in range(5)]
        if _load().orc_restrict(C.byref(self.g), _dpp(self.geo), _dpp(D), _dpp(out)) != 0:
            raise ValueError("odd grid size")
        return from_dense(out, cn)

    def face_fluxes(self, U: dict, field: int):
        F = [np.zeros(self.NI).reshape(self.n[2] + 1, self.n[1], self.n[0]) for _ in range(3)]
        Fh = [np.zeros_like(F[0]) for _ in range(3)]
        D = to_dense(U, self.n)  # keep the arrays alive across the call
        _load().orc_face_fluxes(C.byref(self.g), _dpp(self.geo), _dpp(D), int(field), _dpp(F),
                                _dpp(Fh))
        return F, Fh

    def conserved_sums(self, U: dict) -> list:
        """Sum of V * U over the fluid CVs of each field, exactly rounded."""
        D = to_dense(U, self.n)
        out = []
        for f, inst in enumerate(FIELD_INST):
            v = self.volume(inst) * D[f]
            out.append(math.fsum(v.ravel().tolist()))
        return out

    def export(self, inst: int, q: int) -> np.ndarray:
        """Geometry quantity in the public staggered layout of the instance."""
        return _inst_to_public(self.geo[inst][q], inst, self.n)

    def export_w(self, inst: int, q: int) -> np.ndarray:
        return _inst_to_public(self.w[inst][q], inst, self.n)

    def export_type(self, inst: int) -> np.ndarray:
        return _inst_to_public(self.ctype[inst].astype(np.float64), inst, self.n)


def _inst_to_public(a: np.ndarray, inst: int, n) -> np.ndarray:
    nx, ny, nz = n
    if inst == 0:
        return a[:nz].copy()
    if inst == 1:
        b = np.empty((nz, ny, nx + 1))
        b[:, :, :nx] = a[:nz]
        b[:, :, nx] = a[:nz, :, 0]
        return b
    if inst == 2:
        b = np.empty((nz, ny + 1, nx))
        b[:, :ny] = a[:nz]
        b[:, ny] = a[:nz, 0]
        return b
    b = a.copy()
    b[0] = 0.0
    b[nz] = 0.0
    return b


def box_moments(grid, h_nodes, ci, cj, rect, za, zb, bottom=False) -> np.ndarray:
    """Clipped moments of one box (tests of the clipper against closed forms)."""
    lib = _load()
    nx, ny, nz = grid.n
    g = _Grid((C.c_int32 * 3)(*grid.n), (C.c_double * 3)(*grid.dx), (C.c_double * 3)(*grid.lo),
              0.5, 0, 0)
    h = np.ascontiguousarray(h_nodes, dtype=np.float64)
    r = np.ascontiguousarray(rect, dtype=np.float64)
    out = np.zeros(14)
    lib.orc_box_moments(C.byref(g), _dptr(h), int(ci), int(cj), _dptr(r), float(za), float(zb),
                        int(bottom), _dptr(out))
    return out


def levelset_piece(grid, phi_nodes, i, j, k, part) -> np.ndarray:
    """[vol, mx, my, mz, EB area vector (3), EB area, 6 face areas, type] of
    box piece `part` of cell (i, j, k) for a level set (moments relative to
    the cell's lower node)."""
    lib = _load()
    g = _Grid((C.c_int32 * 3)(*[int(v) for v in grid.n]), (C.c_double * 3)(*grid.dx),
              (C.c_double * 3)(*grid.lo), float(grid.small_vfrac), 0, 0)
    phi = np.ascontiguousarray(phi_nodes, dtype=np.float64)
    out = np.zeros(15)
    lib.orc_levelset_piece(C.byref(g), _dptr(phi), int(i), int(j), int(k), int(part), _dptr(out))
    return out
