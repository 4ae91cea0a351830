"""Python binding of libebstag (the C ABI declared in include/ebstag.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory and the stream.  Importing this package loads
the in-tree ``libebstag.so``; it raises if the library is missing (build it
with ``python -m paper_2604_11959_amd.build``) - there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libebstag.so")

FIELDS = ("rho", "rhotheta", "rhou", "rhov", "rhow")

EBS_OK, EBS_E_ARG, EBS_E_OOM, EBS_E_HIP, EBS_E_ORDER, EBS_E_UNSUPPORTED = range(6)
EBS_F64, EBS_F32_BULK = 0, 1
EBS_EB_WALL, EBS_EB_FREESTREAM = 0, 1
EBS_LIM_BJ_COMPONENT, EBS_LIM_BJ_SCALAR, EBS_LIM_NONE = 0, 1, 2

# export quantities (EBS_Q_*)
Q = dict(ALPHA=0, BETA_X=1, BETA_Y=2, BETA_Z=3, FX_Y=4, FX_Z=5, FY_X=6, FY_Z=7, FZ_X=8, FZ_Y=9,
         VC_X=10, VC_Y=11, VC_Z=12, A_X=13, A_Y=14, A_Z=15, AREA=16, EBC_X=17, EBC_Y=18, EBC_Z=19,
         TYPE=20, SMALL=21, TIER=22, MASK=23, NCOUNT=24, KAPPA=25, OMEGA=26, VHAT=27,
         XHAT_X=28, XHAT_Y=29, XHAT_Z=30)

# every entry point declared in include/ebstag.h
SYMBOLS = ("ebs_create", "ebs_build_geometry_terrain", "ebs_build_geometry_levelset", "ebs_build_geometry_merged", "ebs_geometry_export", "ebs_geometry_stats", "ebs_alpha_histogram",
           "ebs_advance_stage", "ebs_redistribute", "ebs_rk3_step", "ebs_conserved_sums",
           "ebs_autotune", "ebs_set_tile", "ebs_get_tile", "ebs_set_overlap", "ebs_set_persistent", "ebs_set_range_rule", "ebs_set_sources", "ebs_set_diffusion", "ebs_set_viscosity", "ebs_restrict", "ebs_coarsened_geometry", "ebs_coarsened_geometry_noalloc", "ebs_timing_enable", "ebs_timing_read",
           "ebs_algorithmic_bytes", "ebs_stream_copy", "ebs_last_error", "ebs_destroy")


class EbsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"ebstag status {status}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("dx", C.c_double * 3), ("lo", C.c_double * 3),
                ("periodic", C.c_uint32), ("small_vfrac", C.c_double), ("precision", C.c_int32),
                ("limiter", C.c_int32), ("eb_flux", C.c_int32)]


class Box(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3)]


class SourceParams(C.Structure):
    _fields_ = [("P00", C.c_double), ("R", C.c_double), ("gamma", C.c_double), ("g", C.c_double)]


class DiffusionParams(C.Structure):
    _fields_ = [("alpha_theta", C.c_double), ("eb_mode", C.c_int32), ("theta_wall", C.c_double)]


class ViscosityParams(C.Structure):
    _fields_ = [("mu", C.c_double), ("eb_mode", C.c_int32)]


class State(C.Structure):
    _fields_ = [(name, C.c_void_p) for name in FIELDS]


_lib = None


def load(path: str = LIB_PATH):
    """Load libebstag.so (raises OSError if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} not found: build it with `python -m paper_2604_11959_amd.build`")
    # PyTorch ships its own HIP runtime; loading it first makes the library
    # bind to that one, so streams and device pointers from torch are valid
    # in the library (a second runtime would reject them)
    import torch  # noqa: F401

    lib = C.CDLL(path)
    P = C.POINTER
    st = C.c_int
    sig = {
        "ebs_create": [P(Grid), P(Box), C.c_int32, C.c_void_p, P(C.c_void_p)],
        "ebs_build_geometry_terrain": [C.c_void_p, P(C.c_double), C.c_int32],
        "ebs_build_geometry_levelset": [C.c_void_p, P(C.c_double), C.c_int32],
        "ebs_build_geometry_merged": [C.c_void_p, P(C.c_double), C.c_int32, C.c_int32],
        "ebs_geometry_export": [C.c_void_p, C.c_int32, C.c_int32, P(C.c_double), C.c_size_t],
        "ebs_geometry_stats": [C.c_void_p, P(C.c_int64)],
        "ebs_alpha_histogram": [C.c_void_p, C.c_int32, P(C.c_double), C.c_int32, P(C.c_int64)],
        "ebs_advance_stage": [C.c_void_p, P(State), P(State), P(State), C.c_double],
        "ebs_redistribute": [C.c_void_p, P(State), P(State)],
        "ebs_rk3_step": [C.c_void_p, P(State), P(State), C.c_double, C.c_int32],
        "ebs_conserved_sums": [C.c_void_p, P(State), P(C.c_double), P(C.c_double)],
        "ebs_autotune": [C.c_void_p, C.c_char_p],
        "ebs_set_tile": [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32],
        "ebs_get_tile": [C.c_void_p, P(C.c_int32), P(C.c_int32), P(C.c_int32), P(C.c_int32)],
        "ebs_set_overlap": [C.c_void_p, C.c_int32],
        "ebs_set_persistent": [C.c_void_p, C.c_int32],
        "ebs_set_range_rule": [C.c_void_p, C.c_int32],
        "ebs_set_sources": [C.c_void_p, P(SourceParams), P(C.c_double), P(C.c_double)],
        "ebs_set_diffusion": [C.c_void_p, P(DiffusionParams)],
        "ebs_set_viscosity": [C.c_void_p, P(ViscosityParams)],
        "ebs_restrict": [C.c_void_p, P(State), P(State)],
        "ebs_coarsened_geometry": [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_double), P(C.c_double)],
        "ebs_coarsened_geometry_noalloc": [C.c_void_p, P(C.c_double), P(C.c_double), P(C.c_double),
                                           P(C.c_double)],
        "ebs_timing_enable": [C.c_void_p, C.c_int32],
        "ebs_timing_read": [C.c_void_p, P(C.c_double), P(C.c_int64)],
        "ebs_algorithmic_bytes": [C.c_void_p, P(C.c_double)],
        "ebs_destroy": [C.c_void_p],
        "ebs_stream_copy": [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = st
    lib.ebs_last_error.argtypes = [C.c_void_p]
    lib.ebs_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def stream_copy(dst, src, stream=None):
    """Copy device tensor src into dst (same byte size) with the library's
    streaming copy kernel on the given (default: current) stream."""
    import torch

    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("sizes differ")
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    st = load().ebs_stream_copy(C.c_void_p(dst.data_ptr()), C.c_void_p(src.data_ptr()), nbytes, C.c_void_p(stream))
    if st != EBS_OK:
        raise EbsError(st, "ebs_stream_copy")


def field_shapes(n):
    nx, ny, nz = n
    return {"rho": (nz, ny, nx), "rhotheta": (nz, ny, nx), "rhou": (nz, ny, nx + 1),
            "rhov": (nz, ny + 1, nx), "rhow": (nz + 1, ny, nx)}


def export_shape(n, inst):
    nx, ny, nz = n
    return [(nz, ny, nx), (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)][inst]


def as_state(U: dict) -> State:
    """ebs_state from a dict of contiguous device tensors."""
    for name in FIELDS:
        t = U[name]
        if not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"{name} must be a contiguous device tensor")
    return State(*[U[name].data_ptr() for name in FIELDS])


class Context:
    """One grid + terrain + box list on the current device and stream."""

    def __init__(self, n, dx, lo=(0.0, 0.0, 0.0), boxes=None, precision=EBS_F64,
                 limiter=EBS_LIM_BJ_COMPONENT, eb_flux=EBS_EB_WALL, small_vfrac=0.5, stream=None):
        import torch

        self.lib = load()
        self.n = tuple(int(v) for v in n)
        self.precision = precision
        self.dtype = torch.float64 if precision == EBS_F64 else torch.float32
        g = Grid((C.c_int32 * 3)(*self.n), (C.c_double * 3)(*dx), (C.c_double * 3)(*lo), 0x3,
                 float(small_vfrac), int(precision), int(limiter), int(eb_flux))
        self.grid = g
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        nb = 0
        barr = None
        if boxes:
            nb = len(boxes)
            barr = (Box * nb)(*[Box((C.c_int32 * 3)(*lo_), (C.c_int32 * 3)(*hi_)) for lo_, hi_ in boxes])
        h = C.c_void_p()
        st = self.lib.ebs_create(C.byref(g), barr, nb, C.c_void_p(stream), C.byref(h))
        if st != EBS_OK:
            raise EbsError(st, "ebs_create failed")
        self.h = h

    def _check(self, st: int, what: str):
        if st != EBS_OK:
            msg = self.lib.ebs_last_error(self.h).decode()
            raise EbsError(st, f"{what}: {msg}")

    def close(self):
        if getattr(self, "h", None):
            self.lib.ebs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- geometry
    def build_geometry(self, h_nodes):
        import numpy as np

        h = np.ascontiguousarray(h_nodes, dtype=np.float64)
        self._check(self.lib.ebs_build_geometry_terrain(
            self.h, h.ctypes.data_as(C.POINTER(C.c_double)), 0), "ebs_build_geometry_terrain")

    def build_geometry_levelset(self, phi_nodes):
        """phi_nodes: (nz+1, ny+1, nx+1) nodal level set, nondecreasing in z."""
        import numpy as np

        f = np.ascontiguousarray(phi_nodes, dtype=np.float64)
        nx, ny, nz = self.n
        if f.shape != (nz + 1, ny + 1, nx + 1):
            raise ValueError(f"phi_nodes must have shape {(nz + 1, ny + 1, nx + 1)}")
        self._check(self.lib.ebs_build_geometry_levelset(
            self.h, f.ctypes.data_as(C.POINTER(C.c_double)), 0), "ebs_build_geometry_levelset")

    def build_geometry_merged(self, fine_nodes):
        """Geometry merged from the grid refined by 2: fine terrain heights
        (2ny+1, 2nx+1) or a fine level set (2nz+1, 2ny+1, 2nx+1)."""
        import numpy as np

        f = np.ascontiguousarray(fine_nodes, dtype=np.float64)
        nx, ny, nz = self.n
        kind = 0 if f.ndim == 2 else 1
        want = (2 * ny + 1, 2 * nx + 1) if kind == 0 else (2 * nz + 1, 2 * ny + 1, 2 * nx + 1)
        if f.shape != want:
            raise ValueError(f"fine nodes must have shape {want}")
        self._check(self.lib.ebs_build_geometry_merged(
            self.h, f.ctypes.data_as(C.POINTER(C.c_double)), kind, 0), "ebs_build_geometry_merged")

    def export(self, inst: int, qty: int):
        import numpy as np

        shape = export_shape(self.n, inst)
        out = np.zeros(shape)
        self._check(self.lib.ebs_geometry_export(self.h, int(inst), int(qty),
                                                 out.ctypes.data_as(C.POINTER(C.c_double)), out.size),
                    "ebs_geometry_export")
        return out

    def stats(self):
        import numpy as np

        out = np.zeros(32, dtype=np.int64)
        self._check(self.lib.ebs_geometry_stats(self.h, out.ctypes.data_as(C.POINTER(C.c_int64))),
                    "ebs_geometry_stats")
        return out.reshape(4, 8)

    def alpha_histogram(self, inst: int, edges):
        """Counts of the fluid CVs of an instance per volume-fraction bin
        [edges[b], edges[b+1]) (last bin closed)."""
        import numpy as np

        e = np.ascontiguousarray(edges, dtype=np.float64)
        out = np.zeros(len(e) - 1, dtype=np.int64)
        self._check(self.lib.ebs_alpha_histogram(self.h, int(inst), e.ctypes.data_as(C.POINTER(C.c_double)),
                                                 len(e) - 1, out.ctypes.data_as(C.POINTER(C.c_int64))),
                    "ebs_alpha_histogram")
        return out

    # ---------------------------------------------------------------- state
    def new_state(self, host: dict | None = None):
        import torch

        sh = field_shapes(self.n)
        if host is None:
            return {k: torch.zeros(sh[k], dtype=self.dtype, device="cuda") for k in FIELDS}
        return {k: torch.as_tensor(host[k], dtype=torch.float64).to(self.dtype).to("cuda").contiguous()
                for k in FIELDS}

    def advance(self, Un: dict, Ucur: dict, Uhat: dict, cdt: float):
        a, b, c = as_state(Un), as_state(Ucur), as_state(Uhat)
        self._check(self.lib.ebs_advance_stage(self.h, C.byref(a), C.byref(b), C.byref(c), float(cdt)),
                    "ebs_advance_stage")

    def restrict(self, U: dict, out: dict | None = None) -> dict:
        """Restriction onto the grid coarsened by 2 (new device state unless
        ``out`` is given)."""
        import torch

        cn = tuple(v // 2 for v in self.n)
        if out is None:
            sh = field_shapes(cn)
            out = {k: torch.empty(sh[k], dtype=self.dtype, device="cuda") for k in FIELDS}
        a, b = as_state(U), as_state(out)
        self._check(self.lib.ebs_restrict(self.h, C.byref(a), C.byref(b)), "ebs_restrict")
        return out

    def coarsened_geometry(self, noalloc: bool = False):
        """(alpha, [beta_x, beta_y, beta_z]) of the grid coarsened by 2, each
        (nz/2, ny/2, nx/2), on the host; noalloc selects the entry point that
        stages through the library's fixed device buffer."""
        import numpy as np

        nx, ny, nz = self.n
        sh = (nz // 2, ny // 2, nx // 2)
        arrs = [np.zeros(sh) for _ in range(4)]
        dp = C.POINTER(C.c_double)
        fn = self.lib.ebs_coarsened_geometry_noalloc if noalloc else self.lib.ebs_coarsened_geometry
        self._check(fn(self.h, *[x.ctypes.data_as(dp) for x in arrs]), "ebs_coarsened_geometry")
        return arrs[0], arrs[1:]

    def redistribute(self, Uhat: dict, Uout: dict):
        a, b = as_state(Uhat), as_state(Uout)
        self._check(self.lib.ebs_redistribute(self.h, C.byref(a), C.byref(b)), "ebs_redistribute")

    def rk3_step(self, U: dict, scratch: list, dt: float, use_graph: bool = False):
        u = as_state(U)
        s = (State * 2)(as_state(scratch[0]), as_state(scratch[1]))
        self._check(self.lib.ebs_rk3_step(self.h, C.byref(u), s, float(dt), int(use_graph)),
                    "ebs_rk3_step")

    def conserved_sums(self, U: dict):
        hi = (C.c_double * 5)()
        lo = (C.c_double * 5)()
        self._check(self.lib.ebs_conserved_sums(self.h, C.byref(as_state(U)), hi, lo),
                    "ebs_conserved_sums")
        return list(hi), list(lo)

    # --------------------------------------------------------------- tuning
    def autotune(self, cache_path: str | None = None):
        p = cache_path.encode() if cache_path else None
        self._check(self.lib.ebs_autotune(self.h, p), "ebs_autotune")
        return self.get_tile()

    def set_tile(self, tx: int, ty: int, tz: int = 0, span: int = 0):
        """Tile of the regular-region kernel: tx x ty columns, tz planes (0 keeps
        it); span 1 tiles the whole domain instead of each box."""
        self._check(self.lib.ebs_set_tile(self.h, int(tx), int(ty), int(tz), int(span)), "ebs_set_tile")

    def set_overlap(self, enable: bool):
        """Regular-region kernel concurrent with the general range (True) or serial (default)."""
        self._check(self.lib.ebs_set_overlap(self.h, int(bool(enable))), "ebs_set_overlap")

    def set_persistent(self, enable: bool):
        """Regular-region kernel with a grid of resident blocks walking the tile
        list (True) or one block per tile (False, default)."""
        self._check(self.lib.ebs_set_persistent(self.h, int(bool(enable))), "ebs_set_persistent")

    def set_range_rule(self, rule: int):
        """Rule for the top of the general range used by the next geometry build:
        0 loose, 1 small-CV footprint, 2 (default) the cells the redistribution
        touches."""
        self._check(self.lib.ebs_set_range_rule(self.h, int(rule)), "ebs_set_range_rule")

    def set_sources(self, ref=None):
        """Switch the momentum sources (perturbation pressure gradient and
        buoyancy) on for a reference state ``ref`` with attributes P00, R,
        gamma, g and per-level arrays rhotheta0, rho0 (nz values each), or off
        with None."""
        import numpy as np

        if ref is None:
            self._check(self.lib.ebs_set_sources(self.h, None, None, None), "ebs_set_sources")
            return
        p0 = np.ascontiguousarray(ref.rhotheta0, dtype=np.float64)
        r0 = np.ascontiguousarray(ref.rho0, dtype=np.float64)
        if p0.shape != (self.n[2],) or r0.shape != (self.n[2],):
            raise ValueError("p0 and rho0 need one value per level")
        prm = SourceParams(float(ref.P00), float(ref.R), float(ref.gamma), float(ref.g))
        dp = C.POINTER(C.c_double)
        self._check(self.lib.ebs_set_sources(self.h, C.byref(prm), p0.ctypes.data_as(dp), r0.ctypes.data_as(dp)),
                    "ebs_set_sources")

    def set_diffusion(self, p=None):
        """Thermal diffusion of rho theta with parameters ``p`` (attributes
        alpha_theta, eb_mode, theta_wall), or off with None."""
        if p is None:
            self._check(self.lib.ebs_set_diffusion(self.h, None), "ebs_set_diffusion")
            return
        prm = DiffusionParams(float(p.alpha_theta), int(p.eb_mode), float(p.theta_wall))
        self._check(self.lib.ebs_set_diffusion(self.h, C.byref(prm)), "ebs_set_diffusion")

    def set_viscosity(self, p=None):
        """Momentum diffusion with parameters ``p`` (attributes mu, eb_mode),
        or off with None."""
        if p is None:
            self._check(self.lib.ebs_set_viscosity(self.h, None), "ebs_set_viscosity")
            return
        prm = ViscosityParams(float(p.mu), int(p.eb_mode))
        self._check(self.lib.ebs_set_viscosity(self.h, C.byref(prm)), "ebs_set_viscosity")

    def get_tile(self):
        tx, ty, tz, sp = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        self._check(self.lib.ebs_get_tile(self.h, C.byref(tx), C.byref(ty), C.byref(tz), C.byref(sp)),
                    "ebs_get_tile")
        return tx.value, ty.value, tz.value, sp.value

    def timing(self, enable: bool):
        self._check(self.lib.ebs_timing_enable(self.h, int(enable)), "ebs_timing_enable")

    def timing_read(self):
        ms = C.c_double()
        n = C.c_int64()
        self._check(self.lib.ebs_timing_read(self.h, C.byref(ms), C.byref(n)), "ebs_timing_read")
        return ms.value, n.value

    def algorithmic_bytes(self):
        out = (C.c_double * 2)()
        self._check(self.lib.ebs_algorithmic_bytes(self.h, out), "ebs_algorithmic_bytes")
        return out[0], out[1]
