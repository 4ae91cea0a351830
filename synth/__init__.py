"""Seeded synthetic inputs for the staggered cut-cell update.

This module is the only code shared by the FP64 oracle tests and the HIP path:
it produces terrain heights on grid nodes, initial states and box lists.  It
contains input recipes only -- none of the method's arithmetic (no geometry,
no fluxes, no redistribution).

The workloads stand in for the paper's experiments, which need full physics
and datasets that are not part of this hot path.  They reuse the paper's
terrain form (Witch of Agnesi hill, Section 6.1) and CFL number 0.5
(Sections 6.1, 6.3).

Layout conventions (x fastest, C order arrays):
    h_nodes  (ny+1, nx+1) float64   terrain height at node (X_i, Y_j)
    rho, rhotheta  (nz, ny, nx)
    rhou  (nz, ny, nx+1)    face nx duplicates face 0 (periodic x)
    rhov  (nz, ny+1, nx)    face ny duplicates face 0 (periodic y)
    rhow  (nz+1, ny, nx)    faces 0 and nz are the bottom / top walls (0)

Entries under the terrain are drawn like every other entry (so the draw
sequence does not depend on geometry); the method ignores them.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FIELDS = ("rho", "rhotheta", "rhou", "rhov", "rhow")


@dataclass
class Grid:
    n: tuple          # (nx, ny, nz)
    dx: tuple         # (dx, dy, dz) in metres (or unit lengths)
    lo: tuple = (0.0, 0.0, 0.0)
    small_vfrac: float = 0.5

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def length(self):
        return tuple(self.n[d] * self.dx[d] for d in range(3))


@dataclass
class Workload:
    name: str
    grid: Grid
    h_nodes: np.ndarray
    dt: float
    seed: int
    boxes: list = field(default_factory=list)   # [(lo3, hi3)], half-open cell ranges
    state_kind: str = "c1"
    terrain_note: str = ""
    phi_nodes: np.ndarray = None  # level-set workloads: (nz+1, ny+1, nx+1) nodal values


def field_shapes(n):
    nx, ny, nz = n
    return {
        "rho": (nz, ny, nx),
        "rhotheta": (nz, ny, nx),
        "rhou": (nz, ny, nx + 1),
        "rhov": (nz, ny + 1, nx),
        "rhow": (nz + 1, ny, nx),
    }


def node_coords(grid: Grid):
    nx, ny, _ = grid.n
    x = grid.lo[0] + np.arange(nx + 1, dtype=np.float64) * grid.dx[0]
    y = grid.lo[1] + np.arange(ny + 1, dtype=np.float64) * grid.dx[1]
    return x, y


def cfl_dt(grid: Grid, speed: float = 10.0, cfl: float = 0.5) -> float:
    """Fixed time step at CFL 0.5 for the background wind (computed once)."""
    return cfl * min(grid.dx) / speed


def _periodic_fix(h: np.ndarray) -> np.ndarray:
    """Make the last node row/column equal the first (periodic x and y)."""
    h[:, -1] = h[:, 0]
    h[-1, :] = h[0, :]
    return h


def _min_image(d: np.ndarray, L: float) -> np.ndarray:
    return d - L * np.round(d / L)


# --------------------------------------------------------------------- terrains

def terrain_gaussian_unit(grid: Grid) -> np.ndarray:
    """h = 0.3 exp(-((x-.5)^2 + (y-.5)^2) / 0.15^2), untruncated."""
    x, y = node_coords(grid)
    X, Y = np.meshgrid(x, y)
    h = 0.3 * np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.15 ** 2)
    return _periodic_fix(h)


def terrain_agnesi(grid: Grid, h0=400.0, a=1000.0, centre=None) -> np.ndarray:
    """3-D Witch of Agnesi: the paper's 2-D profile h0 / (1 + (x/a)^2) rotated
    about the hill centre (Section 6.1)."""
    x, y = node_coords(grid)
    Lx, Ly, _ = grid.length
    cx, cy = centre if centre is not None else (grid.lo[0] + Lx / 2, grid.lo[1] + Ly / 2)
    X, Y = np.meshgrid(x, y)
    r2 = (X - cx) ** 2 + (Y - cy) ** 2
    h = h0 / (1.0 + r2 / a ** 2)
    return _periodic_fix(h)


def terrain_gaussian_hills(grid: Grid, seed: int, k_hills: int,
                           hrange=(100.0, 600.0), wrange=(500.0, 2000.0)) -> np.ndarray:
    """Sum of seeded Gaussian hills H exp(-r^2/w^2) with periodic minimum-image
    r, each zeroed where r > 4w so that flat ground is exactly h = 0."""
    rng = np.random.default_rng(seed)
    H = rng.uniform(hrange[0], hrange[1], k_hills)
    W = rng.uniform(wrange[0], wrange[1], k_hills)
    Lx, Ly, _ = grid.length
    cx = grid.lo[0] + rng.uniform(0.0, Lx, k_hills)
    cy = grid.lo[1] + rng.uniform(0.0, Ly, k_hills)
    x, y = node_coords(grid)
    X, Y = np.meshgrid(x, y)
    h = np.zeros_like(X)
    for q in range(k_hills):
        dx = _min_image(X - cx[q], Lx)
        dy = _min_image(Y - cy[q], Ly)
        r2 = dx * dx + dy * dy
        bump = H[q] * np.exp(-r2 / W[q] ** 2)
        bump[r2 > (4.0 * W[q]) ** 2] = 0.0
        h += bump
    return _periodic_fix(h)


def terrain_ridges(grid: Grid, seed: int, n_ridges: int = 24) -> np.ndarray:
    """Seeded hipped-roof ridges with slopes up to 60 degrees, combined by max
    (so the combined slope never exceeds 60 degrees), periodic min-image."""
    rng = np.random.default_rng(seed)
    H = rng.uniform(200.0, 1500.0, n_ridges)
    slope = np.deg2rad(rng.uniform(30.0, 60.0, n_ridges))
    Lr = rng.uniform(5000.0, 20000.0, n_ridges)
    ang = rng.uniform(0.0, math.pi, n_ridges)
    Lx, Ly, _ = grid.length
    cx = grid.lo[0] + rng.uniform(0.0, Lx, n_ridges)
    cy = grid.lo[1] + rng.uniform(0.0, Ly, n_ridges)
    x, y = node_coords(grid)
    X, Y = np.meshgrid(x, y)
    h = np.zeros_like(X)
    for q in range(n_ridges):
        W = H[q] / math.tan(slope[q])
        dx = _min_image(X - cx[q], Lx)
        dy = _min_image(Y - cy[q], Ly)
        c, s = math.cos(ang[q]), math.sin(ang[q])
        dpar = dx * c + dy * s
        dperp = -dx * s + dy * c
        prof = np.minimum(1.0 - np.abs(dperp) / W,
                          1.0 - np.maximum(0.0, np.abs(dpar) - Lr[q] / 2) / W)
        h = np.maximum(h, H[q] * np.maximum(0.0, prof))
    return _periodic_fix(h)


def terrain_plane(grid: Grid, a: float, bx: float, by: float) -> np.ndarray:
    """Planar terrain h = a + bx x + by y (not periodic unless bx = by = 0)."""
    x, y = node_coords(grid)
    X, Y = np.meshgrid(x, y)
    return a + bx * X + by * Y


def terrain_flat(grid: Grid, h0: float) -> np.ndarray:
    nx, ny, _ = grid.n
    return np.full((ny + 1, nx + 1), float(h0))


# ----------------------------------------------------------------------- states

def _dup_periodic(rhou=None, rhov=None):
    if rhou is not None:
        rhou[:, :, -1] = rhou[:, :, 0]
    if rhov is not None:
        rhov[:, -1, :] = rhov[:, 0, :]


def state_unit(grid: Grid, seed: int, u0: float = 10.0) -> dict:
    """rho = 1, rho theta = 300 + 1e-3 (2 xi - 1), rho u = u0, rho v = rho w = 0."""
    rng = np.random.default_rng(seed)
    sh = field_shapes(grid.n)
    xi = rng.random(sh["rho"])
    U = {
        "rho": np.ones(sh["rho"]),
        "rhotheta": 300.0 + 1e-3 * (2.0 * xi - 1.0),
        "rhou": np.full(sh["rhou"], u0),
        "rhov": np.zeros(sh["rhov"]),
        "rhow": np.zeros(sh["rhow"]),
    }
    return U


def state_atmos(grid: Grid, seed: int, u0: float = 10.0, theta_noise: float = 0.1,
                u_noise: float = 0.05) -> dict:
    """Stably stratified state: theta = 300 + 0.003 z + 0.1 N(0,1) K,
    rho = 1.2 exp(-z / 8000), rho u = rho (10 + 0.05 N(0,1)), v = w = 0."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid.n
    sh = field_shapes(grid.n)
    zc = grid.lo[2] + (np.arange(nz, dtype=np.float64) + 0.5) * grid.dx[2]
    rho_z = 1.2 * np.exp(-zc / 8000.0)
    theta = 300.0 + 0.003 * zc[:, None, None] + theta_noise * rng.standard_normal(sh["rho"])
    rho = np.broadcast_to(rho_z[:, None, None], sh["rho"]).copy()
    u = u0 + u_noise * rng.standard_normal((nz, ny, nx))
    rhou = np.empty(sh["rhou"])
    rhou[:, :, :nx] = rho_z[:, None, None] * u
    _dup_periodic(rhou=rhou)
    return {
        "rho": rho,
        "rhotheta": rho * theta,
        "rhou": rhou,
        "rhov": np.zeros(sh["rhov"]),
        "rhow": np.zeros(sh["rhow"]),
    }


def state_uniform(grid: Grid, rho=1.2, theta=300.0, u=10.0, v=0.0, w=0.0) -> dict:
    sh = field_shapes(grid.n)
    U = {
        "rho": np.full(sh["rho"], rho),
        "rhotheta": np.full(sh["rhotheta"], rho * theta),
        "rhou": np.full(sh["rhou"], rho * u),
        "rhov": np.full(sh["rhov"], rho * v),
        "rhow": np.full(sh["rhow"], rho * w),
    }
    U["rhow"][0] = 0.0
    U["rhow"][-1] = 0.0
    return U


def state_random(grid: Grid, seed: int, amp: float = 1.0) -> dict:
    """Smooth-free random state (rho in [1, 2), theta in [290, 310), momenta
    uniform in [-amp, amp)), used by operator-level tests."""
    rng = np.random.default_rng(seed)
    sh = field_shapes(grid.n)
    rho = 1.0 + rng.random(sh["rho"])
    theta = 290.0 + 20.0 * rng.random(sh["rho"])
    U = {"rho": rho, "rhotheta": rho * theta}
    for name in ("rhou", "rhov", "rhow"):
        U[name] = amp * (2.0 * rng.random(sh[name]) - 1.0)
    _dup_periodic(U["rhou"], U["rhov"])
    U["rhow"][0] = 0.0
    U["rhow"][-1] = 0.0
    return U


# ------------------------------------------------------------ reference state

@dataclass
class Reference:
    """Hydrostatic reference state at the cell-centre height of every level,
    with the constants of the equation of state and gravity.  rhotheta0 and
    rho0 define it; p0 is the pressure the recipe started from (equal to the
    equation-of-state value of rhotheta0 up to rounding)."""
    p0: np.ndarray         # (nz,) Pa
    rho0: np.ndarray       # (nz,) kg/m^3
    rhotheta0: np.ndarray  # (nz,) kg K/m^3
    theta0: float = 300.0
    P00: float = 1.0e5
    R: float = 287.0
    gamma: float = 1.4
    g: float = 9.81


def reference_isentropic(grid: Grid, theta0: float = 300.0, P00: float = 1.0e5, R: float = 287.0,
                         gamma: float = 1.4, g: float = 9.81) -> Reference:
    """Dry atmosphere of constant potential temperature theta0 in hydrostatic
    balance (textbook form): Exner function pi(z) = 1 - g z / (cp theta0),
    cp = gamma R / (gamma - 1), p0 = P00 pi^(cp / R), rho0 = p0 / (R theta0 pi),
    taken at z = lo_z + (k + 1/2) dz."""
    nz = grid.n[2]
    z = grid.lo[2] + (np.arange(nz, dtype=np.float64) + 0.5) * grid.dx[2]
    cp = gamma * R / (gamma - 1.0)
    pi = 1.0 - g * z / (cp * theta0)
    p0 = P00 * pi ** (cp / R)
    rho0 = p0 / (R * theta0 * pi)
    return Reference(p0, rho0, rho0 * theta0, theta0, P00, R, gamma, g)


def state_reference(grid: Grid, ref: Reference, seed: int, rho_noise: float = 1e-4,
                    theta_noise: float = 1e-3, theta_amp: float = 1.0, u0: float = 10.0,
                    w_amp: float = 0.5) -> dict:
    """Perturbed reference state: a smooth potential-temperature anomaly plus
    small cell noise, theta = theta0 + theta_amp cos(2 pi x / Lx) cos(2 pi y /
    Ly) sin(pi z / Lz) + theta_noise N(0,1), rho = rho0 (1 + rho_noise
    N(0,1)), rho u = rho0 (u0 + N(0,1)), rho v, rho w = rho0 w_amp N(0,1)
    (walls 0).  All amplitudes 0 give the reference state at rest."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = grid.n
    sh = field_shapes(grid.n)
    r0 = ref.rho0[:, None, None]
    rho = r0 * (1.0 + rho_noise * rng.standard_normal(sh["rho"]))
    L = grid.length
    xc = (np.arange(nx) + 0.5) * grid.dx[0]
    yc = (np.arange(ny) + 0.5) * grid.dx[1]
    zc = (np.arange(nz) + 0.5) * grid.dx[2]
    bump = (np.sin(np.pi * zc / L[2])[:, None, None] * np.cos(2 * np.pi * yc / L[1])[None, :, None]
            * np.cos(2 * np.pi * xc / L[0])[None, None, :])
    theta = ref.theta0 + theta_amp * bump + theta_noise * rng.standard_normal(sh["rho"])
    rhou = np.empty(sh["rhou"])
    rhou[:, :, :nx] = r0 * (u0 + (1.0 if u0 else 0.0) * rng.standard_normal((nz, ny, nx)))
    rhov = np.empty(sh["rhov"])
    rhov[:, :ny, :] = r0 * w_amp * rng.standard_normal((nz, ny, nx))
    _dup_periodic(rhou, rhov)
    r0w = np.concatenate([ref.rho0[:1], ref.rho0])[:, None, None]
    rhow = r0w * w_amp * rng.standard_normal(sh["rhow"])
    rhow[0] = 0.0
    rhow[-1] = 0.0
    return {"rho": rho, "rhotheta": rho * theta, "rhou": rhou, "rhov": rhov, "rhow": rhow}


# ------------------------------------------------------------------------ boxes

def boxes_split(n, seed: int, target: int, block: int = 64, unit: int = 16):
    """Uneven AMR-style box list tiling the domain: chop into block^3 boxes,
    then repeatedly pick a box uniformly among those whose longest side is at
    least 2 unit and split its longest side (ties to the lower axis) at a
    random multiple of `unit`."""
    rng = np.random.default_rng(seed)
    boxes = []
    for k0 in range(0, n[2], block):
        for j0 in range(0, n[1], block):
            for i0 in range(0, n[0], block):
                lo = (i0, j0, k0)
                hi = (min(i0 + block, n[0]), min(j0 + block, n[1]), min(k0 + block, n[2]))
                boxes.append((lo, hi))
    while len(boxes) < target:
        cand = [b for b in boxes if max(h - l for l, h in zip(*b)) >= 2 * unit]
        if not cand:
            break
        b = cand[int(rng.integers(len(cand)))]
        lo, hi = b
        sides = [h - l for l, h in zip(lo, hi)]
        d = int(np.argmax(sides))
        L = sides[d]
        t = int(rng.integers(1, L // unit))
        cut = lo[d] + unit * t
        hi1 = list(hi); hi1[d] = cut
        lo2 = list(lo); lo2[d] = cut
        boxes.remove(b)
        boxes.append((tuple(lo), tuple(hi1)))
        boxes.append((tuple(lo2), tuple(hi)))
    return boxes


# -------------------------------------------------------------------- workloads

# ------------------------------------------------------------------ level sets

def node_coords3(grid: Grid):
    x, y = node_coords(grid)
    z = grid.lo[2] + np.arange(grid.n[2] + 1, dtype=np.float64) * grid.dx[2]
    return x, y, z


def _periodic_fix3(phi: np.ndarray) -> np.ndarray:
    phi[:, :, -1] = phi[:, :, 0]
    phi[:, -1, :] = phi[:, 0, :]
    return phi


def levelset_terrain(grid: Grid, h_nodes: np.ndarray) -> np.ndarray:
    """phi = z - h(x, y) at the nodes: the terrain as a level set."""
    _, _, z = node_coords3(grid)
    return np.ascontiguousarray(z[:, None, None] - h_nodes[None, :, :])


def levelset_hemisphere(grid: Grid, radius: float, centre=None) -> np.ndarray:
    """Signed distance to a hemisphere of the given radius standing on the
    domain bottom (Section 6.2), centred in x and y unless given; periodic
    minimum image in x and y."""
    x, y, z = node_coords3(grid)
    Lx, Ly, _ = grid.length
    cx, cy = centre if centre is not None else (grid.lo[0] + Lx / 2, grid.lo[1] + Ly / 2)
    dx = _min_image(x - cx, Lx)
    dy = _min_image(y - cy, Ly)
    dz = z - grid.lo[2]
    r = np.sqrt(dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2)
    return _periodic_fix3(np.ascontiguousarray(r - radius))


def levelset_box_cylinder(grid: Grid, width: float, height: float, angle: float,
                          centre=None) -> np.ndarray:
    """Signed distance to a wall-mounted square cylinder (Section 6.3) of the
    given width and height standing on the domain bottom, its sides turned by
    `angle` against the grid lines; periodic minimum image in x and y."""
    x, y, z = node_coords3(grid)
    Lx, Ly, _ = grid.length
    cx, cy = centre if centre is not None else (grid.lo[0] + Lx / 2, grid.lo[1] + Ly / 2)
    dx = _min_image(x - cx, Lx)[None, None, :]
    dy = _min_image(y - cy, Ly)[None, :, None]
    dz = (z - grid.lo[2])[:, None, None]
    c, s = np.cos(angle), np.sin(angle)
    qx = np.abs(c * dx + s * dy) - 0.5 * width
    qy = np.abs(-s * dx + c * dy) - 0.5 * width
    qz = np.abs(dz) - height
    qx, qy, qz = np.broadcast_arrays(qx, qy, qz)
    out = np.sqrt(np.maximum(qx, 0) ** 2 + np.maximum(qy, 0) ** 2 + np.maximum(qz, 0) ** 2)
    inside = np.minimum(np.maximum(np.maximum(qx, qy), qz), 0.0)
    return _periodic_fix3(np.ascontiguousarray(out + inside))


def make_levelset_workload(name: str) -> Workload:
    """Level-set geometries of the paper's validation cases, on windows sized
    for the oracle: "hemisphere" (radius 0.5 on the paper's mesh spacing
    10/256, a 64 x 64 x 32 window around it) and "cylinder" (square cylinder
    of width 1 and height 3 at 12 cells per width, turned by 0.3 rad, in a
    48^3 window of edge 4)."""
    if name == "hemisphere":
        d = 10.0 / 256
        g = Grid((64, 64, 32), (d, d, d))
        return Workload("hemisphere_64x64x32", g, None, cfl_dt(g), 21, [((0, 0, 0), g.n)], "unit",
                        phi_nodes=levelset_hemisphere(g, 0.5))
    if name == "cylinder":
        d = 1.0 / 12
        g = Grid((48, 48, 48), (d, d, d))
        return Workload("cylinder_48x48x48", g, None, cfl_dt(g), 22, [((0, 0, 0), g.n)], "unit",
                        phi_nodes=levelset_box_cylinder(g, 1.0, 3.0, 0.3))
    raise ValueError(f"unknown level-set workload {name}")


def make_workload(cfg: int) -> Workload:
    """Configurations 1-5 (see the design notes for the full recipe)."""
    if cfg == 1:
        g = Grid((32, 32, 32), (1 / 32, 1 / 32, 1 / 32))
        return Workload("c1_gauss_32", g, terrain_gaussian_unit(g), 1.5625e-3, 1,
                        [((0, 0, 0), g.n)], "unit")
    if cfg == 2:
        g = Grid((128, 128, 64), (78.125, 78.125, 31.25))
        return Workload("c2_agnesi_128x128x64", g, terrain_agnesi(g), cfl_dt(g), 2,
                        [((0, 0, 0), g.n)], "atmos")
    if cfg == 3:
        g = Grid((256, 256, 128), (78.125, 78.125, 23.4375))
        return Workload("c3_hills8_256x256x128", g, terrain_gaussian_hills(g, 3, 8), cfl_dt(g), 3,
                        [((0, 0, 0), g.n)], "atmos")
    if cfg == 4:
        g = Grid((512, 512, 128), (78.125, 78.125, 23.4375))
        return Workload("c4_boxes512_512x512x128", g, terrain_gaussian_hills(g, 4, 16),
                        cfl_dt(g), 4, boxes_split(g.n, 4, 512), "atmos")
    if cfg == 5:
        g = Grid((1024, 1024, 192), (50.0, 50.0, 20.0))
        return Workload("c5_ridges_1024x1024x192", g, terrain_ridges(g, 5), cfl_dt(g), 5,
                        boxes_split(g.n, 5, 3072), "atmos")
    raise ValueError(f"unknown configuration {cfg}")


def make_state(w: Workload) -> dict:
    if w.state_kind == "unit":
        return state_unit(w.grid, w.seed)
    return state_atmos(w.grid, 1000 + w.seed)


def window(w: Workload, i0: int, j0: int, nx: int, ny: int, nz: int) -> Workload:
    """A periodic sub-problem cut from a workload's terrain (used to time the
    oracle on a bounded sample of a large configuration): the window's nodes
    are taken as they are and the last row / column is made periodic."""
    h = w.h_nodes[j0:j0 + ny + 1, i0:i0 + nx + 1].copy()
    g = Grid((nx, ny, nz), w.grid.dx, w.grid.lo, w.grid.small_vfrac)
    return Workload(w.name + f"_win{nx}x{ny}x{nz}", g, _periodic_fix(h), w.dt, w.seed,
                    [((0, 0, 0), g.n)], w.state_kind)
