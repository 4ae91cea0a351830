"""Independent test helpers: closed forms and brute-force samplers written
from the definitions (fluid = {z > h(x, y)} with h the piecewise-linear
interpolant of the nodal heights on the two triangles of each xy-cell).  They
share no code with the oracle or the library."""
from __future__ import annotations

import itertools
import math

import numpy as np


def halfspace_box_volume(lo, hi, w, d):
    """Exact volume of {p in box: w . p <= d} by inclusion-exclusion over the
    box vertices (coefficients made non-negative by reflection; zero
    coefficients factor out), evaluated in exact rational arithmetic on the
    binary values of the inputs and rounded once at the end."""
    from fractions import Fraction as Fr
    lo = [Fr(float(v)) for v in lo]
    L = [Fr(float(h)) - l for h, l in zip(hi, lo)]
    w = [Fr(float(v)) for v in w]
    D = Fr(float(d)) - sum(wi * li for wi, li in zip(w, lo))
    c = []
    Ls = []
    factor = Fr(1)
    for i in range(3):
        if w[i] < 0:
            D -= w[i] * L[i]
            c.append(-w[i])
            Ls.append(L[i])
        elif w[i] > 0:
            c.append(w[i])
            Ls.append(L[i])
        else:
            factor *= L[i]
    n = len(c)
    if n == 0:
        return float(factor) if D >= 0 else 0.0
    tot = Fr(0)
    for S in itertools.product((0, 1), repeat=n):
        t = D - sum(c[i] * Ls[i] for i in range(n) if S[i])
        if t > 0:
            tot += (-1) ** sum(S) * t ** n
    den = Fr(math.factorial(n))
    for ci in c:
        den *= ci
    return float(factor * tot / den)


def interp_h(h_nodes, grid, x, y):
    """Piecewise-linear terrain at points (x, y) (arrays), two triangles per
    xy-cell split along the (i,j)-(i+1,j+1) diagonal."""
    nx, ny, _ = grid.n
    dx, dy = grid.dx[0], grid.dx[1]
    fx = (np.asarray(x) - grid.lo[0]) / dx
    fy = (np.asarray(y) - grid.lo[1]) / dy
    i = np.clip(np.floor(fx).astype(int), 0, nx - 1)
    j = np.clip(np.floor(fy).astype(int), 0, ny - 1)
    s = fx - i
    t = fy - j
    ha = h_nodes[j, i]
    hb = h_nodes[j, i + 1]
    hc = h_nodes[j + 1, i + 1]
    hd = h_nodes[j + 1, i]
    lower = s >= t
    h = np.where(lower, ha + s * (hb - ha) + t * (hc - hb), ha + s * (hc - hd) + t * (hd - ha))
    gx = np.where(lower, (hb - ha) / dx, (hc - hd) / dx)
    gy = np.where(lower, (hc - hb) / dy, (hd - ha) / dy)
    return h, gx, gy


def sample_cv(h_nodes, grid, box, M=256):
    """Brute-force moments of the fluid part of an axis-aligned box
    (x0, x1, y0, y1, z0, z1) that stays inside the domain in x and y:
    2-D midpoint rule in (x, y) with the z extent integrated exactly.
    Returns volume, centroid (3), and the EB area vector (3)."""
    x0, x1, y0, y1, z0, z1 = box
    xs = x0 + (np.arange(M) + 0.5) * (x1 - x0) / M
    ys = y0 + (np.arange(M) + 0.5) * (y1 - y0) / M
    X, Y = np.meshgrid(xs, ys)
    h, gx, gy = interp_h(h_nodes, grid, X, Y)
    dA = (x1 - x0) * (y1 - y0) / (M * M)
    zc = np.clip(h, z0, z1)
    col = z1 - zc
    V = col.sum() * dA
    cx = (X * col).sum() * dA / V if V > 0 else 0.0
    cy = (Y * col).sum() * dA / V if V > 0 else 0.0
    cz = (0.5 * (z1 * z1 - zc * zc)).sum() * dA / V if V > 0 else 0.0
    inside = (h >= z0) & (h < z1)
    av = np.array([(-gx * inside).sum(), (-gy * inside).sum(), inside.sum()]) * dA
    return V, np.array([cx, cy, cz]), av


def sample_vface(h_nodes, grid, d, f, s0, s1, z0, z1, M=4096):
    """Fluid fraction of the vertical face {x = f} (d = 0) or {y = f} (d = 1)
    over s in [s0, s1] and z in [z0, z1] by a 1-D midpoint rule."""
    s = s0 + (np.arange(M) + 0.5) * (s1 - s0) / M
    if d == 0:
        h, _, _ = interp_h(h_nodes, grid, np.full(M, f), s)
    else:
        h, _, _ = interp_h(h_nodes, grid, s, np.full(M, f))
    return float((z1 - np.clip(h, z0, z1)).mean() / (z1 - z0))


def clip_polygon(poly, a, b, c):
    """Part of a convex polygon [(u, v), ...] where a u + b v + c >= 0
    (one Sutherland-Hodgman pass)."""
    out = []
    n = len(poly)
    for q in range(n):
        P, Q = poly[q], poly[(q + 1) % n]
        fp = a * P[0] + b * P[1] + c
        fq = a * Q[0] + b * Q[1] + c
        if fp >= 0:
            out.append(P)
        if (fp >= 0) != (fq >= 0):
            t = fp / (fp - fq)
            out.append((P[0] + t * (Q[0] - P[0]), P[1] + t * (Q[1] - P[1])))
    return out


def polygon_area_centroid(poly):
    """Area and centroid of a simple polygon by the shoelace formula
    (0, (0, 0) for fewer than three vertices or zero area)."""
    if len(poly) < 3:
        return 0.0, (0.0, 0.0)
    A = cx = cy = 0.0
    n = len(poly)
    for q in range(n):
        x0, y0 = poly[q]
        x1, y1 = poly[(q + 1) % n]
        cr = x0 * y1 - x1 * y0
        A += cr
        cx += (x0 + x1) * cr
        cy += (y0 + y1) * cr
    A *= 0.5
    if A == 0.0:
        return 0.0, (0.0, 0.0)
    return abs(A), (cx / (6 * A), cy / (6 * A))


def rect(u0, u1, v0, v1):
    return [(u0, v0), (u1, v0), (u1, v1), (u0, v1)]


def sample_vface_moments(h_nodes, grid, d, f, s0, s1, z0, z1, M=8192):
    """Fluid fraction and centroid (s, z) of the vertical face {x = f}
    (d = 0) or {y = f} (d = 1), s in [s0, s1], z in [z0, z1]: 1-D midpoint
    rule in s with the z extent of the fluid (z > h) integrated exactly."""
    s = s0 + (np.arange(M) + 0.5) * (s1 - s0) / M
    if d == 0:
        h, _, _ = interp_h(h_nodes, grid, np.full(M, f), s)
    else:
        h, _, _ = interp_h(h_nodes, grid, s, np.full(M, f))
    zc = np.clip(h, z0, z1)
    L = z1 - zc
    tot = L.sum()
    frac = float(tot / M / (z1 - z0))
    if tot <= 0:
        return frac, (0.0, 0.0)
    return frac, (float((s * L).sum() / tot), float((0.5 * (z1 * z1 - zc * zc)).sum() / tot))


def sample_zface_moments(h_nodes, grid, zf, x0, x1, y0, y1, M=512):
    """Fluid fraction and centroid (x, y) of the horizontal face {z = zf}
    over [x0, x1] x [y0, y1] (fluid where h < zf), 2-D midpoint rule."""
    xs = x0 + (np.arange(M) + 0.5) * (x1 - x0) / M
    ys = y0 + (np.arange(M) + 0.5) * (y1 - y0) / M
    X, Y = np.meshgrid(xs, ys)
    h, _, _ = interp_h(h_nodes, grid, X, Y)
    fl = h < zf
    n = fl.sum()
    if n == 0:
        return 0.0, (0.0, 0.0)
    return float(n / (M * M)), (float(X[fl].mean()), float(Y[fl].mean()))


def sample_facet(h_nodes, grid, box, M=400):
    """EB facet inside a box by a 2-D midpoint rule over the box's xy
    rectangle: true area and area-weighted centroid (x, y, h) of the part of
    the terrain surface with z0 <= h < z1."""
    x0, x1, y0, y1, z0, z1 = box
    xs = x0 + (np.arange(M) + 0.5) * (x1 - x0) / M
    ys = y0 + (np.arange(M) + 0.5) * (y1 - y0) / M
    X, Y = np.meshgrid(xs, ys)
    h, gx, gy = interp_h(h_nodes, grid, X, Y)
    inside = (h >= z0) & (h < z1)
    w = np.sqrt(1.0 + gx * gx + gy * gy) * inside
    dA = (x1 - x0) * (y1 - y0) / (M * M)
    A = w.sum() * dA
    if A <= 0:
        return 0.0, np.zeros(3)
    return float(A), np.array([(X * w).sum(), (Y * w).sum(), (h * w).sum()]) * dA / A


# ------------------------------------------------------------------ level sets

def kuhn_phi(phi_nodes, grid, x, y, z):
    """Piecewise-linear interpolant of nodal phi ((nz+1, ny+1, nx+1)) over
    the six Kuhn tetrahedra of each cell, evaluated at points: with the unit
    coordinates sorted u(1) >= u(2) >= u(3) (axes s0, s1, s2) the value is
    (1 - u(1)) phi(0) + (u(1) - u(2)) phi(e_s0) + (u(2) - u(3)) phi(e_s0 + e_s1)
    + u(3) phi(1, 1, 1)."""
    nx, ny, nz = grid.n
    x, y, z = np.broadcast_arrays(np.asarray(x, float), np.asarray(y, float), np.asarray(z, float))
    f = [(x - grid.lo[0]) / grid.dx[0], (y - grid.lo[1]) / grid.dx[1], (z - grid.lo[2]) / grid.dx[2]]
    lim = (nx - 1, ny - 1, nz - 1)
    idx = [np.clip(np.floor(f[d]).astype(int), 0, lim[d]) for d in range(3)]
    u = np.stack([f[d] - idx[d] for d in range(3)], axis=-1)
    order = np.argsort(-u, axis=-1, kind="stable")
    us = np.take_along_axis(u, order, axis=-1)

    def node(bits):
        return phi_nodes[idx[2] + bits[..., 2], idx[1] + bits[..., 1], idx[0] + bits[..., 0]]

    b = np.zeros(u.shape, dtype=int)
    val = (1.0 - us[..., 0]) * node(b)
    for m in range(3):
        np.put_along_axis(b, order[..., m:m + 1], 1, axis=-1)
        w = us[..., m] - (us[..., m + 1] if m < 2 else 0.0)
        val = val + w * node(b)
    return val


def levelset_fluid_length(phi_nodes, grid, x, y, z0, z1):
    """Length of {z in [z0, z1] : phi > 0} on vertical lines at points (x, y)
    (arrays): the interpolant is linear in z between the breakpoints z_k + u dz
    and z_k + v dz (u, v the point's unit x, y coordinates) and the node
    planes, so the positive part of every segment is exact."""
    x = np.asarray(x, float)
    y = np.asarray(y, float)
    dz = grid.dx[2]
    u = (x - grid.lo[0]) / grid.dx[0]
    v = (y - grid.lo[1]) / grid.dx[1]
    u = u - np.floor(u)
    v = v - np.floor(v)
    k0 = int(np.floor((z0 - grid.lo[2]) / dz))
    k1 = int(np.ceil((z1 - grid.lo[2]) / dz))
    bps = [np.full(x.shape, z0), np.full(x.shape, z1)]
    for k in range(k0, k1 + 1):
        zk = grid.lo[2] + k * dz
        for t in (np.zeros(x.shape), u, v):
            bps.append(np.clip(zk + t * dz, z0, z1))
    B = np.sort(np.stack(bps, axis=-1), axis=-1)
    L = np.zeros(x.shape)
    for q in range(B.shape[-1] - 1):
        za, zb = B[..., q], B[..., q + 1]
        fa = kuhn_phi(phi_nodes, grid, x, y, za)
        fb = kuhn_phi(phi_nodes, grid, x, y, zb)
        seg = zb - za
        pos = np.where((fa > 0) & (fb > 0), seg,
                       np.where((fa > 0) | (fb > 0),
                                seg * np.maximum(fa, fb) / np.maximum(np.abs(fa - fb), 1e-300), 0.0))
        L += np.where(seg > 0, pos, 0.0)
    return L
