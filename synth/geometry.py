"""Seeded geometry inputs for embedded-boundary (cut-cell) problems.

An electrode is given by a signed distance function psi (positive in the
gas, negative inside the conductor).  For a grid of n_x * n_y * n_z cubic
cells of side h this module returns, per cell and face, the geometric data
that a cut-cell discretisation takes as input:

- kappa[k][j][i]: the gas volume fraction of the cell (midpoint rule on
  nsub^3 sub-cells; exactly 0 or 1 away from the surface);
- ax[k][j][i'] (i' = 0..nx), ay, az: the gas fraction of each face (the
  face-coefficient layout of the multigrid engine; midpoint rule on nsub^2
  sub-faces);
- the boundary cells (any gas volume, and some solid volume or face) as flat
  C-order indices, with the closest surface point to each cell centre,
  stored as its offset from the centre in units of h.

These are geometry, not the discretisation: the operator built from them
lives in the oracle and in the kernels, separately.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional, Tuple

import numpy as np

NEEDLE_RADIUS = 0.025    # 500 um in a (2 cm)^3 box
NEEDLE_TIP_Z = 0.5       # protrudes 1 cm from the top face
NEEDLE_AXIS = (0.5, 0.5)


@dataclass
class Shape:
    """psi(x, y, z) and its closest surface point (vectorised over arrays)."""
    psi: Callable
    closest: Callable
    name: str = ""


def needle(radius: float = NEEDLE_RADIUS, tip_z: float = NEEDLE_TIP_Z, axis=NEEDLE_AXIS) -> Shape:
    """A cylinder of the given radius along z from z = 1 (the top face) down
    to a hemispherical cap whose lowest point is at tip_z."""
    x0, y0 = axis
    zc = tip_z + radius

    def psi(x, y, z):
        rho = np.hypot(x - x0, y - y0)
        d_cyl = rho - radius
        d_cap = np.sqrt(rho**2 + (z - zc) ** 2) - radius
        return np.where(z >= zc, d_cyl, d_cap)

    def closest(x, y, z):
        rho = np.hypot(x - x0, y - y0)
        safe = np.where(rho > 0, rho, 1.0)
        ux, uy = np.where(rho > 0, (x - x0) / safe, 1.0), np.where(rho > 0, (y - y0) / safe, 0.0)
        cx_cyl, cy_cyl, cz_cyl = x0 + radius * ux, y0 + radius * uy, z
        r3 = np.sqrt(rho**2 + (z - zc) ** 2)
        s3 = np.where(r3 > 0, r3, 1.0)
        cx_cap = x0 + radius * np.where(r3 > 0, (x - x0) / s3, 0.0)
        cy_cap = y0 + radius * np.where(r3 > 0, (y - y0) / s3, 0.0)
        cz_cap = zc + radius * np.where(r3 > 0, (z - zc) / s3, -1.0)
        up = z >= zc
        return (np.where(up, cx_cyl, cx_cap), np.where(up, cy_cyl, cy_cap), np.where(up, cz_cyl, cz_cap))

    return Shape(psi, closest, f"needle_r{radius}_tip{tip_z}")


def sphere(center=(0.5, 0.5, 0.5), radius: float = 0.25) -> Shape:
    cx, cy, cz = center

    def psi(x, y, z):
        return np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) - radius

    def closest(x, y, z):
        r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
        s = np.where(r > 0, r, 1.0)
        return (cx + radius * np.where(r > 0, (x - cx) / s, 1.0), cy + radius * np.where(r > 0, (y - cy) / s, 0.0),
                cz + radius * np.where(r > 0, (z - cz) / s, 0.0))

    return Shape(psi, closest, f"sphere_r{radius}")


def half_space(normal, offset: float) -> Shape:
    """Gas where n . x > offset (n normalised), conductor below."""
    n = np.asarray(normal, dtype=np.float64)
    n = n / np.linalg.norm(n)

    def psi(x, y, z):
        return n[0] * x + n[1] * y + n[2] * z - offset

    def closest(x, y, z):
        d = n[0] * x + n[1] * y + n[2] * z - offset
        return x - d * n[0], y - d * n[1], z - d * n[2]

    return Shape(psi, closest, "half_space")


@dataclass
class Geometry:
    kappa: np.ndarray
    ax: np.ndarray
    ay: np.ndarray
    az: np.ndarray
    bidx: np.ndarray   # flat C-order indices of the boundary cells (int64, sorted)
    boff: np.ndarray   # [nb][3] closest surface point minus cell centre, in units of h (x, y, z)
    name: str = ""


def _frac(shape: Shape, pts) -> np.ndarray:
    return (shape.psi(*pts) > 0).mean(axis=-1)


def cut_geometry(shape: Shape, nx: int, ny: int, nz: int, h: float, nsub: int = 4) -> Geometry:
    """Volume and face fractions (midpoint rule, nsub points per axis) and the
    boundary cells of `shape` on the grid (origin at 0)."""
    s = (np.arange(nsub) + 0.5) / nsub  # sub-point positions in [0, 1]
    band = 0.87 * h  # a cell or face further than this from the surface is uniform

    def cells(x, y, z):
        """Fractions of the cells with lower corners (x, y, z) (1D arrays of equal length)."""
        px = x[:, None] + h * np.repeat(s, nsub * nsub)[None, :]
        py = y[:, None] + h * np.tile(np.repeat(s, nsub), nsub)[None, :]
        pz = z[:, None] + h * np.tile(s, nsub * nsub)[None, :]
        return _frac(shape, (px, py, pz))

    def faces(x, y, z, axis):
        """Fractions of the faces with lower corners (x, y, z) normal to `axis`."""
        u, v = np.repeat(s, nsub), np.tile(s, nsub)
        o = [x[:, None] + 0 * u[None, :], y[:, None] + 0 * u[None, :], z[:, None] + 0 * u[None, :]]
        t = [a for a in range(3) if a != axis]
        o[t[0]] = o[t[0]] + h * u[None, :]
        o[t[1]] = o[t[1]] + h * v[None, :]
        return _frac(shape, tuple(o))

    # volume fractions
    zc, yc, xc = np.meshgrid((np.arange(nz) + 0.5) * h, (np.arange(ny) + 0.5) * h, (np.arange(nx) + 0.5) * h,
                             indexing="ij")
    d = shape.psi(xc, yc, zc)
    kappa = (d > 0).astype(np.float64)
    near = np.abs(d) < band
    kk, jj, ii = np.nonzero(near)
    if kk.size:
        kappa[kk, jj, ii] = cells(ii * h, jj * h, kk * h)
    # face fractions: face centres, then the faces near the surface
    out = []
    for axis, shp in ((0, (nz, ny, nx + 1)), (1, (nz, ny + 1, nx)), (2, (nz + 1, ny, nx))):
        k, j, i = np.meshgrid(np.arange(shp[0]), np.arange(shp[1]), np.arange(shp[2]), indexing="ij")
        fx = (i + (0.0 if axis == 0 else 0.5)) * h
        fy = (j + (0.0 if axis == 1 else 0.5)) * h
        fz = (k + (0.0 if axis == 2 else 0.5)) * h
        df = shape.psi(fx, fy, fz)
        a = (df > 0).astype(np.float64)
        kk, jj, ii = np.nonzero(np.abs(df) < band)
        if kk.size:
            lx = ii * h if axis == 0 else ii * h
            ly = jj * h
            lz = kk * h
            a[kk, jj, ii] = faces(lx.astype(np.float64), ly.astype(np.float64), lz.astype(np.float64), axis)
        out.append(a)
    ax, ay, az = out
    # boundary cells: some gas, and some solid volume or a face short of gas
    mn = np.minimum.reduce([ax[:, :, :-1], ax[:, :, 1:], ay[:, :-1, :], ay[:, 1:, :], az[:-1], az[1:]])
    bmask = (kappa > 0) & ((kappa < 1) | (mn < 1))
    bidx = np.flatnonzero(bmask).astype(np.int64)
    k, r = np.divmod(bidx, nx * ny)
    j, i = np.divmod(r, nx)
    cxp, cyp, czp = (i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h
    sx, sy, sz = shape.closest(cxp, cyp, czp)
    boff = np.stack([(sx - cxp) / h, (sy - cyp) / h, (sz - czp) / h], axis=1)
    return Geometry(kappa, ax, ay, az, bidx, np.ascontiguousarray(boff), shape.name)


def needle_plane(n: int, seed: int = 0, radius: float = NEEDLE_RADIUS, tip_z: float = NEEDLE_TIP_Z, nsub: int = 4):
    """The needle-plane potential of the paper's large example on n^3 cells
    of the unit box (a (2 cm)^3 cube): the needle (radius 500 um, tip 1 cm
    below the top face) and the top face at potential 1, the bottom face
    grounded, zero flux on the sides; the space charge is the seeded
    filament recipe (synth.problems.filament_source; its part inside the
    electrode is not used).  Returns (Problem, Geometry, g)."""
    from synth.problems import Problem, filament_source
    h = 1.0 / n
    G = cut_geometry(needle(radius, tip_z), n, n, n, h, nsub)
    f = filament_source(n, n, n, seed)
    bc = (("N", 0.0),) * 4 + (("D", 0.0), ("D", 1.0))
    return Problem(n, n, n, h, 0.0, f, None, bc, f"needle_plane_s{seed}_{n}"), G, 1.0
