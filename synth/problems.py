"""Seeded problem generators for the variable-permittivity Poisson and the
screened (Helmholtz) radiative-transfer solves.

Every generator returns plain NumPy float64 arrays in C order ``[nz][ny][nx]``
(x fastest) plus the scalar data of the equation

    a*u - div(beta grad u) = f   on an nx*ny*nz grid of cubic cells of side h,

with ``beta`` the cell permittivity (``eps``, or ``None`` for beta = 1), ``a``
the screening coefficient kappa^2 and one boundary condition per box face
(order x-, x+, y-, y+, z-, z+; ``('D', g)`` = Dirichlet value g,
``('N', 0.0)`` = homogeneous Neumann).

The shapes follow the paper's workloads: the potential is solved with a live
electrode face at z = 1, a grounded face at z = 0 and zero-flux side walls
(Sec. 3 rod-plane and Sec. 4 needle-plane set-ups), and the space charge is a
streamer-like filament with a sharp charged head.  The paper's own geometry,
chemistry and Perlin preionisation are not reproducible here, so a seeded
Gaussian filament stands in for them.

Nothing in this module evaluates the discrete operator or any solver step.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# kappa_i * h for the three photon groups of the three-term radiative model.
# The fitted constants of that model are not in the paper, so three values
# spanning weak, medium and strong screening stand in for them.
HELMHOLTZ_KDX = (0.05, 0.3, 1.5)

# filament shape (all lengths in cells of the finest grid unless stated)
FIL_RADIUS_CELLS = 6.0
FIL_ROLLOFF_CELLS = 2.0
FIL_HEAD_AMPLITUDE = 1.0e3
FIL_NOISE_SIGMA = 0.1
FIL_Z_TOP = 0.9
FIL_TIP_RANGE = (0.3, 0.7)
SLAB_TOP = 0.1
SLAB_EPS = 4.0

BATCH_SIZES = (32, 48, 64, 96, 128)


@dataclass
class Problem:
    nx: int
    ny: int
    nz: int
    h: float
    a: float
    f: np.ndarray
    eps: Optional[np.ndarray] = None
    bc: Tuple[Tuple[str, float], ...] = field(default_factory=lambda: (("N", 0.0),) * 6)
    name: str = ""
    # face coefficients (bx [nz][ny][nx+1], by [nz][ny+1][nx], bz [nz+1][ny][nx])
    # given directly instead of a cell coefficient; boundary entries are the
    # coefficients of Dirichlet faces
    faces: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def bc_types(self) -> List[str]:
        return [t for t, _ in self.bc]

    def bc_values(self) -> List[float]:
        return [float(v) for _, v in self.bc]


def cell_centres(nx: int, ny: int, nz: int, h: float):
    """1D coordinate vectors of the cell centres (i + 1/2) h."""
    x = (np.arange(nx, dtype=np.float64) + 0.5) * h
    y = (np.arange(ny, dtype=np.float64) + 0.5) * h
    z = (np.arange(nz, dtype=np.float64) + 0.5) * h
    return x, y, z


POISSON_BC = (("N", 0.0), ("N", 0.0), ("N", 0.0), ("N", 0.0), ("D", 0.0), ("D", 1.0))
HELMHOLTZ_BC = (("D", 0.0),) * 6


def manufactured_poisson(nx: int = 32, ny: Optional[int] = None, nz: Optional[int] = None) -> Problem:
    """Constant-coefficient Poisson problem with the known continuum solution

        phi = z + cos(pi x / Lx) cos(pi y / Ly) sin(2 pi z),

    on [0,Lx] x [0,Ly] x [0,1] with h = 1/nz: grounded z = 0, phi = 1 at
    z = 1, zero flux on the side walls (the cosine factors make the
    correction term Neumann-compatible there).  f = -lap(phi) sampled at
    cell centres.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    h = 1.0 / nz
    lx, ly = nx * h, ny * h
    x, y, z = cell_centres(nx, ny, nz, h)
    amp = np.pi**2 / lx**2 + np.pi**2 / ly**2 + 4.0 * np.pi**2
    f = (
        amp
        * np.sin(2 * np.pi * z)[:, None, None]
        * np.cos(np.pi * y / ly)[None, :, None]
        * np.cos(np.pi * x / lx)[None, None, :]
    )
    return Problem(nx, ny, nz, h, 0.0, np.ascontiguousarray(f), None, POISSON_BC, f"manufactured_{nx}x{ny}x{nz}")


def filament_source(nx: int, ny: int, nz: int, seed: int, tip_shift: float = 0.0) -> np.ndarray:
    """Seeded streamer-like space charge rho on an nx*ny*nz grid, h = 1/nz.

    A Gaussian column of radius 6 cells on the x-y centre of the box runs
    from z = 0.9 down to a random tip height in [0.3, 0.7]; its ends roll off
    over 2 cells, the tip carries a head of amplitude 1e3 and width 2 cells,
    and the whole field is multiplied by mean-one lognormal noise (sigma 0.1).
    Draw order: tip height, then one standard normal per cell in C order.
    tip_shift lowers the drawn tip by that length (the same draws otherwise):
    the filament of a later time of a streamer advancing towards z = 0.
    """
    h = 1.0 / nz
    rng = np.random.default_rng(seed)
    z_tip = rng.uniform(*FIL_TIP_RANGE) - tip_shift
    x, y, z = cell_centres(nx, ny, nz, h)
    x0, y0 = 0.5 * nx * h, 0.5 * ny * h
    r_fil = FIL_RADIUS_CELLS * h
    w = FIL_ROLLOFF_CELLS * h
    g2 = np.exp(-((x[None, :] - x0) ** 2 + (y[:, None] - y0) ** 2) / r_fil**2)  # [ny][nx]
    dist = np.where(z < z_tip, z_tip - z, np.where(z > FIL_Z_TOP, z - FIL_Z_TOP, 0.0))
    body = np.exp(-(dist**2) / w**2)
    head = FIL_HEAD_AMPLITUDE * np.exp(-((z - z_tip) ** 2) / w**2)
    prof = body + head  # [nz]
    rho = rng.standard_normal((nz, ny, nx))
    sig = FIL_NOISE_SIGMA
    rho *= sig
    rho -= 0.5 * sig * sig
    np.exp(rho, out=rho)
    rho *= g2[None, :, :]
    rho *= prof[:, None, None]
    return rho


def slab_permittivity(nx: int, ny: int, nz: int) -> np.ndarray:
    """eps = 4 in cells whose centre lies below z = 0.1 (a dielectric slab on
    the grounded face), eps = 1 (gas) above."""
    h = 1.0 / nz
    _, _, z = cell_centres(nx, ny, nz, h)
    col = np.where(z < SLAB_TOP, SLAB_EPS, 1.0)
    return np.ascontiguousarray(np.broadcast_to(col[:, None, None], (nz, ny, nx)).astype(np.float64))


def streamer_set(nx: int, ny: Optional[int] = None, nz: Optional[int] = None, seed: int = 0,
                 kdx: Sequence[float] = HELMHOLTZ_KDX) -> List[Problem]:
    """The four elliptic solves of one field update on a seeded filament:

    0. potential: variable eps (slab), f = rho, grounded z = 0, phi = 1 on
       z = 1, zero flux on the side walls;
    1-3. photon groups: beta = 1, a = (kdx_i / h)^2, f = rho (the source
       stands in for the ionisation rate), Psi = 0 on every face.
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    h = 1.0 / nz
    rho = filament_source(nx, ny, nz, seed)
    eps = slab_permittivity(nx, ny, nz)
    out = [Problem(nx, ny, nz, h, 0.0, rho, eps, POISSON_BC, f"poisson_s{seed}_{nx}x{ny}x{nz}")]
    for i, c in enumerate(kdx):
        kap = c / h
        out.append(Problem(nx, ny, nz, h, kap * kap, rho, None, HELMHOLTZ_BC,
                           f"helmholtz{i}_s{seed}_{nx}x{ny}x{nz}"))
    return out


def batch_dims(count: int = 64, seed: int = 4, sizes: Sequence[int] = BATCH_SIZES) -> np.ndarray:
    """(count, 3) array of (nx, ny, nz) with each axis drawn independently
    and uniformly from ``sizes``."""
    rng = np.random.default_rng(seed)
    return rng.choice(np.asarray(sizes), size=(count, 3))


def random_problem(nx: int, ny: int, nz: int, seed: int, *, variable_eps: bool = True,
                   a: Optional[float] = None, bc: Optional[Sequence[Tuple[str, float]]] = None,
                   h: Optional[float] = None) -> Problem:
    """Small problem with random coefficients for brute-force checks:
    log-uniform eps in [0.25, 8], uniform f in [-1, 1], random face types
    (at least one Dirichlet face unless a > 0) and values in [-1, 1]."""
    rng = np.random.default_rng(seed)
    h = 1.0 / max(nx, ny, nz) if h is None else h
    eps = np.exp(rng.uniform(np.log(0.25), np.log(8.0), size=(nz, ny, nx))) if variable_eps else None
    f = rng.uniform(-1.0, 1.0, size=(nz, ny, nx))
    if bc is None:
        types = ["D" if t else "N" for t in rng.integers(0, 2, size=6)]
        vals = rng.uniform(-1.0, 1.0, size=6)
        if a is None or a == 0.0:
            if "D" not in types:
                types[int(rng.integers(0, 6))] = "D"
        bc = tuple((t, float(v) if t == "D" else 0.0) for t, v in zip(types, vals))
    if a is None:
        a = float(rng.uniform(0.0, 50.0))
    return Problem(nx, ny, nz, h, float(a), f, eps, tuple(bc), f"random_s{seed}_{nx}x{ny}x{nz}")


def random_faces(nx: int, ny: int, nz: int, seed: int, lo: float = 0.25, hi: float = 8.0):
    """Face coefficients (bx, by, bz), log-uniform in [lo, hi], independent per face."""
    rng = np.random.default_rng(seed)
    shapes = ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx))
    return tuple(np.exp(rng.uniform(np.log(lo), np.log(hi), size=sh)) for sh in shapes)


# Diffusion coefficient of the implicit (TGA) diffusion solves: D(E) on the
# faces.  The transport data that give D as a function of the field are not
# in the paper, so a stand-in with the same structure is used: D rises from
# D_GAS in the background to D_GAS * D_HEAD_RATIO in the high-field region
# around the filament head and along the channel, with mean-one lognormal
# noise per face.
D_GAS = 1.0
D_HEAD_RATIO = 10.0
D_NOISE_SIGMA = 0.1
TGA_DIFFUSION_NUMBER = 4.0  # max(D) dt / h^2 of the benchmark step


def diffusion_faces(nx: int, ny: int, nz: int, seed: int):
    """Seeded face diffusion coefficients (bx, by, bz) for the TGA solves on
    an nx*ny*nz grid (h = 1/nz): D = D_GAS * (1 + (D_HEAD_RATIO - 1) * w) *
    noise, where w in [0, 1] is the filament shape of filament_source (the
    same tip-height draw for the same seed) evaluated at each face centre,
    with the head weighted 1 and the channel 0.5.  Draw order: tip height,
    then one standard normal per face (x faces, y faces, z faces, C order)."""
    h = 1.0 / nz
    rng = np.random.default_rng(seed)
    z_tip = rng.uniform(*FIL_TIP_RANGE)
    x0, y0 = 0.5 * nx * h, 0.5 * ny * h
    r_fil = FIL_RADIUS_CELLS * h
    w = FIL_ROLLOFF_CELLS * h

    def shape(x, y, z):
        g2 = np.exp(-((x - x0) ** 2 + (y - y0) ** 2) / r_fil**2)
        dist = np.where(z < z_tip, z_tip - z, np.where(z > FIL_Z_TOP, z - FIL_Z_TOP, 0.0))
        body = 0.5 * np.exp(-(dist**2) / w**2)
        head = np.exp(-((z - z_tip) ** 2) / w**2)
        return g2 * np.minimum(1.0, body + head)

    xc, yc, zc = cell_centres(nx, ny, nz, h)
    xf = np.arange(nx + 1) * h
    yf = np.arange(ny + 1) * h
    zf = np.arange(nz + 1) * h
    grids = ((zc[:, None, None], yc[None, :, None], xf[None, None, :]),
             (zc[:, None, None], yf[None, :, None], xc[None, None, :]),
             (zf[:, None, None], yc[None, :, None], xc[None, None, :]))
    out = []
    for zz, yy, xx in grids:
        wgt = shape(xx, yy, zz)
        noise = rng.standard_normal(wgt.shape)
        noise *= D_NOISE_SIGMA
        noise -= 0.5 * D_NOISE_SIGMA**2
        np.exp(noise, out=noise)
        out.append(np.ascontiguousarray(D_GAS * (1.0 + (D_HEAD_RATIO - 1.0) * wgt) * noise))
    return tuple(out)


AMR_BOX_COARSE = 16   # coarse cells per box side along x and y (32 fine cells)
AMR_BOX_GAP = 1       # uncovered coarse cells between consecutive boxes along z
AMR_BOX_MARGIN = 4    # coarse cells the column extends beyond the filament's ends


def streamer_composite(n: int, seed: int = 0, box: int = AMR_BOX_COARSE):
    """A two-level composite problem around a seeded filament: the potential
    problem of streamer_set(n) on the base grid, refined (ratio 2) by a
    column of boxes of box x box x box coarse cells centred on the filament's
    axis, from AMR_BOX_MARGIN cells below its tip to as far above its top,
    AMR_BOX_GAP uncovered coarse cells between consecutive boxes, each box at
    least one coarse cell inside the domain.  The fine sources and
    permittivities are the same recipes (filament_source, slab_permittivity)
    on the 2n^3 grid, cut to the boxes; the fine source draws use seed + 1.

    Returns (base Problem, boxes as ((lo), (hi)) fine ranges x y z, f_fine,
    eps_fine)."""
    base = streamer_set(n, seed=seed)[0]
    z_tip = np.random.default_rng(seed).uniform(*FIL_TIP_RANGE)
    k_lo = max(1, int(np.floor(z_tip * n)) - AMR_BOX_MARGIN)
    k_hi = min(n - 1, int(np.ceil(FIL_Z_TOP * n)) + AMR_BOX_MARGIN)
    c0 = n // 2 - box // 2
    boxes = []
    k = k_lo
    while k + box <= k_hi or (not boxes and k + box <= n - 1):
        boxes.append(((2 * c0, 2 * c0, 2 * k), (2 * (c0 + box), 2 * (c0 + box), 2 * (k + box))))
        k += box + AMR_BOX_GAP
    rho_f = filament_source(2 * n, 2 * n, 2 * n, seed + 1)
    eps_f = slab_permittivity(2 * n, 2 * n, 2 * n)
    cut = lambda a, lo, hi: np.ascontiguousarray(a[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])
    f_fine = [cut(rho_f, lo, hi) for lo, hi in boxes]
    eps_fine = [cut(eps_f, lo, hi) for lo, hi in boxes]
    return base, boxes, f_fine, eps_fine
