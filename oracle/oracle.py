"""Front end of the CPU FP64 oracle (test infrastructure only).

The heavy lifting is plain C in ``mg_oracle.c``; this module compiles it with
gcc, marshals NumPy arrays through ctypes and adds a pure-Python dense
assembly of the same discrete operator for tiny grids (brute-force checks).

Discrete problem (paper Sec. 2: potential and radiative-transfer equations,
second-order cell-centred finite volumes; see mg_oracle.c for the formulas):

    (A u)_P = a u_P + h^-2 [ sum_interior beta_f (u_P - u_N) + sum_Dirichlet 2 beta_P u_P ]
    b_P     = f_P + h^-2 sum_Dirichlet 2 beta_P g
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
# MG_ORACLE_NATIVE=1: a build tuned for the host it runs on (-O3 -march=native),
# for timing the oracle on that host; the default build is portable.
_NATIVE = os.environ.get("MG_ORACLE_NATIVE") == "1"
_LIB_PATH = os.path.join(_HERE, "liboracle_native.so" if _NATIVE else "liboracle.so")
_lock = threading.Lock()
_lib = None

DIRICHLET, NEUMANN = 0, 1


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (OpenMP for the CG vector loops)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        opt = ["-O3", "-march=native"] if _NATIVE else ["-O2", "-march=x86-64-v3"]
        cmd = ["gcc", *opt, "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-o", tmp,
               _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
                build(force=True)
            lib = ctypes.CDLL(_LIB_PATH)
            dp = ctypes.POINTER(ctypes.c_double)
            ip = ctypes.POINTER(ctypes.c_int)
            c_int, c_dbl = ctypes.c_int, ctypes.c_double
            lib.orc_apply.argtypes = [c_int, c_int, c_int, c_dbl, c_dbl, dp, ip, dp, dp]
            lib.orc_apply.restype = None
            lib.orc_rhs.argtypes = [c_int, c_int, c_int, c_dbl, c_dbl, dp, ip, dp, dp, dp]
            lib.orc_rhs.restype = None
            lib.orc_residual.argtypes = [c_int, c_int, c_int, c_dbl, c_dbl, dp, ip, dp, dp, dp, dp, dp]
            lib.orc_residual.restype = c_dbl
            lib.orc_cg.argtypes = [c_int, c_int, c_int, c_dbl, c_dbl, dp, ip, dp, dp, dp, c_dbl, c_int, dp]
            lib.orc_cg.restype = c_int
            lib.orc_vcycle_solve.argtypes = [c_int, c_int, c_int, c_dbl, c_dbl, dp, ip, dp, dp, dp, c_dbl,
                                             c_int, c_int, c_int, c_int, dp, dp]
            lib.orc_vcycle_solve.restype = c_int
            lib.orc_rbgs.argtypes = [c_int, c_int, c_int, c_dbl, c_dbl, dp, ip, dp, dp, dp, c_int]
            lib.orc_rbgs.restype = None
            lib.orc_threads.argtypes = []
            lib.orc_threads.restype = c_int
            lib.orc_prolong_add.argtypes = [c_int, c_int, c_int, ip, dp, dp]
            lib.orc_prolong_add.restype = None
            for name, base in (("orc_apply_faces", [c_int, c_int, c_int, c_dbl, c_dbl, dp, dp, dp, ip, dp, dp]),
                               ("orc_rhs_faces", [c_int, c_int, c_int, c_dbl, c_dbl, dp, dp, dp, ip, dp, dp, dp]),
                               ("orc_residual_faces", [c_int, c_int, c_int, c_dbl, c_dbl, dp, dp, dp, ip, dp, dp, dp,
                                                       dp, dp]),
                               ("orc_cg_faces", [c_int, c_int, c_int, c_dbl, c_dbl, dp, dp, dp, ip, dp, dp, dp,
                                                 c_dbl, c_int, dp]),
                               ("orc_vcycle_solve_faces", [c_int, c_int, c_int, c_dbl, c_dbl, dp, dp, dp, ip, dp,
                                                           dp, dp, c_dbl, c_int, c_int, c_int, c_int, dp, dp]),
                               ("orc_rbgs_faces", [c_int, c_int, c_int, c_dbl, c_dbl, dp, dp, dp, ip, dp, dp, dp,
                                                   c_int])):
                getattr(lib, name).argtypes = base
            lib.orc_apply_faces.restype = None
            lib.orc_rhs_faces.restype = None
            lib.orc_residual_faces.restype = c_dbl
            lib.orc_cg_faces.restype = c_int
            lib.orc_vcycle_solve_faces.restype = c_int
            lib.orc_rbgs_faces.restype = None
            lib.orc_rbgs_level.argtypes = [c_int, c_int, c_int, c_dbl, c_dbl, dp, ip, c_int, dp, dp, c_int]
            lib.orc_rbgs_level.restype = c_int
            lib.orc_num_levels.argtypes = [c_int, c_int, c_int, c_int]
            lib.orc_num_levels.restype = c_int
            _lib = lib
    return _lib


def _dp(arr: Optional[np.ndarray]):
    if arr is None:
        return ctypes.POINTER(ctypes.c_double)()
    assert arr.dtype == np.float64 and arr.flags.c_contiguous
    return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _prob_args(p):
    bct = np.array([DIRICHLET if t == "D" else NEUMANN for t in p.bc_types()], dtype=np.int32)
    g = np.array(p.bc_values(), dtype=np.float64)
    eps = None if p.eps is None else np.ascontiguousarray(p.eps, dtype=np.float64)
    return bct, g, eps


def _ip(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _faces(p):
    """The face arrays of a face-coefficient problem (contiguous FP64), or None."""
    if getattr(p, "faces", None) is None:
        return None
    if p.eps is not None:
        raise ValueError("a problem has either a cell coefficient or face coefficients")
    bx, by, bz = (np.ascontiguousarray(a, dtype=np.float64) for a in p.faces)
    assert bx.shape == (p.nz, p.ny, p.nx + 1) and by.shape == (p.nz, p.ny + 1, p.nx)
    assert bz.shape == (p.nz + 1, p.ny, p.nx)
    return bx, by, bz


def _call(lib, name, p, eps, *rest):
    """Call orc_<name>(dims, h, a, coefficient, ...) in the cell or face form."""
    fc = _faces(p)
    if fc is None:
        return getattr(lib, "orc_" + name)(p.nx, p.ny, p.nz, p.h, p.a, _dp(eps), *rest)
    return getattr(lib, "orc_" + name + "_faces")(p.nx, p.ny, p.nz, p.h, p.a, *(_dp(a) for a in fc), *rest)


def apply(p, u: np.ndarray) -> np.ndarray:
    """A u with homogeneous boundary values."""
    lib = _load()
    bct, _, eps = _prob_args(p)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.empty_like(u)
    _call(lib, "apply", p, eps, _ip(bct), _dp(u), _dp(out))
    return out


def rhs(p) -> np.ndarray:
    """b = f plus the Dirichlet boundary terms."""
    lib = _load()
    bct, g, eps = _prob_args(p)
    f = np.ascontiguousarray(p.f, dtype=np.float64)
    b = np.empty_like(f)
    _call(lib, "rhs", p, eps, _ip(bct), _dp(g), _dp(f), _dp(b))
    return b


def residual(p, u: np.ndarray) -> Tuple[np.ndarray, float, float]:
    """(r = b - A u, ||r||_2, ||b||_2)."""
    lib = _load()
    bct, g, eps = _prob_args(p)
    f = np.ascontiguousarray(p.f, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    r = np.empty_like(f)
    bn = ctypes.c_double(0.0)
    rn = _call(lib, "residual", p, eps, _ip(bct), _dp(g), _dp(f), _dp(u), _dp(r), ctypes.byref(bn))
    return r, float(rn), float(bn.value)


def solve_cg(p, rtol: float = 1e-13, maxit: int = 200000, u0: Optional[np.ndarray] = None):
    """Plain CG; returns (u, iterations, relative residual)."""
    lib = _load()
    bct, g, eps = _prob_args(p)
    f = np.ascontiguousarray(p.f, dtype=np.float64)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, order="C")
    rel = ctypes.c_double(0.0)
    it = _call(lib, "cg", p, eps, _ip(bct), _dp(g), _dp(f), _dp(u), rtol, maxit, ctypes.byref(rel))
    return u, int(it), float(rel.value)


def solve_vcycle(p, rtol: float = 1e-13, max_cycles: int = 100, nu1: int = 2, nu2: int = 2,
                 coarsest_max: int = 2, u0: Optional[np.ndarray] = None, history: bool = False):
    """Lexicographic Gauss-Seidel V(nu1,nu2) cycles; returns (u, cycles, relres[, history])."""
    lib = _load()
    bct, g, eps = _prob_args(p)
    f = np.ascontiguousarray(p.f, dtype=np.float64)
    u = np.zeros_like(f) if u0 is None else np.array(u0, dtype=np.float64, order="C")
    rel = ctypes.c_double(0.0)
    hist = np.zeros(max_cycles, dtype=np.float64)
    c = _call(lib, "vcycle_solve", p, eps, _ip(bct), _dp(g), _dp(f), _dp(u), rtol, max_cycles, nu1, nu2,
              coarsest_max, ctypes.byref(rel), _dp(hist))
    if history:
        return u, int(c), float(rel.value), hist[:c].copy()
    return u, int(c), float(rel.value)


def rbgs(p, u: np.ndarray, sweeps: int = 1) -> np.ndarray:
    """Red-black Gauss-Seidel sweeps (red = (i+j+k) even first) from u."""
    lib = _load()
    bct, g, eps = _prob_args(p)
    f = np.ascontiguousarray(p.f, dtype=np.float64)
    out = np.array(u, dtype=np.float64, order="C")
    _call(lib, "rbgs", p, eps, _ip(bct), _dp(g), _dp(f), _dp(out), sweeps)
    return out


def level_dims(p, level: int) -> Tuple[int, int, int]:
    """(nx, ny, nz) of level `level` of the hierarchy that halves every axis
    while all are even and the largest exceeds 1."""
    nx, ny, nz = p.nx, p.ny, p.nz
    for _ in range(level):
        if nx % 2 or ny % 2 or nz % 2 or max(nx, ny, nz) <= 1:
            raise ValueError(f"level {level} does not exist for {p.nx}x{p.ny}x{p.nz}")
        nx, ny, nz = nx // 2, ny // 2, nz // 2
    return nx, ny, nz


def rbgs_level(p, level: int, b: np.ndarray, u: np.ndarray, sweeps: int = 1) -> np.ndarray:
    """Red-black sweeps of the homogeneous equation A_l u = b of hierarchy
    level `level` (level 0: the finest operator without boundary values)."""
    lib = _load()
    if _faces(p) is not None:
        raise ValueError("rbgs_level takes cell-coefficient problems")
    bct, _, eps = _prob_args(p)
    nx, ny, nz = level_dims(p, level)
    b = np.ascontiguousarray(b, dtype=np.float64)
    out = np.array(u, dtype=np.float64, order="C")
    assert b.shape == (nz, ny, nx) and out.shape == (nz, ny, nx)
    nlev = lib.orc_rbgs_level(p.nx, p.ny, p.nz, p.h, p.a, _dp(eps), _ip(bct), level, _dp(b), _dp(out), sweeps)
    assert level < nlev
    return out


def solve_reference(p, rtol: float = 1e-13) -> np.ndarray:
    """u* to relative residual rtol (V-cycle oracle; CG finishes the job if
    the V-cycle stalls above rtol)."""
    u, _, rel = solve_vcycle(p, rtol=rtol, max_cycles=200)
    if rel > rtol:
        u, _, rel = solve_cg(p, rtol=rtol, u0=u)
    return u


def prolong_add(e: np.ndarray, u: np.ndarray, bc_types: Sequence[str]) -> np.ndarray:
    """u + P e: cell-centred trilinear prolongation of the coarse field e
    (shape (nzc, nyc, nxc)) onto the fine grid of twice its size per axis,
    ghost values reflected across the box faces (negated at Dirichlet faces,
    where the correction vanishes)."""
    lib = _load()
    e = np.ascontiguousarray(e, dtype=np.float64)
    nzc, nyc, nxc = e.shape
    out = np.array(u, dtype=np.float64, copy=True, order="C")
    assert out.shape == (2 * nzc, 2 * nyc, 2 * nxc)
    bct = np.array([DIRICHLET if t == "D" else NEUMANN for t in bc_types], dtype=np.int32)
    lib.orc_prolong_add(nxc, nyc, nzc, _ip(bct), _dp(e), _dp(out))
    return out


def threads() -> int:
    """Threads used by the oracle's OpenMP loops."""
    return int(_load().orc_threads())


def num_levels(nx: int, ny: int, nz: int, coarsest_max: int = 2) -> int:
    return int(_load().orc_num_levels(nx, ny, nz, coarsest_max))


# ---------------------------------------------------------------- dense


def dense_matrix(p) -> Tuple[np.ndarray, np.ndarray]:
    """Assemble (A, b) cell by cell from the definition, in pure Python.

    Written independently of mg_oracle.c: it walks the six neighbours of
    every cell and adds the face term of the second-order cell-centred
    discretisation (interior faces: the harmonic mean of the two cell
    coefficients, or the given face coefficient; Dirichlet faces: the linear
    ghost with the boundary cell's coefficient, or the given boundary face
    coefficient; zero Neumann flux).  Only for tiny grids (n <= ~2000)."""
    nx, ny, nz = p.nx, p.ny, p.nz
    n = nx * ny * nz
    A = np.zeros((n, n))
    b = np.array(p.f, dtype=np.float64).reshape(-1).copy()
    ih2 = 1.0 / (p.h * p.h)
    faces = getattr(p, "faces", None)
    beta = np.ones((nz, ny, nx)) if p.eps is None else np.asarray(p.eps, dtype=np.float64)
    types = p.bc_types()
    vals = p.bc_values()
    steps = [(-1, 0, 0, 0), (1, 0, 0, 1), (0, -1, 0, 2), (0, 1, 0, 3), (0, 0, -1, 4), (0, 0, 1, 5)]

    def lin(i, j, k):
        return (k * ny + j) * nx + i

    def face(i, j, k, face_id):
        """Given face coefficient on side face_id of cell (i, j, k)."""
        bx, by, bz = faces
        if face_id < 2:
            return bx[k, j, i + (face_id == 1)]
        if face_id < 4:
            return by[k, j + (face_id == 3), i]
        return bz[k + (face_id == 5), j, i]

    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                P = lin(i, j, k)
                A[P, P] += p.a
                bP = beta[k, j, i]
                for di, dj, dk, fid in steps:
                    ii, jj, kk = i + di, j + dj, k + dk
                    if 0 <= ii < nx and 0 <= jj < ny and 0 <= kk < nz:
                        if faces is not None:
                            bf = face(i, j, k, fid)
                        else:
                            bN = beta[kk, jj, ii]
                            bf = 2.0 * bP * bN / (bP + bN)
                        A[P, P] += ih2 * bf
                        A[P, lin(ii, jj, kk)] -= ih2 * bf
                    elif types[fid] == "D":
                        bb = face(i, j, k, fid) if faces is not None else bP
                        A[P, P] += 2.0 * ih2 * bb
                        b[P] += 2.0 * ih2 * bb * vals[fid]
    return A, b


def dense_solve(p) -> np.ndarray:
    A, b = dense_matrix(p)
    return np.linalg.solve(A, b).reshape(p.nz, p.ny, p.nx)


# ---------------------------------------------------------------- TGA


def tga_coefficients(dt: float, eps: float = 1e-6) -> Tuple[float, float, float]:
    """(mu1, mu2, mu3) of the implicit diffusion advance of paper Sec. 2.1,
    step (vi), Eq. (tga): (I - mu1 L)(I - mu2 L) n_new = (I + mu3 L) n.

    The paper takes the coefficients from its software's documentation; this
    is the Twizell-Gumel-Arigu choice (Twizell, Gumel & Arigu 1996): with
    q = 2 - sqrt(2) - eps and r = sqrt(q^2 - 4q + 2) (real for eps > 0),
    mu1 = (q - r)/2 dt, mu2 = (q + r)/2 dt, mu3 = (1 - q) dt.  The amplification
    (1 + mu3 z)/((1 - mu1 z)(1 - mu2 z)) of an eigenvalue z dt of L then equals
    exp(z dt) to second order and tends to 0 as z dt -> -infinity."""
    q = 2.0 - np.sqrt(2.0) - eps
    r = np.sqrt(q * q - 4.0 * q + 2.0)
    return 0.5 * (q - r) * dt, 0.5 * (q + r) * dt, (1.0 - q) * dt


def tga_step(faces, h: float, dt: float, n: np.ndarray, eps: float = 1e-6, rtol: float = 1e-13) -> np.ndarray:
    """One TGA diffusion advance of n (Eq. (tga)) with the face diffusion
    coefficients `faces` = (bx, by, bz) and zero flux on every box face (the
    diffusion solves of Sec. 2, item (ii)).  L u = div(D grad u) is the
    operator A of a = 0 with a minus sign.  First (I - mu1 L) y = (I + mu3 L) n,
    then (I - mu2 L) n_new = y; each Helmholtz equation is solved by the
    oracle in the form (1/mu) u - div(D grad u) = rhs / mu."""
    from synth.problems import Problem
    nz, ny, nx = n.shape
    mu1, mu2, mu3 = tga_coefficients(dt, eps)
    neu = (("N", 0.0),) * 6

    def prob(a, f):
        return Problem(nx, ny, nz, h, a, np.ascontiguousarray(f), None, neu, "tga", faces=faces)

    Ln = -apply(prob(0.0, n), n)
    y = solve_reference(prob(1.0 / mu1, (n + mu3 * Ln) / mu1), rtol)
    return solve_reference(prob(1.0 / mu2, y / mu2), rtol)


# ---------------------------------------------------------------- field, relaxation time


def field(p, phi: np.ndarray) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """E = -grad(phi) at the cell centres by central differences over two
    cells (paper Sec. 2: the field follows from the potential), with the
    ghost values of the discretisation beyond the box: 2g - phi_P beyond a
    Dirichlet face (value g), phi_P beyond a Neumann face.  Returns
    (Ex, Ey, Ez), each [nz][ny][nx]."""
    phi = np.asarray(phi, dtype=np.float64)
    types, vals = p.bc_types(), p.bc_values()
    out = []
    for axis, (lo, hi) in zip((2, 1, 0), ((0, 1), (2, 3), (4, 5))):
        first = np.take(phi, [0], axis=axis)
        last = np.take(phi, [phi.shape[axis] - 1], axis=axis)
        g_lo = 2.0 * vals[lo] - first if types[lo] == "D" else first
        g_hi = 2.0 * vals[hi] - last if types[hi] == "D" else last
        ext = np.concatenate([g_lo, phi, g_hi], axis=axis)
        n = phi.shape[axis]
        fwd = np.take(ext, np.arange(2, n + 2), axis=axis)
        bwd = np.take(ext, np.arange(0, n), axis=axis)
        out.append(-(fwd - bwd) / (2.0 * p.h))
    return out[0], out[1], out[2]


def relaxation_time(p, phi: np.ndarray, sigma: np.ndarray, eps0: float = 1.0):
    """(max |E|, max |J|, dt_E) with J = sigma E (the drift current of a
    conductivity sigma) and the dielectric relaxation time of the paper's
    time-step table, dt_E = eps0 |E| / |J|, taken with the largest values
    over the grid (one step size for the whole domain)."""
    ex, ey, ez = field(p, phi)
    emag = np.sqrt(ex * ex + ey * ey + ez * ez)
    jmax = float(np.max(np.asarray(sigma) * emag))
    emax = float(np.max(emag))
    return emax, jmax, (eps0 * emax / jmax if jmax > 0 else np.inf)
