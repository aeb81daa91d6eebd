"""ctypes binding of the C ABI in include/mg.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Device arrays
are passed as torch tensors (contiguous, float64, on the GPU); their data
pointers and the current torch stream go straight to the library, which does
all the work in its own HIP kernels.  There is no fallback: if libmg.so is
missing or the GPU is absent the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence, Tuple

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmg.so")

MG_OK, MG_NOT_CONVERGED = 0, 1
MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_EDIVERGED = -1, -2, -3, -4
MG_BC_DIRICHLET, MG_BC_NEUMANN = 0, 1
MG_FP64, MG_FP32_IR, MG_BF16_IR = 0, 1, 2
MG_GUESS = 1
MG_NUM_TILES = 6
MG_STORE_F64, MG_STORE_F32, MG_STORE_BF16 = 0, 1, 2
MG_OPT_CORRECTION_WEIGHT = 1

PRECISIONS = {"fp64": MG_FP64, "fp32": MG_FP32_IR, "bf16": MG_BF16_IR}


class MgDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("h", ctypes.c_double),
                ("precision", ctypes.c_int), ("nu1", ctypes.c_int), ("nu2", ctypes.c_int),
                ("bottom_max", ctypes.c_int), ("max_cycles", ctypes.c_int), ("rtol", ctypes.c_double)]


class MgBcs(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int * 6), ("value", ctypes.c_double * 6)]


class MgStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("rel_res0", ctypes.c_double), ("rel_res", ctypes.c_double),
                ("fell_back", ctypes.c_int), ("ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class MgaBox(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int * 3), ("hi", ctypes.c_int * 3)]


class MgError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libmg.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_08857_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I, D = ctypes.c_int, ctypes.c_double
    pI, pD = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    sig = {
        "mg_desc_default": (None, [ctypes.POINTER(MgDesc), I, I, I, D]),
        "mg_create": (I, [ctypes.POINTER(MgDesc), P, ctypes.POINTER(P)]),
        "mg_set_coeffs": (I, [P, P, D, ctypes.POINTER(MgBcs)]),
        "mg_solve": (I, [P, P, P, ctypes.c_uint, ctypes.POINTER(MgStats)]),
        "mg_solve_batched": (I, [I, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P), ctypes.c_uint,
                                 ctypes.POINTER(MgStats)]),
        "mg_destroy": (I, [P]),
        "mg_last_error": (ctypes.c_char_p, []),
        "mg_residual": (I, [P, P, P, P, pD, pD]),
        "mg_smooth": (I, [P, P, P, I]),
        "mg_prolong_add": (I, [P, I, P, P]),
        "mg_smooth_level": (I, [P, I, I, P, P, I, I, I]),
        "mg_set_face_coeffs": (I, [P, P, P, P, D, ctypes.POINTER(MgBcs)]),
        "mg_apply": (I, [P, D, D, P, P]),
        "mg_set_face_coeffs_diag": (I, [P, P, P, P, P, D, ctypes.POINTER(MgBcs)]),
        "mg_field": (I, [P, P, P, D, P, P, P, pD, pD, pD]),
        "mg_relaxation_substeps": (I, [D, D, D, pI]),
        "mg_tga_step": (I, [P, D, P, P, ctypes.c_uint, ctypes.POINTER(MgStats)]),
        "mg_residual_noalloc": (I, [ctypes.POINTER(MgDesc), P, D, ctypes.POINTER(MgBcs), P, P, P, pD, pD, P]),
        "mg_set_option": (I, [P, I, D]),
        "mg_num_levels": (I, [P]),
        "mg_level_dims": (I, [P, I, pI, pI, pI]),
        "mg_set_tiling": (I, [P, I, I]),
        "mg_tile_shape": (I, [I, pI, pI]),
        "mg_autotune": (I, [P, I, pI, pI, pD]),
        "mg_timing": (I, [P, I]),
        "mg_timing_read": (I, [P, ctypes.POINTER(ctypes.c_long), pD, pD, ctypes.POINTER(ctypes.c_char_p)]),
        "mga_create": (I, [ctypes.POINTER(MgDesc), I, ctypes.POINTER(MgaBox), P, ctypes.POINTER(P)]),
        "mga_set_coeffs": (I, [P, P, ctypes.POINTER(P), D, ctypes.POINTER(MgBcs)]),
        "mga_solve": (I, [P, P, ctypes.POINTER(P), P, ctypes.POINTER(P), ctypes.c_uint, ctypes.POINTER(MgStats)]),
        "mga_apply": (I, [P, P, ctypes.POINTER(P), P, ctypes.POINTER(P)]),
        "mga_destroy": (I, [P]),
        "mge_create": (I, [ctypes.POINTER(MgDesc), P, ctypes.POINTER(P)]),
        "mge_set_geometry": (I, [P, P, P, P, P, ctypes.c_long, ctypes.POINTER(ctypes.c_long), pD, P, D,
                                 ctypes.POINTER(MgBcs), P, D]),
        "mge_solve": (I, [P, P, P, ctypes.c_uint, ctypes.POINTER(MgStats)]),
        "mge_apply": (I, [P, P, P]),
        "mge_rhs": (I, [P, P, P]),
        "mge_timing": (I, [P, I]),
        "mge_timing_read": (I, [P, ctypes.POINTER(ctypes.c_long), pD, pD, ctypes.POINTER(ctypes.c_char_p)]),
        "mge_destroy": (I, [P]),
        "mga_timing": (I, [P, I]),
        "mga_timing_read": (I, [P, ctypes.POINTER(ctypes.c_long), pD, pD, ctypes.POINTER(ctypes.c_char_p)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch.Tensor")
    if t.device.type != "cuda" or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError("device arrays must be contiguous float64 CUDA tensors")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _check(rc: int) -> int:
    if rc < 0:
        raise MgError(rc, mg_last_error())
    return rc


def mg_last_error() -> str:
    return load().mg_last_error().decode()


def mg_desc_default(nx: int, ny: int, nz: int, h: float, **kw) -> MgDesc:
    d = MgDesc()
    load().mg_desc_default(ctypes.byref(d), nx, ny, nz, h)
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        setattr(d, k, v)
    return d


def make_bcs(types: Sequence, values: Sequence[float]) -> MgBcs:
    """types: 'D'/'N' or MG_BC_* per face (x-, x+, y-, y+, z-, z+)."""
    b = MgBcs()
    for f in range(6):
        t = types[f]
        if isinstance(t, str):
            t = MG_BC_DIRICHLET if t == "D" else MG_BC_NEUMANN
        b.type[f] = t
        b.value[f] = float(values[f])
    return b


def mg_create(desc: MgDesc, stream=None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(load().mg_create(ctypes.byref(desc), _stream_handle(stream), ctypes.byref(ctx)))
    return ctx


def mg_set_coeffs(ctx, eps, a: float, bcs: MgBcs) -> int:
    return _check(load().mg_set_coeffs(ctx, _ptr(eps), float(a), ctypes.byref(bcs)))


def mg_set_face_coeffs(ctx, bx, by, bz, a: float, bcs: MgBcs) -> int:
    return _check(load().mg_set_face_coeffs(ctx, _ptr(bx), _ptr(by), _ptr(bz), float(a), ctypes.byref(bcs)))


def mg_set_face_coeffs_diag(ctx, bx, by, bz, d, a: float, bcs: MgBcs) -> int:
    return _check(load().mg_set_face_coeffs_diag(ctx, _ptr(bx), _ptr(by), _ptr(bz), _ptr(d), float(a),
                                                  ctypes.byref(bcs)))


def mg_field(ctx, phi, sigma=None, eps0: float = 1.0, ex=None, ey=None, ez=None) -> Tuple[float, float, float]:
    """(max |E|, max |J|, dt_E); E components written to ex, ey, ez if given."""
    me, mj, dte = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load().mg_field(ctx, _ptr(phi), _ptr(sigma), float(eps0), _ptr(ex), _ptr(ey), _ptr(ez), ctypes.byref(me),
                           ctypes.byref(mj), ctypes.byref(dte)))
    return me.value, mj.value, dte.value


def mg_relaxation_substeps(dt_fine: float, dt_e: float, alpha: float) -> int:
    m = ctypes.c_int()
    _check(load().mg_relaxation_substeps(float(dt_fine), float(dt_e), float(alpha), ctypes.byref(m)))
    return m.value


def mg_apply(ctx, alpha: float, beta: float, x, y) -> int:
    return _check(load().mg_apply(ctx, float(alpha), float(beta), _ptr(x), _ptr(y)))


def mg_tga_step(ctx, dt: float, n, out, flags: int = 0) -> Tuple[int, List[MgStats]]:
    st = (MgStats * 2)()
    rc = _check(load().mg_tga_step(ctx, float(dt), _ptr(n), _ptr(out), flags, st))
    return rc, list(st)


def mg_solve(ctx, f, x, flags: int = 0) -> Tuple[int, MgStats]:
    st = MgStats()
    rc = _check(load().mg_solve(ctx, _ptr(f), _ptr(x), flags, ctypes.byref(st)))
    return rc, st


def mg_solve_batched(ctxs: Sequence, fs: Sequence, xs: Sequence, flags: int = 0) -> Tuple[int, List[MgStats]]:
    n = len(ctxs)
    P = ctypes.c_void_p
    carr = (P * n)(*[c.value if isinstance(c, P) else c for c in ctxs])
    farr = (P * n)(*[_ptr(t) for t in fs])
    xarr = (P * n)(*[_ptr(t) for t in xs])
    st = (MgStats * n)()
    rc = _check(load().mg_solve_batched(n, carr, farr, xarr, flags, st))
    return rc, list(st)


def mg_destroy(ctx) -> int:
    return _check(load().mg_destroy(ctx))


def mg_residual(ctx, f, x, r=None) -> Tuple[float, float]:
    rn, bn = ctypes.c_double(), ctypes.c_double()
    _check(load().mg_residual(ctx, _ptr(f), _ptr(x), _ptr(r), ctypes.byref(rn), ctypes.byref(bn)))
    return rn.value, bn.value


def mg_residual_noalloc(desc: MgDesc, eps, a: float, bcs: MgBcs, f, x, r=None, stream=None) -> Tuple[float, float]:
    rn, bn = ctypes.c_double(), ctypes.c_double()
    _check(load().mg_residual_noalloc(ctypes.byref(desc), _ptr(eps), float(a), ctypes.byref(bcs), _ptr(f), _ptr(x),
                                      _ptr(r), ctypes.byref(rn), ctypes.byref(bn), _stream_handle(stream)))
    return rn.value, bn.value


def mg_smooth(ctx, f, x, sweeps: int) -> int:
    return _check(load().mg_smooth(ctx, _ptr(f), _ptr(x), sweeps))


def mg_smooth_level(ctx, l: int, store: int, b, x, sweeps: int, tile: int = 0, zchunk: int = 0) -> int:
    return _check(load().mg_smooth_level(ctx, l, store, _ptr(b), _ptr(x), sweeps, tile, zchunk))


def mg_set_option(ctx, key: int, value: float) -> int:
    return _check(load().mg_set_option(ctx, key, float(value)))


def mg_prolong_add(ctx, l: int, e, u) -> int:
    return _check(load().mg_prolong_add(ctx, l, _ptr(e), _ptr(u)))


def mg_num_levels(ctx) -> int:
    return load().mg_num_levels(ctx)


def mg_level_dims(ctx, l: int) -> Tuple[int, int, int]:
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().mg_level_dims(ctx, l, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def mg_set_tiling(ctx, tile: int, zchunk: int) -> int:
    return _check(load().mg_set_tiling(ctx, tile, zchunk))


def mg_tile_shape(t: int) -> Tuple[int, int]:
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(load().mg_tile_shape(t, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def mg_autotune(ctx, reps: int = 5) -> Tuple[int, int, float]:
    t, z, us = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    _check(load().mg_autotune(ctx, reps, ctypes.byref(t), ctypes.byref(z), ctypes.byref(us)))
    return t.value, z.value, us.value


def mg_timing(ctx, enable: int) -> int:
    return _check(load().mg_timing(ctx, int(enable)))


def mg_timing_read(ctx) -> Tuple[int, float, str, float]:
    """(launches, total ms, kernel description, mean algorithmic bytes per launch)."""
    n, ms, by, k = ctypes.c_long(), ctypes.c_double(), ctypes.c_double(), ctypes.c_char_p()
    _check(load().mg_timing_read(ctx, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(k)))
    per = by.value / n.value if n.value else 0.0
    return n.value, ms.value, (k.value or b"").decode(), per


def _ptr_array(ts: Optional[Sequence]):
    if ts is None:
        return None
    return (ctypes.c_void_p * max(len(ts), 1))(*[_ptr(t) for t in ts])


def mga_create(desc: MgDesc, boxes: Sequence, stream=None) -> ctypes.c_void_p:
    """boxes: ((lo_x, lo_y, lo_z), (hi_x, hi_y, hi_z)) fine-cell ranges."""
    arr = (MgaBox * max(len(boxes), 1))()
    for q, (lo, hi) in enumerate(boxes):
        arr[q].lo[:] = [int(v) for v in lo]
        arr[q].hi[:] = [int(v) for v in hi]
    ctx = ctypes.c_void_p()
    _check(load().mga_create(ctypes.byref(desc), len(boxes), arr, _stream_handle(stream), ctypes.byref(ctx)))
    return ctx


def mga_set_coeffs(ctx, eps_base, eps_fine, a: float, bcs: MgBcs) -> int:
    return _check(load().mga_set_coeffs(ctx, _ptr(eps_base), _ptr_array(eps_fine), float(a), ctypes.byref(bcs)))


def mga_solve(ctx, f_base, f_fine: Sequence, x_base, x_fine: Sequence, flags: int = 0) -> Tuple[int, MgStats]:
    st = MgStats()
    rc = _check(load().mga_solve(ctx, _ptr(f_base), _ptr_array(f_fine), _ptr(x_base), _ptr_array(x_fine), flags,
                                 ctypes.byref(st)))
    return rc, st


def mga_apply(ctx, x_base, x_fine: Sequence, y_base, y_fine: Sequence) -> int:
    return _check(load().mga_apply(ctx, _ptr(x_base), _ptr_array(x_fine), _ptr(y_base), _ptr_array(y_fine)))


def mga_timing(ctx, enable: int) -> int:
    return _check(load().mga_timing(ctx, int(enable)))


def mga_timing_read(ctx) -> Tuple[int, float, str, float]:
    """(launches, ms, kernel, algorithmic bytes per launch) of the base grid's timed smoother."""
    n, ms, by, k = ctypes.c_long(), ctypes.c_double(), ctypes.c_double(), ctypes.c_char_p()
    _check(load().mga_timing_read(ctx, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(k)))
    per = by.value / n.value if n.value else 0.0
    return n.value, ms.value, (k.value or b"").decode(), per


def mga_destroy(ctx) -> int:
    return _check(load().mga_destroy(ctx))


def mge_create(desc: MgDesc, stream=None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(load().mge_create(ctypes.byref(desc), _stream_handle(stream), ctypes.byref(ctx)))
    return ctx


def mge_set_geometry(ctx, kappa, ax, ay, az, bidx, boff, eps, a: float, bcs: MgBcs, g=None, g_eb: float = 0.0) -> int:
    """bidx (int64) and boff ([nb][3] float64) are host numpy arrays; the others device tensors."""
    import numpy as np
    bi = np.ascontiguousarray(bidx, dtype=np.int64)
    bo = np.ascontiguousarray(boff, dtype=np.float64).reshape(-1)
    return _check(load().mge_set_geometry(
        ctx, _ptr(kappa), _ptr(ax), _ptr(ay), _ptr(az), bi.size,
        bi.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), bo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        _ptr(eps), float(a), ctypes.byref(bcs), _ptr(g), float(g_eb)))


def mge_solve(ctx, f, x, flags: int = 0) -> Tuple[int, MgStats]:
    st = MgStats()
    rc = _check(load().mge_solve(ctx, _ptr(f), _ptr(x), flags, ctypes.byref(st)))
    return rc, st


def mge_apply(ctx, x, y) -> int:
    return _check(load().mge_apply(ctx, _ptr(x), _ptr(y)))


def mge_rhs(ctx, f, b) -> int:
    return _check(load().mge_rhs(ctx, _ptr(f), _ptr(b)))


def mge_timing(ctx, enable: int) -> int:
    return _check(load().mge_timing(ctx, int(enable)))


def mge_timing_read(ctx) -> Tuple[int, float, str, float]:
    n, ms, by, k = ctypes.c_long(), ctypes.c_double(), ctypes.c_double(), ctypes.c_char_p()
    _check(load().mge_timing_read(ctx, ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by), ctypes.byref(k)))
    per = by.value / n.value if n.value else 0.0
    return n.value, ms.value, (k.value or b"").decode(), per


def mge_destroy(ctx) -> int:
    return _check(load().mge_destroy(ctx))


class Solver:
    """Owns one context: create + set_coeffs on construction, destroy on close."""

    def __init__(self, nx, ny, nz, h, *, eps=None, faces=None, a=0.0, bc_types=("N",) * 6,
                 bc_values=(0.0,) * 6, stream=None, **desc_kw):
        self.desc = mg_desc_default(nx, ny, nz, h, **desc_kw)
        self.ctx = mg_create(self.desc, stream)
        try:
            if faces is not None:
                mg_set_face_coeffs(self.ctx, *faces, a, make_bcs(bc_types, bc_values))
            else:
                mg_set_coeffs(self.ctx, eps, a, make_bcs(bc_types, bc_values))
        except Exception:
            mg_destroy(self.ctx)
            self.ctx = None
            raise

    def solve(self, f, x, flags: int = 0):
        return mg_solve(self.ctx, f, x, flags)

    def residual(self, f, x, r=None):
        return mg_residual(self.ctx, f, x, r)

    def tga_step(self, dt, n, out, flags: int = 0):
        return mg_tga_step(self.ctx, dt, n, out, flags)

    def close(self):
        if self.ctx is not None:
            mg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
