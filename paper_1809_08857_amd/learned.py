"""ctypes binding of the C ABI in include/mgl.h (argument marshalling only):
the learned initial guess of the three screened photon-group solves.

Every function has the name of the C entry point it calls.  Device arrays
are torch tensors (contiguous, on the GPU: FP64 fields, FP32 targets
[z][y][x][3]); their pointers and the current torch stream go to
``libmgl.so``, whose HIP kernels do all the work.  There is no fallback: if
the library is missing or the GPU is absent the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np

from .mg import MgError, MG_OK, _stream_handle  # noqa: F401

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmgl.so")
WEIGHTS_DIR = os.path.join(PKG, "weights")

LAYER_NAMES = ("e0a", "e0b", "d0", "e1a", "e1b", "d1", "e2a", "e2b", "d2", "b3a", "b3b", "u2",
               "c2a", "c2b", "u1", "c1a", "c1b", "u0", "c0a", "c0b", "head")


class MglDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int)]


class MglAdam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float)]


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libmgl.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1809_08857_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    pP, pF, pD, pI = (ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_float),
                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int))
    sig = {
        "mgl_create": (I, [ctypes.POINTER(MglDesc), P, pP]),
        "mgl_destroy": (I, [P]),
        "mgl_last_error": (ctypes.c_char_p, []),
        "mgl_num_params": (ctypes.c_size_t, []),
        "mgl_init_params": (I, [P, ctypes.c_ulonglong]),
        "mgl_set_params": (I, [P, pF, ctypes.c_size_t]),
        "mgl_get_params": (I, [P, pF, ctypes.c_size_t]),
        "mgl_set_scales": (I, [P, pD]),
        "mgl_get_scales": (I, [P, pD]),
        "mgl_make_target": (I, [P, P, pP, pD, P, pD]),
        "mgl_train_step": (I, [P, I, pP, pP, ctypes.POINTER(MglAdam), pD]),
        "mgl_eval_loss": (I, [P, P, P, pD]),
        "mgl_get_grads": (I, [P, pF, ctypes.c_size_t]),
        "mgl_predict": (I, [P, P, pD, pP]),
        "mgl_save": (I, [P, ctypes.c_char_p]),
        "mgl_load": (I, [P, ctypes.c_char_p]),
        "mgl_read_tensor": (I, [P, I, I, pF, ctypes.c_size_t]),
        "mgl_tensor_shape": (I, [P, I, pI]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def mgl_last_error() -> str:
    return load().mgl_last_error().decode()


def _check(rc: int) -> int:
    if rc < 0:
        raise MgError(rc, mgl_last_error())
    return rc


def _dev(t, dtype_name: str) -> int:
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32}[dtype_name]
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != dt or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dt} CUDA tensor")
    return t.data_ptr()


def _ptrs(ts, dtype_name):
    arr = (ctypes.c_void_p * len(ts))(*[_dev(t, dtype_name) for t in ts])
    return arr


def _d3(v) -> ctypes.Array:
    return (ctypes.c_double * 3)(*[float(x) for x in v])


def mgl_num_params() -> int:
    return int(load().mgl_num_params())


def mgl_create(nx: int, ny: int, nz: int, stream=None) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    _check(load().mgl_create(ctypes.byref(MglDesc(nx, ny, nz)), _stream_handle(stream), ctypes.byref(out)))
    return out


def mgl_destroy(net) -> int:
    return _check(load().mgl_destroy(net))


def mgl_init_params(net, seed: int) -> int:
    return _check(load().mgl_init_params(net, int(seed)))


def mgl_set_params(net, theta: np.ndarray) -> int:
    a = np.ascontiguousarray(theta, dtype=np.float32)
    return _check(load().mgl_set_params(net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))


def mgl_get_params(net) -> np.ndarray:
    a = np.empty(mgl_num_params(), dtype=np.float32)
    _check(load().mgl_get_params(net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
    return a


def mgl_get_grads(net) -> np.ndarray:
    a = np.empty(mgl_num_params(), dtype=np.float32)
    _check(load().mgl_get_grads(net, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
    return a


def mgl_set_scales(net, scales: Sequence[float]) -> int:
    return _check(load().mgl_set_scales(net, _d3(scales)))


def mgl_get_scales(net) -> Tuple[float, float, float]:
    a = (ctypes.c_double * 3)()
    _check(load().mgl_get_scales(net, a))
    return tuple(a)


def mgl_make_target(net, s, psi: Sequence, kappa2: Sequence[float], t, want_max: bool = False):
    mx = (ctypes.c_double * 3)()
    _check(load().mgl_make_target(net, _dev(s, "f64"), _ptrs(psi, "f64"), _d3(kappa2), _dev(t, "f32"),
                                  mx if want_max else None))
    return tuple(mx) if want_max else None


def mgl_train_step(net, s_list: Sequence, t_list: Sequence, lr: Optional[float] = None,
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> float:
    if len(s_list) != len(t_list) or not s_list:
        raise ValueError("need matching, non-empty sample lists")
    opt = MglAdam(lr, beta1, beta2, eps) if lr is not None else None
    loss = ctypes.c_double()
    _check(load().mgl_train_step(net, len(s_list), _ptrs(s_list, "f64"), _ptrs(t_list, "f32"),
                                 ctypes.byref(opt) if opt is not None else None, ctypes.byref(loss)))
    return loss.value


def mgl_eval_loss(net, s, t) -> float:
    loss = ctypes.c_double()
    _check(load().mgl_eval_loss(net, _dev(s, "f64"), _dev(t, "f32"), ctypes.byref(loss)))
    return loss.value


def mgl_predict(net, s, kappa2: Sequence[float], guesses: Sequence) -> int:
    if len(guesses) != 3:
        raise ValueError("need three guess arrays")
    return _check(load().mgl_predict(net, _dev(s, "f64"), _d3(kappa2), _ptrs(guesses, "f64")))


def mgl_save(net, path: str) -> int:
    return _check(load().mgl_save(net, path.encode()))


def mgl_load(net, path: str) -> int:
    return _check(load().mgl_load(net, path.encode()))


def mgl_tensor_shape(net, layer: int) -> Tuple[int, int, int, int]:
    d = (ctypes.c_int * 4)()
    _check(load().mgl_tensor_shape(net, layer, d))
    return tuple(d)


def mgl_read_tensor(net, which: int, layer: int) -> np.ndarray:
    shape = mgl_tensor_shape(net, layer)
    a = np.empty(shape, dtype=np.float32)
    _check(load().mgl_read_tensor(net, which, layer, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
    return a


class Net:
    """Owning wrapper of one network on one grid (calls the mgl_* functions)."""

    def __init__(self, nx: int, ny: int, nz: int, stream=None):
        self.shape = (nz, ny, nx)
        self.net = mgl_create(nx, ny, nz, stream)

    def close(self):
        if self.net is not None:
            mgl_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
