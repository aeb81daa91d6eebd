"""Host-side checks of the C ABI that need no GPU: the library loads, every
entry point declared in include/*.h is exported, and argument validation
rejects bad descriptors before any device work."""
import ctypes
import os
import re

import pytest

from paper_1809_08857_amd import build as mgbuild
from paper_1809_08857_amd import mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-zA-Z_][\w\s\*]*?\b((?:mg|mgl|mga|mge)_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mg.LIB_PATH):
        mgbuild.build()
    return mg.load()


@pytest.mark.parametrize("header,libfile", [("mg.h", "libmg.so"), ("mgl.h", "libmgl.so"), ("mga.h", "libmg.so"),
                                                ("mge.h", "libmg.so")])
def test_every_declared_symbol_is_exported(header, libfile):
    names = _declared(header)
    assert len(names) >= 5
    so = ctypes.CDLL(os.path.join(ROOT, "paper_1809_08857_amd", libfile))
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing


def test_desc_default(lib):
    d = mg.mg_desc_default(32, 16, 8, 0.5)
    assert (d.nx, d.ny, d.nz, d.h) == (32, 16, 8, 0.5)
    assert (d.precision, d.nu1, d.nu2, d.bottom_max, d.max_cycles) == (mg.MG_FP64, 2, 2, 16, 50)
    assert d.rtol == 1e-10


@pytest.mark.parametrize("field,value", [("nx", 0), ("h", 0.0), ("h", -1.0), ("precision", 7), ("nu1", -1),
                                         ("nu2", 9), ("bottom_max", 1), ("bottom_max", 17), ("max_cycles", 0),
                                         ("rtol", 0.0), ("rtol", 2.0)])
def test_create_rejects_bad_desc(lib, field, value):
    d = mg.mg_desc_default(32, 32, 32, 1 / 32)
    setattr(d, field, value)
    ctx = ctypes.c_void_p(123)
    rc = lib.mg_create(ctypes.byref(d), None, ctypes.byref(ctx))
    assert rc == mg.MG_EINVAL and ctx.value is None
    assert mg.mg_last_error().startswith("mg_create")


@pytest.mark.parametrize("dims", [(33, 32, 32), (34, 34, 34), (64, 48, 17)])
def test_create_rejects_uncoarsenable_grid(lib, dims):
    d = mg.mg_desc_default(*dims, 0.1)
    ctx = ctypes.c_void_p()
    assert lib.mg_create(ctypes.byref(d), None, ctypes.byref(ctx)) == mg.MG_EINVAL
    assert "bottom_max" in mg.mg_last_error()


def test_null_arguments(lib):
    assert lib.mg_solve(None, None, None, 0, None) == mg.MG_EINVAL
    assert lib.mg_set_coeffs(None, None, 0.0, None) == mg.MG_EINVAL
    assert lib.mg_destroy(None) == mg.MG_OK
    assert lib.mg_solve_batched(-1, None, None, None, 0, None) == mg.MG_EINVAL
    assert lib.mg_residual(None, None, None, None, None, None) == mg.MG_EINVAL
    assert lib.mg_num_levels(None) == 0


def test_tile_shapes(lib):
    shapes = [mg.mg_tile_shape(t) for t in range(1, mg.MG_NUM_TILES + 1)]
    assert len(set(shapes)) == mg.MG_NUM_TILES
    for tx, ty in shapes:
        assert tx % 2 == 0 and tx * ty // 2 in (64, 128, 256, 512)
    with pytest.raises(mg.MgError):
        mg.mg_tile_shape(0)


def test_learned_guess_parameter_count_matches_the_oracle():
    """The flat parameter layout is an interface shared by the library and
    the oracle: both must count the same parameters."""
    from oracle import nn_oracle
    from paper_1809_08857_amd import learned
    if not os.path.exists(learned.LIB_PATH):
        mgbuild.build()
    assert learned.mgl_num_params() == nn_oracle.num_params()


@pytest.mark.parametrize("dims", [(12, 16, 16), (16, 16, 4), (0, 8, 8), (8, 8, 20)])
def test_learned_guess_rejects_grids_that_do_not_coarsen(dims):
    from paper_1809_08857_amd import learned
    lib = learned.load()
    out = ctypes.c_void_p(5)
    rc = lib.mgl_create(ctypes.byref(learned.MglDesc(*dims)), None, ctypes.byref(out))
    assert rc == mg.MG_EINVAL and out.value is None
    assert learned.mgl_last_error().startswith("mgl_create")


def test_learned_guess_null_arguments():
    from paper_1809_08857_amd import learned
    lib = learned.load()
    assert lib.mgl_set_params(None, None, 0) == mg.MG_EINVAL
    assert lib.mgl_predict(None, None, None, None) == mg.MG_EINVAL
    assert lib.mgl_destroy(None) == mg.MG_OK


def test_relaxation_substeps(lib):
    """m = floor(alpha dt_E / dt_fine), at least 1 (the host side of the
    multirate schedule; no device work)."""
    m = ctypes.c_int()
    assert lib.mg_relaxation_substeps(ctypes.c_double(1e-3), ctypes.c_double(2.5e-2), ctypes.c_double(1.0),
                                      ctypes.byref(m)) == 0 and m.value == 25
    assert lib.mg_relaxation_substeps(ctypes.c_double(1e-3), ctypes.c_double(2.5e-2), ctypes.c_double(0.1),
                                      ctypes.byref(m)) == 0 and m.value == 2
    assert lib.mg_relaxation_substeps(ctypes.c_double(1.0), ctypes.c_double(0.1), ctypes.c_double(1.0),
                                      ctypes.byref(m)) == 0 and m.value == 1
    assert lib.mg_relaxation_substeps(ctypes.c_double(1.0), ctypes.c_double(float("inf")), ctypes.c_double(1.0),
                                      ctypes.byref(m)) == 0 and m.value == 1000000000
    assert lib.mg_relaxation_substeps(ctypes.c_double(0.0), ctypes.c_double(1.0), ctypes.c_double(1.0),
                                      ctypes.byref(m)) == -1


@pytest.mark.parametrize("boxes,why", [
    ([((0, 4, 4), (8, 12, 12))], "inside the domain"),
    ([((4, 4, 4), (12, 12, 13))], "even"),
    ([((4, 4, 4), (4, 12, 12))], "even"),
    ([((4, 4, 4), (10, 10, 10)), ((10, 4, 4), (16, 10, 10))], "apart"),
    ([((4, 4, 4), (10, 10, 10)), ((6, 6, 6), (8, 8, 8))], "apart"),
])
def test_mga_create_rejects_bad_boxes(lib, boxes, why):
    d = mg.mg_desc_default(16, 16, 16, 1 / 16)
    with pytest.raises(mg.MgError) as e:
        mg.mga_create(d, boxes, stream=_NoStream())
    assert e.value.code == mg.MG_EINVAL and why in mg.mg_last_error()
    assert mg.mg_last_error().startswith("mga_create")


def test_mga_create_rejects_low_precision(lib):
    d = mg.mg_desc_default(16, 16, 16, 1 / 16)
    d.precision = mg.MG_FP32_IR
    with pytest.raises(mg.MgError):
        mg.mga_create(d, [((4, 4, 4), (12, 12, 12))], stream=_NoStream())
    assert "MG_FP64" in mg.mg_last_error()


class _NoStream:
    cuda_stream = None
