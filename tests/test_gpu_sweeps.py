"""Per-kernel parity of the red-black sweeps that the solves run below the
finest FP64 level: the FP32 and BF16 storage sweeps of the mixed-precision
inner cycle (level 0 and the coarse levels), and the FP64 stored-face
sweeps of the coarse levels, each against the oracle's red-black sweep of
the same level equation (paper Sec. 2, item (ii)), through the C ABI call
mg_smooth_level.

Both sides start from the same values rounded to the storage type (x and
the right-hand side b).  One sweep in storage precision computes each new
value in FP32 from FP32 copies of the coefficients and rounds it to the
storage type once, so the bar per entry is the storage type's unit roundoff
(2^-8 relative for BF16, 2^-24 for FP32: half a unit in the last place of
a value at the bottom of its binade; to 1 % over that)
plus the FP32 arithmetic of the update (4e-6 of the field's largest value);
FP64 stored-face sweeps agree to 1e-12 of the largest value.  Chunks of
1, 3, 8 and 9 planes are shorter and longer than the FP32/BF16 plane ring
(8 slots); odd and even row lengths take different load paths."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import dev, make_solver

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1809_08857_amd import mg  # noqa: E402

STORE = {"fp32": mg.MG_STORE_F32, "bf16": mg.MG_STORE_BF16}
HALF_ULP = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -8}  # unit roundoff: 2^-p, p = 24 / 8 significant bits


def _round(a, prec):
    """The library's conversion: FP64 -> FP32 (-> BF16), to nearest even."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(torch.float32)
    if prec == "bf16":
        t = t.to(torch.bfloat16)
    return t.to(torch.float64).numpy()


def _problem(kind, dims, seed):
    nx, ny, nz = dims
    if kind == "const":
        return synth.random_problem(nx, ny, nz, seed, variable_eps=False, a=37.0)
    return synth.random_problem(nx, ny, nz, seed, variable_eps=True, a=0.0)


CASES = [  # (kind, fine dims, level)
    ("const", (48, 20, 40), 0),
    ("const", (15, 14, 16), 0),    # odd rows (a grid the bottom solver handles alone)
    ("cell", (48, 20, 40), 0),
    ("cell", (15, 14, 16), 0),     # odd rows
    ("cell", (48, 20, 40), 1),     # stored faces (FP32 copies of the averaged faces)
    ("const", (48, 20, 40), 1),
    ("cell", (128, 64, 96), 2),    # stored faces two levels down
]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("zchunk", [1, 3, 8, 9])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_lowp_sweep_parity(prec, zchunk, case):
    kind, dims, level = CASES[case]
    p = _problem(kind, dims, 40 + case)
    print(f"lowp sweep {prec} {kind} {dims} level {level} zchunk {zchunk}", flush=True)
    s = make_solver(p, precision=prec)
    try:
        lx, ly, lz = mg.mg_level_dims(s.ctx, level)
        assert (lx, ly, lz) == oracle.level_dims(p, level)
        rng = np.random.default_rng(case * 10 + zchunk)
        b = _round(rng.standard_normal((lz, ly, lx)) * 50.0, prec)
        x0 = _round(rng.standard_normal((lz, ly, lx)), prec)
        x = dev(x0)
        mg.mg_smooth_level(s.ctx, level, STORE[prec], dev(b), x, 1, 0, zchunk)
        got = x.cpu().numpy()
    finally:
        s.close()
    ref = oracle.rbgs_level(p, level, b, x0, 1)
    tol = 1.01 * HALF_ULP[prec] * np.abs(ref) + 4e-6 * np.abs(ref).max()
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (int(bad.sum()), float(np.abs(got - ref).max()), float(np.abs(ref).max()))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("zchunk", [0, 5])
def test_lowp_beta1_every_tile(prec, tile, zchunk):
    """The 4- and 2-byte beta = 1 sweep in every tile shape, on a grid whose
    tiles are ragged in x and y (104 = 64 + 40 cells, 40 rows) and whose
    z-chunks leave a short last chunk."""
    p = _problem("const", (104, 40, 24), 90 + tile)
    print(f"lowp beta=1 sweep {prec} tile {tile} zchunk {zchunk}", flush=True)
    s = make_solver(p, precision=prec)
    try:
        rng = np.random.default_rng(tile * 10 + zchunk)
        b = _round(rng.standard_normal(p.shape) * 50.0, prec)
        x0 = _round(rng.standard_normal(p.shape), prec)
        x = dev(x0)
        mg.mg_smooth_level(s.ctx, 0, STORE[prec], dev(b), x, 1, tile, zchunk)
        got = x.cpu().numpy()
    finally:
        s.close()
    ref = oracle.rbgs_level(p, 0, b, x0, 1)
    tol = 1.01 * HALF_ULP[prec] * np.abs(ref) + 4e-6 * np.abs(ref).max()
    bad = np.abs(got - ref) > tol
    assert not bad.any(), (int(bad.sum()), float(np.abs(got - ref).max()), float(np.abs(ref).max()))


@pytest.mark.parametrize("zchunk", [0, 1, 3, 8, 9])
@pytest.mark.parametrize("dims,level", [((64, 32, 48), 1), ((64, 32, 48), 2), ((60, 20, 44), 1),
                                        ((60, 20, 44), 2), ((96, 64, 64), 3)])
def test_stored_face_sweep_parity_fp64(zchunk, dims, level):
    """The FP64 sweeps of the potential's coarse levels, which stream the
    averaged face coefficients (two sweeps)."""
    p = _problem("cell", dims, 7 + level)
    p.bc = (("N", 0.0), ("D", 0.3), ("N", 0.0), ("D", -1.0), ("D", 0.0), ("D", 1.0))
    print(f"stored faces fp64 {dims} level {level} zchunk {zchunk}", flush=True)
    s = make_solver(p)
    try:
        lx, ly, lz = mg.mg_level_dims(s.ctx, level)
        rng = np.random.default_rng(level * 7 + zchunk)
        b = rng.standard_normal((lz, ly, lx)) * 50.0
        x0 = rng.standard_normal((lz, ly, lx))
        x = dev(x0)
        mg.mg_smooth_level(s.ctx, level, mg.MG_STORE_F64, dev(b), x, 2, 0, zchunk)
        got = x.cpu().numpy()
    finally:
        s.close()
    ref = oracle.rbgs_level(p, level, b, x0, 2)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("tile", range(1, mg.MG_NUM_TILES + 1))
def test_stored_face_sweep_every_tile(tile):
    p = _problem("cell", (128, 48, 40), 91)
    s = make_solver(p)
    try:
        lx, ly, lz = mg.mg_level_dims(s.ctx, 1)
        rng = np.random.default_rng(tile)
        b = rng.standard_normal((lz, ly, lx))
        x0 = rng.standard_normal((lz, ly, lx))
        x = dev(x0)
        mg.mg_smooth_level(s.ctx, 1, mg.MG_STORE_F64, dev(b), x, 1, tile, 5)
        got = x.cpu().numpy()
    finally:
        s.close()
    ref = oracle.rbgs_level(p, 1, b, x0, 1)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_level0_fp64_matches_mg_smooth():
    """Level 0 in FP64 is the finest equation with its boundary values:
    the same sweep as mg_smooth."""
    p = synth.streamer_set(32, seed=1)[0]
    s = make_solver(p)
    try:
        rng = np.random.default_rng(2)
        x0 = rng.standard_normal(p.shape)
        a, b = dev(x0), dev(x0)
        mg.mg_smooth(s.ctx, dev(p.f), a, 3)
        mg.mg_smooth_level(s.ctx, 0, mg.MG_STORE_F64, dev(p.f), b, 3)
        assert torch.equal(a, b)
    finally:
        s.close()


def test_smooth_level_rejects_bad_arguments():
    p = synth.streamer_set(32, seed=1)[0]
    s = make_solver(p)
    try:
        x = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
        f = dev(p.f)
        with pytest.raises(mg.MgError):
            mg.mg_smooth_level(s.ctx, 0, mg.MG_STORE_F32, f, x, 1)  # an FP64 context has no FP32 copies
        with pytest.raises(mg.MgError):
            mg.mg_smooth_level(s.ctx, 99, mg.MG_STORE_F64, f, x, 1)
        with pytest.raises(mg.MgError):
            mg.mg_smooth_level(s.ctx, 0, 7, f, x, 1)
    finally:
        s.close()
