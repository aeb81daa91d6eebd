"""GPU parity of the multigrid engine against the CPU FP64 oracle, through
the C ABI.  Tolerances: element-wise kernels (residual, smoother) agree to
rounding (1e-12 relative to the field's magnitude: the two sides sum the six
face terms in different orders); solves reach relative residual 1e-10 and
agree with the oracle's solution (relative residual 1e-13) to 1e-9 in
relative L2, the accuracy bar of the engine."""
import numpy as np
import pytest

import oracle
import synth
from synth.problems import Problem
from tests.gpu_util import dev, gpu_solve, make_solver, rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1809_08857_amd import mg  # noqa: E402

RTOL = 1e-10
ERR = 1e-9


def rtol_for(p):
    """The potential (a = 0) has error/residual ratios of ~10-25 near
    convergence, so it is solved to 1e-11 to keep the 1e-9 error bar; the
    screened equations have ratio ~1 and stop at 1e-10."""
    return 1e-11 if p.a == 0.0 else RTOL


def _problems_small():
    out = [
        synth.random_problem(40, 24, 36, 11),                      # ragged tiles, 3 levels + bottom
        synth.random_problem(72, 40, 24, 12, variable_eps=False),  # const beta, a > 0
        synth.streamer_set(64, seed=2)[0],                         # slab eps + filament
        synth.streamer_set(64, seed=2)[2],                         # photon group, all Dirichlet
        synth.random_problem(15, 9, 7, 13),                        # odd dims, bottom solver only
    ]
    return out


@pytest.mark.parametrize("k", range(5))
def test_residual_parity(k):
    p = _problems_small()[k]
    print(f"residual parity: {p.name}", flush=True)
    rng = np.random.default_rng(k)
    u = rng.standard_normal(p.shape)
    r_ref, rn_ref, bn_ref = oracle.residual(p, u)
    s = make_solver(p)
    try:
        r = torch.empty(p.shape, dtype=torch.float64, device="cuda")
        rn, bn = s.residual(dev(p.f), dev(u), r)
    finally:
        s.close()
    r = r.cpu().numpy()
    scale = np.abs(r_ref).max()
    assert np.abs(r - r_ref).max() <= 1e-12 * scale
    assert abs(rn - rn_ref) <= 1e-12 * rn_ref
    assert abs(bn - bn_ref) <= 1e-12 * bn_ref


@pytest.mark.parametrize("k", range(5))
@pytest.mark.parametrize("sweeps", [1, 2])
def test_smoother_parity(k, sweeps):
    p = _problems_small()[k]
    print(f"smoother parity: {p.name} sweeps={sweeps}", flush=True)
    rng = np.random.default_rng(100 + k)
    u0 = rng.standard_normal(p.shape)
    ref = oracle.rbgs(p, u0, sweeps)
    s = make_solver(p)
    try:
        x = dev(u0)
        mg.mg_smooth(s.ctx, dev(p.f), x, sweeps)
        got = x.cpu().numpy()
    finally:
        s.close()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("tile", range(1, mg.MG_NUM_TILES + 1))
@pytest.mark.parametrize("zchunk", [3, 64])
@pytest.mark.parametrize("cell_eps", [True, False])
def test_smoother_every_tile_variant(tile, zchunk, cell_eps):
    """Every (TX, TY) tile and a z-chunk that splits the grid unevenly, with
    cell coefficients and with beta = 1."""
    p = synth.random_problem(112, 24, 40, 21, variable_eps=cell_eps)
    print(f"tile {tile} zchunk {zchunk} cell_eps {cell_eps}", flush=True)
    rng = np.random.default_rng(tile)
    u0 = rng.standard_normal(p.shape)
    ref = oracle.rbgs(p, u0, 1)
    s = make_solver(p)
    try:
        mg.mg_set_tiling(s.ctx, tile, zchunk)
        x = dev(u0)
        mg.mg_smooth(s.ctx, dev(p.f), x, 1)
        got = x.cpu().numpy()
    finally:
        s.close()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("zchunk", [1, 2, 4, 5, 6, 7, 9])
@pytest.mark.parametrize("cell_eps", [True, False])
@pytest.mark.parametrize("dims", [(64, 32, 24), (15, 13, 16)])
def test_smoother_plane_ring_chunks(zchunk, cell_eps, dims):
    """The sweeps stream z planes through a ring of PD + 3 register slots
    (5 for FP64) and unroll the plane loop that many steps at a time: chunks
    shorter than, equal to and longer than the ring, with ragged last
    chunks, even and odd row lengths."""
    p = synth.random_problem(*dims, 60 + zchunk, variable_eps=cell_eps)
    print(f"plane ring: {p.name} zchunk {zchunk} cell_eps {cell_eps}", flush=True)
    rng = np.random.default_rng(zchunk)
    u0 = rng.standard_normal(p.shape)
    ref = oracle.rbgs(p, u0, 2)
    s = make_solver(p)
    try:
        mg.mg_set_tiling(s.ctx, 3, zchunk)
        x = dev(u0)
        mg.mg_smooth(s.ctx, dev(p.f), x, 2)
        got = x.cpu().numpy()
    finally:
        s.close()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


_BC_PATTERNS = [
    (("D", 0.3), ("D", -0.7), ("D", 0.5), ("D", -0.2), ("D", 0.9), ("D", -0.4)),
    (("N", 0.0), ("N", 0.0), ("N", 0.0), ("N", 0.0), ("N", 0.0), ("D", 0.6)),
    (("D", 0.8), ("N", 0.0), ("N", 0.0), ("D", -0.5), ("D", 0.1), ("N", 0.0)),
    (("N", 0.0), ("D", -0.9), ("D", 0.4), ("N", 0.0), ("N", 0.0), ("D", 0.7)),
]


@pytest.mark.parametrize("pattern", range(len(_BC_PATTERNS)))
@pytest.mark.parametrize("dims,wide", [((56, 20, 36), False), ((15, 13, 11), False), ((64, 40, 24), True)])
def test_smoother_boundary_faces(pattern, dims, wide):
    """Cell coefficients against each kind of box face on every side: the
    sweep encodes Dirichlet and Neumann faces in the values of the cells
    outside the box.  Several tiles with a ragged tail, an odd nx, and
    coefficients spread over twelve decades."""
    p = synth.random_problem(*dims, 40 + pattern, bc=_BC_PATTERNS[pattern], a=0.0)
    if wide:
        rng = np.random.default_rng(pattern)
        p = Problem(p.nx, p.ny, p.nz, p.h, p.a, p.f, np.exp(rng.uniform(np.log(1e-6), np.log(1e6), p.shape)),
                    p.bc, p.name + "_wide")
    print(f"smoother boundary faces: {p.name} {p.bc}", flush=True)
    rng = np.random.default_rng(200 + pattern)
    u0 = rng.standard_normal(p.shape)
    ref = oracle.rbgs(p, u0, 1)
    s = make_solver(p)
    try:
        x = dev(u0)
        mg.mg_smooth(s.ctx, dev(p.f), x, 1)
        got = x.cpu().numpy()
    finally:
        s.close()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("pattern", range(len(_BC_PATTERNS)))
def test_prolongation_parity(pattern):
    """u += P e at every level of a ragged three-level hierarchy (each face
    type on each side) against the oracle's prolongation."""
    p = synth.random_problem(56, 20, 36, 50 + pattern, bc=_BC_PATTERNS[pattern], a=0.0)
    s = make_solver(p)
    try:
        nlev = mg.mg_num_levels(s.ctx)
        assert nlev >= 3
        rng = np.random.default_rng(300 + pattern)
        for lev in range(nlev - 1):
            fx, fy, fz = mg.mg_level_dims(s.ctx, lev)
            cx, cy, cz = mg.mg_level_dims(s.ctx, lev + 1)
            print(f"prolongation {p.name} level {lev}: {cx}x{cy}x{cz} -> {fx}x{fy}x{fz}", flush=True)
            e = rng.standard_normal((cz, cy, cx))
            u0 = rng.standard_normal((fz, fy, fx))
            ref = oracle.prolong_add(e, u0, p.bc_types())
            u = dev(u0)
            mg.mg_prolong_add(s.ctx, lev, dev(e), u)
            got = u.cpu().numpy()
            assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max(), lev
        with pytest.raises(mg.MgError):
            mg.mg_prolong_add(s.ctx, nlev - 1, dev(np.zeros(1)), dev(np.zeros(1)))
    finally:
        s.close()


def _manufactured_exact(n):
    h = 1.0 / n
    c = (np.arange(n) + 0.5) * h
    lam = (4 / h**2) * (2 * np.sin(np.pi * h / 2) ** 2 + np.sin(np.pi * h) ** 2)
    mode = np.sin(2 * np.pi * c)[:, None, None] * np.cos(np.pi * c)[None, :, None] * np.cos(np.pi * c)[None, None, :]
    return c[:, None, None] + (6 * np.pi**2 / lam) * mode


def test_manufactured_32():
    p = synth.manufactured_poisson(32)
    x, rc, st = gpu_solve(p, rtol=rtol_for(p))
    print(st, flush=True)
    assert rc == mg.MG_OK and st["rel_res"] <= rtol_for(p)
    _, rn, bn = oracle.residual(p, x)
    assert rn / bn <= RTOL * 1.0001
    assert rel_l2(x, _manufactured_exact(32)) <= ERR
    assert rel_l2(x, oracle.solve_reference(p)) <= ERR


@pytest.mark.parametrize("k", range(5))
def test_solve_parity_small(k):
    p = _problems_small()[k]
    x, rc, st = gpu_solve(p, rtol=rtol_for(p))
    print(p.name, st, flush=True)
    assert rc == mg.MG_OK and st["rel_res"] <= rtol_for(p)
    _, rn, bn = oracle.residual(p, x)
    assert rn / bn <= RTOL * 1.0001
    assert rel_l2(x, oracle.solve_reference(p)) <= ERR


@pytest.mark.parametrize("which", range(4))
def test_streamer_set_128(which):
    p = synth.streamer_set(128, seed=0)[which]
    x, rc, st = gpu_solve(p, rtol=rtol_for(p))
    print(p.name, st, flush=True)
    assert rc == mg.MG_OK and st["rel_res"] <= rtol_for(p)
    assert st["cycles"] <= 14
    _, rn, bn = oracle.residual(p, x)
    assert rn / bn <= RTOL * 1.0001
    assert rel_l2(x, oracle.solve_reference(p)) <= ERR


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("which", range(4))
def test_mixed_precision_64(prec, which):
    p = synth.streamer_set(64, seed=1)[which]
    x, rc, st = gpu_solve(p, precision=prec, rtol=rtol_for(p))
    print(prec, p.name, st, flush=True)
    assert rc == mg.MG_OK and st["rel_res"] <= rtol_for(p)
    _, rn, bn = oracle.residual(p, x)
    assert rn / bn <= RTOL * 1.0001
    assert rel_l2(x, oracle.solve_reference(p)) <= ERR


@pytest.mark.parametrize("dims", [(8, 8, 8), (12, 10, 6), (15, 15, 15), (1, 1, 1), (2, 16, 4)])
def test_bottom_only_grids(dims):
    """Grids that the single-workgroup bottom solver handles on its own."""
    p = synth.random_problem(*dims, seed=sum(dims))
    x, rc, st = gpu_solve(p, rtol=rtol_for(p))
    assert rc == mg.MG_OK and st["rel_res"] <= rtol_for(p)
    assert rel_l2(x, oracle.dense_solve(p) if p.cells <= 1000 else oracle.solve_reference(p)) <= ERR


def test_guess_accepted_and_rejected():
    p = synth.streamer_set(64, seed=4)[1]
    ref = oracle.solve_reference(p)
    # a close guess is kept and saves cycles
    _, _, st0 = gpu_solve(p)
    x, rc, st = gpu_solve(p, x0=ref * (1 + 1e-4), flags=mg.MG_GUESS)
    assert rc == mg.MG_OK and st["fell_back"] == 0 and st["cycles"] < st0["cycles"]
    assert rel_l2(x, ref) <= ERR
    # a guess worse than zero is rejected and the solve still converges
    rng = np.random.default_rng(0)
    bad = 1e6 * rng.standard_normal(p.shape)
    x, rc, st = gpu_solve(p, x0=bad, flags=mg.MG_GUESS)
    assert rc == mg.MG_OK and st["fell_back"] == 1 and st["rel_res0"] == 1.0
    assert rel_l2(x, ref) <= ERR


def test_zero_rhs_gives_zero():
    p = Problem(32, 32, 32, 1 / 32, 4.0, np.zeros((32, 32, 32)), None, (("D", 0.0),) * 6)
    x, rc, st = gpu_solve(p, x0=np.ones(p.shape), flags=mg.MG_GUESS)
    assert rc == mg.MG_OK and np.all(x == 0)


def test_invalid_inputs_rejected():
    p = synth.streamer_set(32, seed=0)[0]
    eps = p.eps.copy()
    eps[3, 4, 5] = -1.0
    with pytest.raises(mg.MgError) as e:
        mg.Solver(p.nx, p.ny, p.nz, p.h, eps=dev(eps), a=0.0, bc_types=p.bc_types(), bc_values=p.bc_values())
    assert e.value.code == mg.MG_EINVAL
    eps[3, 4, 5] = np.nan
    with pytest.raises(mg.MgError):
        mg.Solver(p.nx, p.ny, p.nz, p.h, eps=dev(eps), a=0.0, bc_types=p.bc_types(), bc_values=p.bc_values())
    eps[3, 4, 5] = 1e101  # above the largest accepted coefficient (1e100)
    with pytest.raises(mg.MgError):
        mg.Solver(p.nx, p.ny, p.nz, p.h, eps=dev(eps), a=0.0, bc_types=p.bc_types(), bc_values=p.bc_values())
    s = make_solver(p)
    try:
        f = p.f.copy()
        f[0, 0, 0] = np.inf
        x = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
        with pytest.raises(mg.MgError) as e:
            s.solve(dev(f), x)
        assert e.value.code == mg.MG_EINVAL
        # one cycle is not enough: soft error with valid stats
        d = mg.mg_desc_default(p.nx, p.ny, p.nz, p.h, max_cycles=1)
    finally:
        s.close()
    x, rc, st = gpu_solve(p, max_cycles=1)
    assert rc == mg.MG_NOT_CONVERGED and st["cycles"] == 1 and st["rel_res"] > RTOL


def test_deterministic():
    p = synth.streamer_set(64, seed=3)[0]
    x1, _, s1 = gpu_solve(p)
    x2, _, s2 = gpu_solve(p)
    assert np.array_equal(x1, x2) and s1["rel_res"] == s2["rel_res"]


def test_autotune_keeps_parity():
    p = synth.streamer_set(64, seed=5)[0]
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal(p.shape)
    ref = oracle.rbgs(p, u0, 1)
    s = make_solver(p)
    try:
        tile, zc, us = mg.mg_autotune(s.ctx, 2)
        print("autotune", tile, zc, us, flush=True)
        assert 1 <= tile <= mg.MG_NUM_TILES and zc >= 1 and us > 0
        x = dev(u0)
        mg.mg_smooth(s.ctx, dev(p.f), x, 1)
        got = x.cpu().numpy()
        f = dev(p.f)
        xs = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
        rc, st = s.solve(f, xs)
        assert rc == mg.MG_OK
    finally:
        s.close()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
