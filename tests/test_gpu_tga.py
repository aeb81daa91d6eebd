"""GPU parity of the face-coefficient operator and of the TGA implicit
diffusion advance (paper Sec. 2, item (ii): face-centred D, zero flux
everywhere; Sec. 2.1, step (vi), Eq. (tga)) against the oracle's face form,
through the C ABI (mg_set_face_coeffs, mg_apply, mg_smooth, mg_residual,
mg_solve, mg_tga_step).

Element-wise kernels agree to 1e-12 of the field's largest value (the two
sides sum the face terms in different orders).  Solves stop at relative
residual 1e-11 here, and the TGA step's two Helmholtz solves have condition
numbers near 15 at the diffusion number used (max D dt / h^2 = 4), so the
step agrees with the oracle's step to 1e-9 relative L2."""
import numpy as np
import pytest

import oracle
import synth
from synth.problems import Problem
from tests.gpu_util import dev, gpu_solve, make_solver, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1809_08857_amd import mg  # noqa: E402

NEU = (("N", 0.0),) * 6


def _face_problem(dims, seed, a=3.0, bc=None):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    if bc is None:
        types = ["D" if t else "N" for t in rng.integers(0, 2, 6)]
        bc = tuple((t, float(rng.uniform(-1, 1)) if t == "D" else 0.0) for t in types)
    return Problem(nx, ny, nz, 1.0 / max(dims), a, rng.uniform(-1, 1, (nz, ny, nx)), None, bc,
                   f"faces_s{seed}", faces=synth.random_faces(nx, ny, nz, seed + 50, 0.1, 10.0))


DIMS = [(40, 24, 36), (64, 32, 48), (15, 14, 16)]


@pytest.mark.parametrize("k", range(len(DIMS)))
def test_face_residual_and_apply(k):
    p = _face_problem(DIMS[k], k)
    print(f"face residual {p.name} {DIMS[k]}", flush=True)
    rng = np.random.default_rng(k)
    u = rng.standard_normal(p.shape)
    r_ref, rn_ref, bn_ref = oracle.residual(p, u)
    s = make_solver(p)
    try:
        r = torch.empty(p.shape, dtype=torch.float64, device="cuda")
        rn, bn = s.residual(dev(p.f), dev(u), r)
        y = torch.empty(p.shape, dtype=torch.float64, device="cuda")
        mg.mg_apply(s.ctx, 0.5, -2.0, dev(u), y)
        y = y.cpu().numpy()
    finally:
        s.close()
    r = r.cpu().numpy()
    assert np.abs(r - r_ref).max() <= 1e-12 * np.abs(r_ref).max()
    assert abs(rn - rn_ref) <= 1e-12 * rn_ref and abs(bn - bn_ref) <= 1e-12 * bn_ref
    y_ref = 0.5 * u - 2.0 * oracle.apply(p, u)
    assert np.abs(y - y_ref).max() <= 1e-12 * np.abs(y_ref).max()


@pytest.mark.parametrize("tile", [0, 1, 3, 4, 6])
@pytest.mark.parametrize("zchunk", [0, 1, 3, 8, 9])
def test_face_sweep_level0(tile, zchunk):
    p = _face_problem((64, 32, 48), 7)
    print(f"face sweep tile {tile} zchunk {zchunk}", flush=True)
    u0 = np.random.default_rng(tile * 10 + zchunk).standard_normal(p.shape)
    ref = oracle.rbgs(p, u0, 2)
    s = make_solver(p)
    try:
        mg.mg_set_tiling(s.ctx, tile, zchunk)
        x = dev(u0)
        mg.mg_smooth(s.ctx, dev(p.f), x, 2)
        got = x.cpu().numpy()
    finally:
        s.close()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_face_solve_matches_oracle(seed):
    p = _face_problem((64, 64, 64), 20 + seed, a=[0.0, 5.0, 400.0][seed])
    if p.a == 0.0:
        p.bc = (("N", 0.0), ("N", 0.0), ("D", 0.2), ("N", 0.0), ("D", 0.0), ("D", 1.0))
    print(f"face solve {p.name} a={p.a}", flush=True)
    x, rc, st = gpu_solve(p, rtol=1e-11)
    print(st, flush=True)
    assert rc == mg.MG_OK
    ref = oracle.solve_reference(p)
    assert rel_l2(x, ref) <= 1e-9


@pytest.mark.parametrize("n", [64, 128])
@pytest.mark.parametrize("guess", [False, True])
def test_tga_step_matches_oracle(n, guess):
    faces = synth.diffusion_faces(n, n, n, 3)
    h = 1.0 / n
    dt = synth.TGA_DIFFUSION_NUMBER * h * h / max(a.max() for a in faces)
    n0 = synth.filament_source(n, n, n, 3)
    print(f"tga {n}^3 guess={guess} dt={dt:.3e}", flush=True)
    p = Problem(n, n, n, h, 1.0, n0, None, NEU, "tga", faces=faces)
    s = make_solver(p, rtol=1e-11)
    try:
        out = torch.empty(p.shape, dtype=torch.float64, device="cuda")
        rc, st = s.tga_step(dt, dev(n0), out, mg.MG_GUESS if guess else 0)
        print([q.as_dict() for q in st], flush=True)
        assert rc == mg.MG_OK
        got = out.cpu().numpy()
    finally:
        s.close()
    ref = oracle.tga_step(faces, h, dt, n0)
    err = rel_l2(got, ref)
    print(f"error vs oracle {err:.2e}", flush=True)
    assert err <= 1e-9
    assert abs(got.sum() - n0.sum()) <= 1e-8 * np.abs(n0).sum()


def test_face_coefficient_errors():
    p = _face_problem((32, 32, 32), 5, bc=NEU)
    faces = [dev(a) for a in p.faces]
    desc = mg.mg_desc_default(32, 32, 32, p.h, precision="fp32")
    ctx = mg.mg_create(desc)
    try:
        with pytest.raises(mg.MgError):
            mg.mg_set_face_coeffs(ctx, *faces, 1.0, mg.make_bcs(["N"] * 6, [0.0] * 6))
    finally:
        mg.mg_destroy(ctx)
    ctx = mg.mg_create(mg.mg_desc_default(32, 32, 32, p.h))
    try:
        bad = [f.clone() for f in faces]
        bad[1][3, 4, 5] = 0.0
        with pytest.raises(mg.MgError):
            mg.mg_set_face_coeffs(ctx, *bad, 1.0, mg.make_bcs(["N"] * 6, [0.0] * 6))
        bad[1][3, 4, 5] = float("nan")
        with pytest.raises(mg.MgError):
            mg.mg_set_face_coeffs(ctx, *bad, 1.0, mg.make_bcs(["N"] * 6, [0.0] * 6))
        # the TGA step needs zero flux on every face
        mg.mg_set_face_coeffs(ctx, *faces, 1.0, mg.make_bcs(["N"] * 5 + ["D"], [0.0] * 6))
        x = dev(p.f)
        out = torch.empty_like(x)
        with pytest.raises(mg.MgError):
            mg.mg_tga_step(ctx, 1e-3, x, out)
        mg.mg_set_face_coeffs(ctx, *faces, 1.0, mg.make_bcs(["N"] * 6, [0.0] * 6))
        with pytest.raises(mg.MgError):
            mg.mg_tga_step(ctx, -1.0, x, out)
        with pytest.raises(mg.MgError):
            mg.mg_tga_step(ctx, 1e-3, x, x)
    finally:
        mg.mg_destroy(ctx)
