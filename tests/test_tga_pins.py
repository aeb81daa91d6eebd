"""Pins of the oracle's face-coefficient operator and of its TGA diffusion
advance (paper Sec. 2, item (ii): implicit diffusion with face-centred
coefficients and zero flux everywhere; Sec. 2.1, step (vi), Eq. (tga)).

- The TGA coefficients: the amplification of one step,
  R(z) = (1 + mu3 z) / ((1 - mu1 z)(1 - mu2 z)), matches exp(z) to second
  order (its error falls eightfold when z halves) and vanishes for z -> -inf.
- On a Neumann cosine mode, an exact eigenvector of the discrete Laplacian
  with eigenvalue -lambda_h (constant D), one oracle TGA step multiplies the
  mode by exactly R(-D lambda_h dt).
- A TGA step conserves the total sum with any face coefficients (zero-flux
  divergence form).
- The face form of the operator: faces made from a cell coefficient by
  harmonic means give the cell form's operator; random faces give a
  symmetric operator; a dense brute-force solve with random faces and random
  boundary types agrees with the oracle's V-cycle and CG; all-Neumann
  Helmholtz conserves a * sum(u) = sum(f)."""
import numpy as np
import pytest

import oracle
import synth
from synth.problems import Problem

NEU = (("N", 0.0),) * 6


def _faces_from_cell(eps):
    """Harmonic means of neighbouring cells; boundary faces take the
    boundary cell's own value."""
    nz, ny, nx = eps.shape
    hm = lambda p, q: 2 * p * q / (p + q)
    bx = np.empty((nz, ny, nx + 1))
    bx[:, :, 1:nx] = hm(eps[:, :, :-1], eps[:, :, 1:])
    bx[:, :, 0], bx[:, :, nx] = eps[:, :, 0], eps[:, :, -1]
    by = np.empty((nz, ny + 1, nx))
    by[:, 1:ny, :] = hm(eps[:, :-1, :], eps[:, 1:, :])
    by[:, 0, :], by[:, ny, :] = eps[:, 0, :], eps[:, -1, :]
    bz = np.empty((nz + 1, ny, nx))
    bz[1:nz] = hm(eps[:-1], eps[1:])
    bz[0], bz[nz] = eps[0], eps[-1]
    return bx, by, bz


def _R(z, dt=1.0):
    m1, m2, m3 = oracle.tga_coefficients(dt)
    return (1 + m3 * z) / ((1 - m1 * z) * (1 - m2 * z))


def test_tga_amplification_second_order_and_l_stable():
    errs = [abs(_R(-z) - np.exp(-z)) for z in (0.1, 0.05, 0.025)]
    assert 7.0 < errs[0] / errs[1] < 9.0 and 7.0 < errs[1] / errs[2] < 9.0
    assert abs(_R(-1e8)) < 1e-7
    m1, m2, m3 = oracle.tga_coefficients(1.0)
    assert m1 > 0 and m2 > 0 and m3 > 0


def test_tga_step_on_neumann_cosine_mode():
    n, c, dt = 16, 2.5, 3e-3
    h = 1.0 / n
    x = (np.arange(n) + 0.5) * h
    mode = (np.cos(np.pi * x)[None, None, :] * np.cos(2 * np.pi * x)[None, :, None]
            * np.cos(np.pi * x)[:, None, None])
    lam = (4 / h**2) * (2 * np.sin(np.pi * h / 2) ** 2 + np.sin(np.pi * h) ** 2)
    faces = tuple(np.full(sh, c) for sh in ((n, n, n + 1), (n, n + 1, n), (n + 1, n, n)))
    out = oracle.tga_step(faces, h, dt, mode)
    assert np.abs(out - _R(-c * lam * dt) * mode).max() < 1e-11


def test_tga_step_conserves_the_sum():
    nx, ny, nz = 12, 8, 16
    faces = synth.random_faces(nx, ny, nz, 3, 0.1, 10.0)
    n0 = np.random.default_rng(4).random((nz, ny, nx))
    out = oracle.tga_step(faces, 1.0 / nz, 5e-3, n0)
    assert abs(out.sum() - n0.sum()) < 1e-11 * np.abs(n0).sum()
    assert np.abs(out - n0).max() > 1e-3  # it did diffuse


def test_faces_from_cell_equal_the_cell_form():
    p = synth.random_problem(10, 8, 6, 5)
    q = Problem(p.nx, p.ny, p.nz, p.h, p.a, p.f, None, p.bc, "faces", faces=_faces_from_cell(p.eps))
    u = np.random.default_rng(1).standard_normal(p.shape)
    assert np.abs(oracle.apply(q, u) - oracle.apply(p, u)).max() <= 1e-12 * np.abs(oracle.apply(p, u)).max()
    assert np.abs(oracle.rhs(q) - oracle.rhs(p)).max() <= 1e-12 * np.abs(oracle.rhs(p)).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_face_operator_symmetric(seed):
    nx, ny, nz = 9, 7, 6
    rng = np.random.default_rng(seed)
    types = tuple(("D" if t else "N", 0.0) for t in rng.integers(0, 2, 6))
    q = Problem(nx, ny, nz, 1.0 / nz, 3.0, np.zeros((nz, ny, nx)), None, types, faces=synth.random_faces(nx, ny, nz, seed))
    u, v = rng.standard_normal((2, nz, ny, nx))
    a, b = np.vdot(u, oracle.apply(q, v)), np.vdot(oracle.apply(q, u), v)
    assert abs(a - b) <= 1e-12 * max(abs(a), 1.0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_face_form_dense_bruteforce(seed):
    nx, ny, nz = 8, 8, 8
    rng = np.random.default_rng(100 + seed)
    types = ["D" if t else "N" for t in rng.integers(0, 2, 6)]
    types[int(rng.integers(0, 6))] = "D"
    bc = tuple((t, float(rng.uniform(-1, 1)) if t == "D" else 0.0) for t in types)
    q = Problem(nx, ny, nz, 1.0 / nz, float(rng.uniform(0, 20)), rng.uniform(-1, 1, (nz, ny, nx)), None, bc,
                faces=synth.random_faces(nx, ny, nz, 7 + seed))
    ref = oracle.dense_solve(q)
    u_mg, _, rel = oracle.solve_vcycle(q, rtol=1e-14, coarsest_max=2)
    u_cg, _, _ = oracle.solve_cg(q, rtol=1e-14)
    assert np.abs(u_mg - ref).max() <= 1e-11 * np.abs(ref).max()
    assert np.abs(u_cg - ref).max() <= 1e-11 * np.abs(ref).max()


def test_face_form_neumann_helmholtz_conservation():
    nx, ny, nz = 12, 10, 8
    rng = np.random.default_rng(9)
    q = Problem(nx, ny, nz, 1.0 / nz, 7.0, rng.standard_normal((nz, ny, nx)), None, NEU,
                faces=synth.random_faces(nx, ny, nz, 9))
    u, _, _ = oracle.solve_cg(q, rtol=1e-14)
    assert abs(q.a * u.sum() - q.f.sum()) <= 1e-10 * np.abs(q.f).sum()


def test_face_form_rbgs_black_residual_vanishes():
    """After one red-black sweep every black cell satisfies its own equation."""
    nx, ny, nz = 10, 6, 8
    rng = np.random.default_rng(3)
    q = Problem(nx, ny, nz, 1.0 / nz, 2.0, rng.standard_normal((nz, ny, nx)), None,
                (("D", 0.5), ("N", 0.0), ("N", 0.0), ("D", -1.0), ("N", 0.0), ("D", 0.2)),
                faces=synth.random_faces(nx, ny, nz, 4))
    u = oracle.rbgs(q, rng.standard_normal((nz, ny, nx)), 1)
    r, _, _ = oracle.residual(q, u)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    black = (i + j + k) % 2 == 1
    assert np.abs(r[black]).max() <= 1e-11 * np.abs(r).max()
    assert np.abs(r[~black]).max() > 1e-3


def test_diffusion_faces_generator_shape_and_range():
    bx, by, bz = synth.diffusion_faces(16, 12, 20, 0)
    assert bx.shape == (20, 12, 17) and by.shape == (20, 13, 16) and bz.shape == (21, 12, 16)
    for a in (bx, by, bz):
        assert a.min() > 0.5 and a.max() < 15.0
    assert max(a.max() for a in (bx, by, bz)) > 5.0  # the head region is present
