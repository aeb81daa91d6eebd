"""Pins of the embedded-boundary (cut-cell) oracle (paper Sec. 2: finite
volumes with an embedded boundary formalism, second-order cell-centred
elliptic operators; Sec. 4: a needle electrode).

- Linear potentials are reproduced exactly around a tilted planar electrode
  (every term of a cut-cell row is exact for linear functions and the
  embedded face closes the divergence theorem): a wrong ray point, a wrong
  one-sided difference weight, a sign of the embedded term or a dropped
  aperture fails it.
- The embedded areas of a sphere sum to its surface area (to the accuracy
  of the sampled apertures), and its area vectors sum to zero.
- The potential of a sphere held at V in a box whose faces carry V R / r
  converges to V R / r at second order.
- Without an electrode the cut-cell problem is the single-grid problem.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import eb_oracle as eb
from synth import geometry as geo
from synth.problems import Problem

DIR = (("D", 0.0),) * 6


def _face_centres(n, h, d):
    """Coordinates (x, y, z) of the centres of box face d's cell faces, [nz|ny][..] arrays."""
    axis, hi = d // 2, d % 2
    c = (np.arange(n) + 0.5) * h
    w = 1.0 if hi else 0.0
    a, b = np.meshgrid(c, c, indexing="ij")  # [slow][fast] of the two tangential axes (z or y, then y or x)
    if axis == 0:
        return np.full_like(a, w), b, a
    if axis == 1:
        return b, np.full_like(a, w), a
    return b, a, np.full_like(a, w)


def _linear_problem(n, shape, coef, a=0.0):
    h = 1.0 / n
    G = geo.cut_geometry(shape, n, n, n, h)
    lin = lambda x, y, z: coef[0] + coef[1] * x + coef[2] * y + coef[3] * z
    zc, yc, xc = np.meshgrid(*(((np.arange(n) + 0.5) * h,) * 3), indexing="ij")
    u = lin(xc, yc, zc)
    g = u.copy()                                   # covered cells: the centre value
    k, r = np.divmod(G.bidx, n * n)
    j, i = np.divmod(r, n)
    xb = np.stack([(i + 0.5), (j + 0.5), (k + 0.5)], axis=1) + G.boff
    g.reshape(-1)[G.bidx] = lin(*(xb.T * h))       # boundary cells: the surface point
    fv = {d: lin(*_face_centres(n, h, d)) for d in range(6)}
    p = Problem(n, n, n, h, a, a * u, None, DIR)
    return eb.EBProblem(p, G, g, fv, "linear"), u


@pytest.mark.parametrize("normal,offset", [((0.3, -0.2, 1.0), 0.37), ((1.0, 0.6, 0.25), 0.71), ((-0.4, 1.0, 0.5), 0.1)])
def test_linear_exact_around_a_tilted_plane(normal, offset):
    prob, u = _linear_problem(12, geo.half_space(normal, offset), (0.3, -1.2, 0.7, 2.1))
    assert prob.geom.bidx.size > 50
    got = eb.solve(prob)
    assert np.abs(got - u).max() < 1e-11


def test_linear_exact_around_a_sphere_with_screening():
    prob, u = _linear_problem(14, geo.sphere((0.47, 0.52, 0.5), 0.27), (1.0, 0.5, -2.0, 1.5), a=3.0)
    got = eb.solve(prob)
    assert np.abs(got - u).max() < 1e-11


def test_sphere_area_and_closure():
    n, R = 40, 0.3
    G = geo.cut_geometry(geo.sphere((0.5, 0.5, 0.5), R), n, n, n, 1.0 / n, nsub=8)
    prob = eb.EBProblem(Problem(n, n, n, 1.0 / n, 0.0, np.zeros((n, n, n)), None, DIR), G)
    A, nu, _, _ = eb.embedded_faces(prob)
    area = A.sum() / n**2
    assert abs(area - 4 * np.pi * R**2) < 0.01 * 4 * np.pi * R**2
    assert np.linalg.norm((A[:, None] * nu).sum(axis=0)) < 1e-9 * A.sum()
    # the inward normal of a sphere points away from its centre
    k, r = np.divmod(G.bidx, n * n)
    j, i = np.divmod(r, n)
    rad = np.stack([i + 0.5, j + 0.5, k + 0.5], axis=1) / n - 0.5
    big = A > 0.3
    cosang = (nu[big] * rad[big]).sum(axis=1) / np.linalg.norm(rad[big], axis=1)
    assert cosang.min() > 0.9


def _sphere_error(n, R=0.2, V=1.0):
    h = 1.0 / n
    c = (0.5, 0.5, 0.5)
    G = geo.cut_geometry(geo.sphere(c, R), n, n, n, h, nsub=8)
    exact = lambda x, y, z: V * R / np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    fv = {d: exact(*_face_centres(n, h, d)) for d in range(6)}
    p = Problem(n, n, n, h, 0.0, np.zeros((n, n, n)), None, DIR)
    u = eb.solve(eb.EBProblem(p, G, V, fv, "sphere"))
    zc, yc, xc = np.meshgrid(*(((np.arange(n) + 0.5) * h,) * 3), indexing="ij")
    m = G.kappa > 0
    return np.abs(u - exact(xc, yc, zc))[m].max()


def test_sphere_potential_second_order():
    e1, e2 = _sphere_error(16), _sphere_error(32)
    assert e2 < e1
    assert np.log2(e1 / e2) > 1.5, (e1, e2)


def test_without_electrode_is_the_single_grid_problem():
    p = synth.random_problem(8, 8, 8, 5)
    n = 8
    G = geo.Geometry(np.ones((n, n, n)), np.ones((n, n, n + 1)), np.ones((n, n + 1, n)), np.ones((n + 1, n, n)),
                     np.zeros(0, dtype=np.int64), np.zeros((0, 3)))
    u = eb.solve(eb.EBProblem(p, G, 0.0))
    want = oracle.dense_solve(p)
    assert np.abs(u - want).max() <= 1e-11 * np.abs(want).max()


def test_covered_cells_hold_the_electrode_potential():
    n = 16
    G = geo.cut_geometry(geo.needle(0.15, 0.4), n, n, n, 1.0 / n)
    bc = (("N", 0.0),) * 4 + (("D", 0.0), ("D", 1.0))
    p = Problem(n, n, n, 1.0 / n, 0.0, np.zeros((n, n, n)), None, bc)
    u = eb.solve(eb.EBProblem(p, G, 1.0))
    assert np.all(u[G.kappa == 0] == 1.0)
    # the potential of the cells wholly in the gas lies between the grounded
    # plane and the electrode (cut cells whose centre lies inside the
    # electrode carry the smooth continuation of the potential, which may
    # exceed it)
    gas = u[G.kappa == 1]
    assert gas.min() > 0.0 and gas.max() < 1.0


def test_rows_one_at_a_time_match_the_assembled_residual():
    n = 14
    rng = np.random.default_rng(3)
    G = geo.cut_geometry(geo.needle(0.2, 0.45), n, n, n, 1.0 / n)
    bc = (("N", 0.0), ("D", 0.4), ("N", 0.0), ("N", 0.0), ("D", -0.2), ("D", 1.0))
    p = Problem(n, n, n, 1.0 / n, 2.5, rng.standard_normal((n, n, n)), np.exp(rng.uniform(-1, 1, (n, n, n))), bc)
    prob = eb.EBProblem(p, G, 0.8)
    u = rng.standard_normal((n, n, n))
    Am, b = eb.assemble(prob)
    r = b - Am @ u.reshape(-1)
    cells = np.concatenate([G.bidx[::7], np.flatnonzero(G.kappa.reshape(-1) == 0)[::5], rng.integers(0, n**3, 40)])
    got = eb.residual_at(prob, u, cells)
    assert np.allclose(got, r[cells], rtol=1e-12, atol=1e-12 * np.abs(r).max())
    assert np.allclose(eb.rhs_only(prob).reshape(-1), b, rtol=1e-13, atol=1e-13 * np.abs(b).max())
