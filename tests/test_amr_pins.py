"""Pins of the composite (two-level AMR) oracle (paper Secs. 2-4: the
elliptic equations on a base grid refined by patches; second-order
cell-centred discretisation).

- Linear potentials are reproduced exactly on the composite grid, with
  several patches, for a linear function along each axis: the ghost values
  beyond the coarse-fine interface are exact for linear functions and the
  refluxed coarse faces carry the exact flux.  A wrong interpolation weight
  or a missing sub-face fails this at the first cells by the interface.
- Conservation: with zero-flux box faces, the volume-weighted sum of A u
  equals a times the volume-weighted sum of u for any u (the coarse and fine
  sides of every interface face see the same flux).
- Constants solve all-Neumann Helmholtz problems exactly.
- Without patches the composite problem is the single-grid problem.
- Boxes that touch the domain or each other are rejected."""
import numpy as np
import pytest

import oracle
import synth
from oracle import amr_oracle as amr
from synth.problems import Problem

NEU = (("N", 0.0),) * 6
BOXES = [((4, 6, 8), (12, 14, 20)), ((16, 4, 6), (28, 12, 14)), ((6, 18, 18), (14, 28, 28))]


def _zero_fine(boxes):
    return [np.zeros((hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])) for lo, hi in boxes]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_solution_exact(axis):
    n = 16
    h = 1.0 / n
    bc = [("N", 0.0)] * 6
    bc[2 * axis] = ("D", -0.5)
    bc[2 * axis + 1] = ("D", 2.5)
    p = Problem(n, n, n, h, 0.0, np.zeros((n, n, n)), None, tuple(bc))
    comp = amr.Composite(p, BOXES, _zero_fine(BOXES))
    ub, uf = amr.solve(comp)
    lin = lambda c: -0.5 + 3.0 * c
    cc = (np.arange(n) + 0.5) * h
    want = lin(cc).reshape([n if d == 2 - axis else 1 for d in range(3)])
    assert np.abs(ub - want).max() < 1e-12
    for (lo, hi), a in zip(BOXES, uf):
        fc = (np.arange(lo[axis], hi[axis]) + 0.5) * h / 2
        shape = [1, 1, 1]
        shape[2 - axis] = fc.size
        assert np.abs(a - lin(fc).reshape(shape)).max() < 1e-12


def test_conservation_neumann():
    n = 16
    rng = np.random.default_rng(2)
    p = Problem(n, n, n, 1.0 / n, 3.0, np.zeros((n, n, n)), np.exp(rng.uniform(-1, 1, (n, n, n))), NEU)
    eps_f = [np.exp(rng.uniform(-1, 1, s.shape)) for s in _zero_fine(BOXES)]
    comp = amr.Composite(p, BOXES, _zero_fine(BOXES), eps_f)
    ub = rng.standard_normal((n, n, n))
    uf = [rng.standard_normal(a.shape) for a in _zero_fine(BOXES)]
    yb, yf = amr.apply(comp, ub, uf)
    mask = amr.coverage(n, n, n, BOXES) < 0
    vc, vf = p.h**3, (p.h / 2) ** 3
    lhs = vc * yb[mask].sum() + vf * sum(a.sum() for a in yf)
    rhs = p.a * (vc * ub[mask].sum() + vf * sum(a.sum() for a in uf))
    assert abs(lhs - rhs) <= 1e-12 * (abs(rhs) + vc * np.abs(yb).sum())


def test_constant_solves_neumann_helmholtz():
    n = 16
    p = Problem(n, n, n, 1.0 / n, 2.0, np.full((n, n, n), 6.0), None, NEU)
    comp = amr.Composite(p, BOXES, [np.full(a.shape, 6.0) for a in _zero_fine(BOXES)])
    ub, uf = amr.solve(comp)
    assert np.abs(ub - 3.0).max() < 1e-12 and max(np.abs(a - 3.0).max() for a in uf) < 1e-12


def test_without_patches_is_the_single_grid_problem():
    p = synth.random_problem(12, 10, 8, 3)
    comp = amr.Composite(p, [], [])
    ub, _ = amr.solve(comp)
    assert np.abs(ub - oracle.dense_solve(p)).max() <= 1e-11 * np.abs(ub).max()


@pytest.mark.parametrize("boxes", [
    [((0, 4, 4), (8, 12, 12))],                          # touches the domain
    [((4, 4, 4), (12, 12, 33))],                          # odd bound
    [((4, 4, 4), (10, 10, 10)), ((10, 4, 4), (16, 10, 10))],  # touching boxes
])
def test_bad_boxes_rejected(boxes):
    with pytest.raises(ValueError):
        amr.check_boxes(16, 16, 16, boxes)


def test_sampled_rows_match_the_assembled_residual():
    n = 16
    rng = np.random.default_rng(5)
    bc = (("D", 0.3), ("N", 0.0), ("D", -1.0), ("N", 0.0), ("N", 0.0), ("D", 2.0))
    p = Problem(n, n, n, 1.0 / n, 1.5, rng.standard_normal((n, n, n)), np.exp(rng.uniform(-1, 1, (n, n, n))), bc)
    fz = _zero_fine(BOXES)
    comp = amr.Composite(p, BOXES, [rng.standard_normal(a.shape) for a in fz],
                         [np.exp(rng.uniform(-1, 1, a.shape)) for a in fz])
    ub = rng.standard_normal((n, n, n))
    uf = [rng.standard_normal(a.shape) for a in fz]
    A, b, ix = amr.assemble(comp)
    r = b - A @ amr.pack(comp, ub, uf, ix)
    cells, want = [], []
    for K, J, I in [(0, 0, 0), (5, 7, 1), (3, 2, 3), (15, 15, 15), (4, 9, 6)]:  # (4, 9, 6) borders box 0
        if ix.base_id[K, J, I] >= 0:
            cells.append(("c", I, J, K))
            want.append(r[ix.base_id[K, J, I]])
    for q, (lo, hi) in enumerate(BOXES):
        for c in (lo, tuple(h - 1 for h in hi), tuple((l + h) // 2 for l, h in zip(lo, hi))):
            cells.append(("f", q, *c))
            want.append(r[ix.fine(q, *c)])
    got = amr.residual_at(comp, ub, uf, cells)
    assert np.allclose(got, want, rtol=1e-13, atol=1e-12 * np.abs(r).max())
