"""Pins of the oracle's field E = -grad(phi) and dielectric relaxation time
(the time-step table of paper Sec. 2.2: dt_E = eps0 |E| / |J|; Sec. 2: the
field follows from the potential), computed by central differences with the
discretisation's ghost values beyond the box.

- A potential linear along an axis with the matching Dirichlet values gives
  the exact constant field in every cell, boundary cells included (the
  linear ghost continues the line).
- A quadratic potential gives the exact derivative at every interior cell,
  and at the cells beside a zero-flux face where the quadratic's slope
  vanishes (the mirrored ghost is exact there).
- A uniform conductivity sigma gives dt_E = eps0 / sigma exactly; the
  largest |E| and |J| are those of the cells that hold them."""
import numpy as np
import pytest

import oracle
from synth.problems import Problem


def _centres(n, h):
    return (np.arange(n) + 0.5) * h


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_potential_constant_field(axis):
    nx, ny, nz = 12, 10, 8
    h = 1.0 / 8
    shape = (nz, ny, nx)
    c = [_centres(nx, h), _centres(ny, h), _centres(nz, h)][axis]
    L = [nx, ny, nz][axis] * h
    bshape = [1, 1, 1]
    bshape[2 - axis] = c.size
    phi = np.broadcast_to((0.3 + 2.0 * c).reshape(bshape), shape).copy()
    bc = [("N", 0.0)] * 6
    bc[2 * axis] = ("D", 0.3)
    bc[2 * axis + 1] = ("D", 0.3 + 2.0 * L)
    p = Problem(nx, ny, nz, h, 0.0, np.zeros(shape), None, tuple(bc))
    E = oracle.field(p, phi)
    for d in range(3):
        want = -2.0 if d == axis else 0.0
        assert np.abs(E[d] - want).max() < 1e-12


def test_quadratic_potential_interior_and_mirror_faces():
    n = 16
    h = 1.0 / n
    x = _centres(n, h)
    phi = (x[None, None, :] ** 2 + 3 * x[None, :, None] ** 2 - x[:, None, None] ** 2).copy()
    p = Problem(n, n, n, h, 0.0, np.zeros((n, n, n)), None, (("N", 0.0),) * 6)
    ex, ey, ez = oracle.field(p, phi)
    want_x = -2 * x[None, None, :] * np.ones((n, n, n))
    want_y = -6 * x[None, :, None] * np.ones((n, n, n))
    want_z = 2 * x[:, None, None] * np.ones((n, n, n))
    inner = (slice(None), slice(None), slice(0, n - 1))  # the x+ face is zero flux but the slope is not 0 there
    assert np.abs(ex[inner] - want_x[inner]).max() < 1e-12
    assert np.abs(ey[:, : n - 1, :] - want_y[:, : n - 1, :]).max() < 1e-12
    assert np.abs(ez[: n - 1] - want_z[: n - 1]).max() < 1e-12
    assert np.abs(ex[..., n - 1] - want_x[..., n - 1]).max() > 1e-2  # the mismatched face is seen


def test_relaxation_time_uniform_conductivity():
    n = 12
    h = 1.0 / n
    rng = np.random.default_rng(3)
    phi = rng.standard_normal((n, n, n))
    p = Problem(n, n, n, h, 0.0, np.zeros((n, n, n)), None,
                (("N", 0.0), ("N", 0.0), ("D", 0.5), ("N", 0.0), ("D", 0.0), ("D", 1.0)))
    emax, jmax, dte = oracle.relaxation_time(p, phi, np.full((n, n, n), 4.0), eps0=2.0)
    assert abs(dte - 0.5) < 1e-15
    ex, ey, ez = oracle.field(p, phi)
    mag = np.sqrt(ex**2 + ey**2 + ez**2)
    assert emax == mag.max() and jmax == 4.0 * mag.max()
    sigma = np.zeros((n, n, n))
    sigma[2, 3, 4] = 7.0
    emax, jmax, dte = oracle.relaxation_time(p, phi, sigma)
    assert jmax == 7.0 * mag[2, 3, 4] and abs(dte - mag.max() / jmax) < 1e-15
