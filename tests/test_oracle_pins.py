"""Pins of the CPU FP64 oracle against facts the mathematics fixes.

The paper prints no worked example for its elliptic solves, so every pin is a
closed form of the discrete problem, an invariant, or a brute-force dense
solve of tiny grids (assembled independently in pure Python).  Each pin is
chosen so that a plausible slip in the oracle fails it:

* wrong Dirichlet ghost (factor 1 instead of 2), wrong sign, dropped term,
  swapped axes -> closed-form solutions on non-cubic boxes (P1, P4, linear);
* arithmetic instead of harmonic face means, wrong boundary coefficient ->
  layered permittivity (P3);
* asymmetric assembly -> symmetry (P5) and the dense solve (P6);
* broken restriction/prolongation -> mesh-independent V-cycle counts (P8).
"""
import numpy as np
import pytest

import oracle
import synth
from synth.problems import Problem


def _centres(n, h):
    return (np.arange(n) + 0.5) * h


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- P1 / P2


def manufactured_discrete_exact(nx, ny, nz):
    """Exact solution of the discrete config-1 problem: cell-centred cosine
    modes are Neumann eigenvectors, sine modes with the linear ghost are
    Dirichlet eigenvectors and linear functions are reproduced exactly."""
    h = 1.0 / nz
    lx, ly = nx * h, ny * h
    x, y, z = _centres(nx, h), _centres(ny, h), _centres(nz, h)
    amp = np.pi**2 / lx**2 + np.pi**2 / ly**2 + 4 * np.pi**2
    lam = (4 / h**2) * (np.sin(np.pi * h / (2 * lx)) ** 2 + np.sin(np.pi * h / (2 * ly)) ** 2
                        + np.sin(np.pi * h) ** 2)
    mode = (np.sin(2 * np.pi * z)[:, None, None] * np.cos(np.pi * y / ly)[None, :, None]
            * np.cos(np.pi * x / lx)[None, None, :])
    return z[:, None, None] + (amp / lam) * mode, z[:, None, None] + mode


@pytest.mark.parametrize("dims", [(8, 8, 8), (16, 16, 16), (32, 32, 32), (8, 12, 16), (24, 8, 16)])
def test_p1_manufactured_discrete_exact(dims):
    p = synth.manufactured_poisson(*dims)
    exact, _ = manufactured_discrete_exact(*dims)
    u, cycles, rel = oracle.solve_vcycle(p, rtol=1e-13)
    assert rel <= 1e-13
    assert _rel(u, exact) < 1e-11
    if p.cells <= 4096:
        ucg, _, rel_cg = oracle.solve_cg(p, rtol=1e-13)
        assert _rel(ucg, exact) < 1e-11


def test_p2_second_order():
    errs = []
    for n in (8, 16, 32):
        p = synth.manufactured_poisson(n)
        _, cont = manufactured_discrete_exact(n, n, n)
        u = oracle.solve_reference(p)
        errs.append(np.sqrt(np.mean((u - cont) ** 2)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.5 < r1 < 4.1 and 3.8 < r2 < 4.1, errs


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_linear_along_each_axis(axis):
    """Dirichlet g0/g1 on the two faces normal to one axis, Neumann elsewhere,
    f = 0, beta = 1: u is exactly the linear interpolant at cell centres."""
    dims = [6, 10, 14]
    n = dims[axis]
    h = 0.1
    types = [("N", 0.0)] * 6
    g0, g1 = -0.7, 2.3
    types[2 * axis] = ("D", g0)
    types[2 * axis + 1] = ("D", g1)
    nx, ny, nz = dims
    p = Problem(nx, ny, nz, h, 0.0, np.zeros((nz, ny, nx)), None, tuple(types))
    s = _centres(n, h) / (n * h)
    lin = g0 + (g1 - g0) * s
    shape = [1, 1, 1]
    shape[2 - axis] = n
    exact = np.broadcast_to(lin.reshape(shape), (nz, ny, nx))
    u, _, rel = oracle.solve_cg(p, rtol=1e-14)
    assert np.abs(u - exact).max() < 1e-11


# ---------------------------------------------------------------- P3


@pytest.mark.parametrize("axis", [0, 2])
def test_p3_layered_permittivity_exact(axis):
    """eps = 4 below an interface lying on a face, 1 above, no charge,
    grounded at 0 and 1 V at the far face: the discrete solution equals the
    continuum piecewise-linear potential (constant displacement flux q)."""
    n, m, kI = 32, 4, 7
    h = 1.0 / n
    coord = _centres(n, h)
    eps1d = np.where(np.arange(n) < kI, 4.0, 1.0)
    types = [("N", 0.0)] * 6
    types[2 * axis] = ("D", 0.0)
    types[2 * axis + 1] = ("D", 1.0)
    if axis == 2:
        nx, ny, nz = m, m, n
        eps = np.broadcast_to(eps1d[:, None, None], (nz, ny, nx)).copy()
    else:
        nx, ny, nz = n, m, m
        eps = np.broadcast_to(eps1d[None, None, :], (nz, ny, nx)).copy()
    p = Problem(nx, ny, nz, h, 0.0, np.zeros((nz, ny, nx)), eps, tuple(types))
    zI = kI * h
    q = 1.0 / (zI / 4 + 1 - zI)
    lin = np.where(coord < zI, q * coord / 4, q * zI / 4 + q * (coord - zI))
    exact = (np.broadcast_to(lin[:, None, None], (nz, ny, nx)) if axis == 2
             else np.broadcast_to(lin[None, None, :], (nz, ny, nx)))
    u, _, rel = oracle.solve_vcycle(p, rtol=1e-14, coarsest_max=4)
    assert np.abs(u - exact).max() < 1e-11


def test_p3_generator_slab_interface():
    """The generator's slab (eps = 4 for cell centres below z = 0.1) puts the
    interface on the face k = ceil(0.1 nz - 1/2); with rho = 0 the potential
    is the layered closed form with that interface."""
    n = 40
    p = synth.streamer_set(4, 4, n, seed=0)[0]
    p.f = np.zeros_like(p.f)
    kI = int(np.sum(_centres(n, 1.0 / n) < 0.1))
    zI = kI / n
    q = 1.0 / (zI / 4 + 1 - zI)
    z = _centres(n, 1.0 / n)
    lin = np.where(z < zI, q * z / 4, q * zI / 4 + q * (z - zI))
    u, _, _ = oracle.solve_cg(p, rtol=1e-14)
    assert np.abs(u - lin[:, None, None]).max() < 1e-11


# ---------------------------------------------------------------- P4


def test_p4_helmholtz_neumann_constant():
    nx, ny, nz = 6, 8, 10
    kap2 = 37.0
    f = np.full((nz, ny, nx), 3.5)
    p = Problem(nx, ny, nz, 0.1, kap2, f, None, (("N", 0.0),) * 6)
    u, _, _ = oracle.solve_cg(p, rtol=1e-14)
    assert np.abs(u - 3.5 / kap2).max() < 1e-13


@pytest.mark.parametrize("kdx", [0.05, 0.3, 1.5])
def test_p4_helmholtz_dirichlet_sine_mode(kdx):
    nx, ny, nz = 12, 16, 20
    h = 1.0 / nz
    L = (nx * h, ny * h, nz * h)
    x, y, z = _centres(nx, h), _centres(ny, h), _centres(nz, h)
    f = (np.sin(np.pi * z / L[2])[:, None, None] * np.sin(np.pi * y / L[1])[None, :, None]
         * np.sin(np.pi * x / L[0])[None, None, :])
    a = (kdx / h) ** 2
    lam = (4 / h**2) * sum(np.sin(np.pi * h / (2 * Ld)) ** 2 for Ld in L)
    p = Problem(nx, ny, nz, h, a, f, None, (("D", 0.0),) * 6)
    u, _, _ = oracle.solve_vcycle(p, rtol=1e-14)
    assert np.abs(u - f / (a + lam)).max() < 1e-12 * np.abs(f / (a + lam)).max() * 100


# ---------------------------------------------------------------- P5 / P6


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p5_symmetry(seed):
    p = synth.random_problem(7, 5, 6, seed)
    rng = np.random.default_rng(100 + seed)
    u = rng.standard_normal(p.shape)
    v = rng.standard_normal(p.shape)
    lhs = np.vdot(u, oracle.apply(p, v))
    rhs = np.vdot(oracle.apply(p, u), v)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_p5_spd_dense():
    p = synth.streamer_set(8, seed=3)[0]
    A, _ = oracle.dense_matrix(p)
    assert np.allclose(A, A.T, rtol=0, atol=1e-12 * np.abs(A).max())
    lam = np.linalg.eigvalsh(A)
    assert lam.min() > 0


@pytest.mark.parametrize("dims,seed", [((8, 8, 8), 0), ((8, 8, 8), 1), ((8, 4, 6), 2), ((6, 8, 4), 3),
                                       ((4, 6, 8), 4)])
def test_p6_dense_bruteforce(dims, seed):
    p = synth.random_problem(*dims, seed)
    A, b = oracle.dense_matrix(p)
    # the two independent assemblies agree on random vectors
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(p.shape)
    assert _rel(oracle.apply(p, w).reshape(-1), A @ w.reshape(-1)) < 1e-14
    assert _rel(oracle.rhs(p).reshape(-1), b) < 1e-14
    ud = np.linalg.solve(A, b).reshape(p.shape)
    ucg, _, _ = oracle.solve_cg(p, rtol=1e-14)
    uvc, _, rel = oracle.solve_vcycle(p, rtol=1e-14, coarsest_max=2)
    assert _rel(ucg, ud) < 1e-11
    assert _rel(uvc, ud) < 1e-11


# ---------------------------------------------------------------- P7


def test_p7_neumann_helmholtz_conservation():
    p = synth.random_problem(8, 6, 10, 5, variable_eps=True, a=20.0, bc=(("N", 0.0),) * 6)
    u, _, _ = oracle.solve_cg(p, rtol=1e-14)
    assert abs(p.a * u.sum() - p.f.sum()) < 1e-11 * np.abs(p.f).sum()


def test_p7_discrete_divergence_theorem():
    """Interior fluxes telescope: sum(A u) - a sum(u) equals the Dirichlet
    boundary outflow h^-2 sum 2 beta_P u_P over boundary cells."""
    p = synth.random_problem(6, 7, 8, 9)
    rng = np.random.default_rng(1)
    u = rng.standard_normal(p.shape)
    Au = oracle.apply(p, u)
    ih2 = 1 / p.h**2
    beta = p.eps
    out = 0.0
    t = p.bc_types()
    if t[0] == "D": out += np.sum(2 * beta[:, :, 0] * u[:, :, 0])
    if t[1] == "D": out += np.sum(2 * beta[:, :, -1] * u[:, :, -1])
    if t[2] == "D": out += np.sum(2 * beta[:, 0, :] * u[:, 0, :])
    if t[3] == "D": out += np.sum(2 * beta[:, -1, :] * u[:, -1, :])
    if t[4] == "D": out += np.sum(2 * beta[0] * u[0])
    if t[5] == "D": out += np.sum(2 * beta[-1] * u[-1])
    lhs = Au.sum() - p.a * u.sum()
    assert abs(lhs - ih2 * out) < 1e-11 * ih2 * np.abs(u).sum()


# ---------------------------------------------------------------- P8


def test_p8_mesh_independent_cycles():
    counts = []
    for n in (16, 32, 64):
        for p in synth.streamer_set(n, seed=1):
            _, c, rel = oracle.solve_vcycle(p, rtol=1e-10)
            assert rel <= 1e-10
            counts.append(c)
    counts = np.array(counts).reshape(3, 4)
    assert counts.max() <= 14, counts
    assert (counts.max(0) - counts.min(0)).max() <= 3, counts


# ---------------------------------------------------------------- smoother


@pytest.mark.parametrize("seed", [0, 1])
def test_rbgs_black_residual_zero_after_sweep(seed):
    """After a red-black sweep every black cell satisfies its own equation
    (its neighbours, all red, do not change after it), while red cells in
    general do not; a black-first sweep would show the opposite."""
    p = synth.random_problem(9, 7, 6, seed)
    rng = np.random.default_rng(seed)
    u = oracle.rbgs(p, rng.standard_normal(p.shape), 1)
    r, _, bn = oracle.residual(p, u)
    k, j, i = np.indices(p.shape)
    black = ((i + j + k) & 1) == 1
    assert np.abs(r[black]).max() < 1e-12 * np.abs(r).max() + 1e-13 * bn
    assert np.abs(r[~black]).max() > 1e-6 * np.abs(r).max()


def test_rbgs_fixed_point_and_convergence():
    p = synth.random_problem(8, 8, 8, 7)
    ud = oracle.dense_solve(p)
    assert _rel(oracle.rbgs(p, ud, 1), ud) < 1e-13
    u = oracle.rbgs(p, np.zeros(p.shape), 400)
    assert _rel(u, ud) < 1e-8


# ------------------------------------------------------ prolongation pins
# Trilinear cell-centred prolongation (weights 3/4 and 1/4 per axis, ghost
# values reflected across the box faces, negated at Dirichlet faces).


def test_prolong_preserves_constants_with_neumann_faces():
    e = np.full((3, 5, 4), 2.5)
    u = oracle.prolong_add(e, np.zeros((6, 10, 8)), ["N"] * 6)
    assert np.allclose(u, 2.5, rtol=0, atol=1e-15)


def test_prolong_reproduces_linear_fields_inside():
    """Away from the faces the interpolation is exact for linear fields, on
    a box with three different extents and three different slopes (a
    swapped axis or a wrong weight breaks it)."""
    nzc, nyc, nxc = 4, 5, 6
    H = 0.2
    Zc, Yc, Xc = np.meshgrid(*[(np.arange(n) + 0.5) * H for n in (nzc, nyc, nxc)], indexing="ij")
    lin = lambda x, y, z: 0.3 + 1.7 * x - 0.9 * y + 2.3 * z  # noqa: E731
    e = lin(Xc, Yc, Zc)
    u0 = np.random.default_rng(5).standard_normal((2 * nzc, 2 * nyc, 2 * nxc))
    u = oracle.prolong_add(e, u0, ["N", "D", "N", "D", "D", "N"])
    Zf, Yf, Xf = np.meshgrid(*[(np.arange(2 * n) + 0.5) * H / 2 for n in (nzc, nyc, nxc)], indexing="ij")
    inner = (slice(1, -1),) * 3
    assert np.allclose((u - u0)[inner], lin(Xf, Yf, Zf)[inner], rtol=0, atol=1e-13)


def test_prolong_dirichlet_ghost_halves_boundary_cells():
    """A constant correction c next to a Dirichlet face: the ghost is -c, so a
    fine cell touching one face gets c/2, an edge cell c/4, a corner c/8."""
    c = 3.0
    u = oracle.prolong_add(np.full((3, 3, 3), c), np.zeros((6, 6, 6)), ["D"] * 6)
    assert u[3, 3, 3] == pytest.approx(c)
    assert u[3, 3, 0] == pytest.approx(c / 2) and u[3, 0, 3] == pytest.approx(c / 2)
    assert u[0, 3, 3] == pytest.approx(c / 2)
    assert u[3, 0, 5] == pytest.approx(c / 4)
    assert u[0, 0, 0] == pytest.approx(c / 8) and u[5, 5, 5] == pytest.approx(c / 8)
    # a Neumann face reflects without a sign: the same cell keeps c
    u = oracle.prolong_add(np.full((3, 3, 3), c), np.zeros((6, 6, 6)), ["N", "D", "D", "D", "D", "D"])
    assert u[3, 3, 0] == pytest.approx(c) and u[3, 3, 5] == pytest.approx(c / 2)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("level", [1, 2])
def test_coarse_level_layered_exact(axis, level):
    """The coarse operators are rediscretisations: a coarse face takes the
    mean of the four fine faces it covers.  For permittivity layered along
    one axis with the interface on a coarse face, the coarse equation then
    has the same exact solution as the fine one: the continuum
    piecewise-linear potential sampled at the coarse cell centres (each
    coarse face between two layers holds the harmonic mean of the two, the
    flux-continuous value; a face taken from the wrong fine plane would hold
    a layer's own value and shift the kink).  The Dirichlet value 1 of the
    far face enters the homogeneous coarse equation as the right-hand side
    2 beta g / h_l^2 of the cells beside it (beta = 1 there)."""
    n, m, kI = 32, 4, 8
    h = 1.0 / n
    eps1d = np.where(np.arange(n) < kI, 4.0, 1.0)
    types = [("N", 0.0)] * 6
    types[2 * axis] = ("D", 0.0)
    types[2 * axis + 1] = ("D", 1.0)
    shape = [m, m, m]  # (nz, ny, nx)
    shape[2 - axis] = n
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    eps = np.broadcast_to(eps1d.reshape(bshape), shape).copy()
    nz, ny, nx = shape
    p = Problem(nx, ny, nz, h, 0.0, np.zeros(shape), eps, tuple(types))
    hl = h * 2**level
    nl = n >> level
    coord = _centres(nl, hl)
    zI = kI * h
    q = 1.0 / (zI / 4 + 1 - zI)
    lin = np.where(coord < zI, q * coord / 4, q * zI / 4 + q * (coord - zI))
    lx, ly, lz = oracle.level_dims(p, level)
    lshape = [1, 1, 1]
    lshape[2 - axis] = nl
    exact = np.broadcast_to(lin.reshape(lshape), (lz, ly, lx))
    b = np.zeros((lz, ly, lx))
    sl = [slice(None)] * 3
    sl[2 - axis] = nl - 1
    b[tuple(sl)] = 2.0 / hl**2
    u = np.zeros_like(b)
    for _ in range(40):
        u = oracle.rbgs_level(p, level, b, u, 100)
    assert np.abs(u - exact).max() < 1e-11


def test_rbgs_level_zero_is_the_homogeneous_finest_sweep():
    """Level 0 of rbgs_level is the finest operator with zero boundary
    values: the same as rbgs on the problem with every Dirichlet value set to
    0 and f = b."""
    p = synth.random_problem(12, 10, 8, 31)
    rng = np.random.default_rng(5)
    b = rng.standard_normal(p.shape)
    u0 = rng.standard_normal(p.shape)
    q = Problem(p.nx, p.ny, p.nz, p.h, p.a, b, p.eps, tuple((t, 0.0) for t, _ in p.bc))
    assert np.array_equal(oracle.rbgs_level(p, 0, b, u0, 2), oracle.rbgs(q, u0, 2))
