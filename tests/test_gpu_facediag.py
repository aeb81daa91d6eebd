"""GPU parity of the stored-face operator with a per-cell diagonal
(mg_set_face_coeffs_diag: faces allowed to vanish, plus d u), the symmetric
part of a cut-cell operator (paper Sec. 2, the embedded boundary
formalism), against the cut-cell oracle on problems without embedded faces:
there the oracle's operator is exactly kappa a u + aperture-weighted faces
(identity rows on covered cells), i.e. faces alpha_f beta_f and d = kappa a
(1 / h^2 on covered cells).

Solves stop at relative residual 1e-12 and agree with the oracle's direct
solution to 1e-9 relative L2; residuals agree element-wise to 1e-12 of the
largest."""
import numpy as np
import pytest

from oracle import eb_oracle as eb
from synth import geometry as geo
from synth.problems import Problem
from tests.gpu_util import dev, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1809_08857_amd import mg  # noqa: E402


def _harm(a, b):
    return 2.0 * a * b / (a + b)


def _case(dims, seed, covered=True):
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    h = 1.0 / max(dims)
    kappa = rng.uniform(0.3, 1.0, (nz, ny, nx))
    ax = rng.uniform(0.0, 1.0, (nz, ny, nx + 1))
    ay = rng.uniform(0.0, 1.0, (nz, ny + 1, nx))
    az = rng.uniform(0.0, 1.0, (nz + 1, ny, nx))
    for a in (ax, ay, az):  # some faces closed altogether
        a[rng.random(a.shape) < 0.1] = 0.0
    if covered:  # a block of covered cells with closed faces around it
        kappa[2:4, 3:6, 1:3] = 0.0
        ax[2:4, 3:6, 1:4] = 0.0
        ay[2:4, 3:7, 1:3] = 0.0
        az[2:5, 3:6, 1:3] = 0.0
    eps = np.exp(rng.uniform(-1.5, 1.5, (nz, ny, nx)))
    types = ["D" if t else "N" for t in rng.integers(0, 2, 6)]
    types[4] = "D"
    bc = tuple((t, float(rng.uniform(-1, 1)) if t == "D" else 0.0) for t in types)
    p = Problem(nx, ny, nz, h, 2.0, rng.standard_normal((nz, ny, nx)), eps, bc, f"facediag_{nx}x{ny}x{nz}")
    G = geo.Geometry(kappa, ax, ay, az, np.zeros(0, dtype=np.int64), np.zeros((0, 3)))
    return eb.EBProblem(p, G, 0.25, None, p.name)


def _engine_inputs(prob):
    q, G = prob.base, prob.geom
    e = q.eps
    bx = G.ax.copy()
    bx[:, :, 1:-1] *= _harm(e[:, :, :-1], e[:, :, 1:])
    bx[:, :, 0] *= e[:, :, 0]
    bx[:, :, -1] *= e[:, :, -1]
    by = G.ay.copy()
    by[:, 1:-1, :] *= _harm(e[:, :-1, :], e[:, 1:, :])
    by[:, 0, :] *= e[:, 0, :]
    by[:, -1, :] *= e[:, -1, :]
    bz = G.az.copy()
    bz[1:-1] *= _harm(e[:-1], e[1:])
    bz[0] *= e[0]
    bz[-1] *= e[-1]
    d = np.where(G.kappa > 0, G.kappa * q.a, 1.0 / q.h**2)
    return bx, by, bz, d


def _rhs(prob):
    """The oracle's right-hand side (kappa f plus box-face terms, g / h^2 on covered cells)."""
    return eb.rhs(prob)


DIMS = [(12, 10, 14), (64, 16, 16), (32, 32, 32)]


@pytest.mark.parametrize("k", range(len(DIMS)))
def test_face_diag_solve_matches_oracle(k):
    prob = _case(DIMS[k], 30 + k)
    q = prob.base
    print(f"face+diag case {q.name}", flush=True)
    bx, by, bz, d = _engine_inputs(prob)
    want = eb.solve(prob)
    b = _rhs(prob)
    desc = mg.mg_desc_default(q.nx, q.ny, q.nz, q.h, rtol=1e-12, max_cycles=200)
    ctx = mg.mg_create(desc)
    try:
        # the box-face values enter through b: zero values in the operator
        mg.mg_set_face_coeffs_diag(ctx, dev(bx), dev(by), dev(bz), dev(d), 0.0,
                                   mg.make_bcs(q.bc_types(), [0.0] * 6))
        x = torch.zeros(q.shape, dtype=torch.float64, device="cuda")
        rc, st = mg.mg_solve(ctx, dev(b), x)
        r = torch.empty_like(x)
        u0 = np.random.default_rng(7).standard_normal(q.shape)
        mg.mg_residual(ctx, dev(b), dev(u0), r)
        torch.cuda.synchronize()
        u, r = x.cpu().numpy(), r.cpu().numpy()
    finally:
        mg.mg_destroy(ctx)
    assert rc == mg.MG_OK, st.as_dict()
    assert rel_l2(u, want) <= 1e-9
    Am, bo = eb.assemble(prob)
    r_want = (bo - Am @ u0.reshape(-1)).reshape(q.shape)
    assert np.abs(r - r_want).max() <= 1e-12 * np.abs(r_want).max()


def test_face_diag_rejects_bad_input():
    prob = _case((12, 10, 14), 40, covered=False)
    q = prob.base
    bx, by, bz, d = _engine_inputs(prob)
    ctx = mg.mg_create(mg.mg_desc_default(q.nx, q.ny, q.nz, q.h))
    bcs = mg.make_bcs(q.bc_types(), [0.0] * 6)
    try:
        bad = d.copy()
        bad[1, 2, 3] = -1.0
        with pytest.raises(mg.MgError, match="diagonal entries"):
            mg.mg_set_face_coeffs_diag(ctx, dev(bx), dev(by), dev(bz), dev(bad), 0.0, bcs)
        # an isolated cell without a diagonal
        bx2, by2, bz2, d2 = bx.copy(), by.copy(), bz.copy(), d.copy()
        bx2[5, 5, 5:7] = 0.0
        by2[5, 5:7, 5] = 0.0
        bz2[5:7, 5, 5] = 0.0
        d2[5, 5, 5] = 0.0
        with pytest.raises(mg.MgError, match="no positive diagonal"):
            mg.mg_set_face_coeffs_diag(ctx, dev(bx2), dev(by2), dev(bz2), dev(d2), 0.0, bcs)
        with pytest.raises(mg.MgError, match="face coefficients"):
            bx3 = bx.copy()
            bx3[0, 0, 0] = -0.5
            mg.mg_set_face_coeffs_diag(ctx, dev(bx3), dev(by), dev(bz), dev(d), 0.0, bcs)
    finally:
        mg.mg_destroy(ctx)
