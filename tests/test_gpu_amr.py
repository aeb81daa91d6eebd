"""GPU parity of the composite two-level (AMR) solves (paper Secs. 2-4: the
elliptic equations on a base grid refined by patches, second-order
cell-centred discretisation) against the composite oracle, through the C
ABI (mga_create, mga_set_coeffs, mga_apply, mga_solve).

- mga_apply agrees with the oracle's assembled operator element by element
  to 1e-12 of the largest entry (the two sides sum the same terms in
  different orders).
- mga_solve at rtol 1e-12: the oracle's own residual of the GPU answer is
  within 2 rtol (volume-weighted L2, as the solver measures it), and the
  answer agrees with the oracle's sparse direct solution to 1e-8 relative
  L2 (the composite operators here have condition numbers below 1e4).
- Covered base cells hold the mean of their eight children.
- At the benchmark size (a 256^3 base grid refined around the filament) the
  oracle evaluates the residual row by row at sampled cells, among them
  every kind of cell beside a coarse-fine interface; each sampled residual
  is bounded by the solver's final residual norm."""
import numpy as np
import pytest

import synth
from oracle import amr_oracle as amr
from synth.problems import Problem, streamer_composite
from tests.gpu_util import dev, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1809_08857_amd import mg  # noqa: E402

BOXES16 = [((4, 6, 8), (12, 14, 20)), ((16, 4, 6), (28, 12, 14)), ((6, 18, 18), (14, 28, 28))]


def _case(k):
    if k == 0:  # cube base, three boxes, cell permittivity, mixed faces, a > 0
        n = 16
        rng = np.random.default_rng(11)
        bc = (("D", 0.3), ("N", 0.0), ("D", -1.0), ("N", 0.0), ("N", 0.0), ("D", 2.0))
        p = Problem(n, n, n, 1.0 / n, 1.5, rng.standard_normal((n, n, n)),
                    np.exp(rng.uniform(-1.5, 1.5, (n, n, n))), bc, "amr_mixed16")
        shapes = [(hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]) for lo, hi in BOXES16]
        return amr.Composite(p, BOXES16, [rng.standard_normal(s) for s in shapes],
                             [np.exp(rng.uniform(-1.5, 1.5, s)) for s in shapes], p.name)
    if k == 1:  # ragged base, beta = 1, Poisson with one Dirichlet pair, boxes of unequal sides
        rng = np.random.default_rng(12)
        nx, ny, nz = 24, 20, 14
        bc = (("N", 0.0), ("N", 0.0), ("N", 0.0), ("N", 0.0), ("D", 0.0), ("D", 1.0))
        p = Problem(nx, ny, nz, 1.0 / nz, 0.0, rng.standard_normal((nz, ny, nx)), None, bc, "amr_ragged")
        boxes = [((2, 4, 4), (18, 10, 12)), ((24, 16, 2), (46, 38, 26))]
        shapes = [(hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0]) for lo, hi in boxes]
        return amr.Composite(p, boxes, [rng.standard_normal(s) for s in shapes], None, p.name)
    if k == 2:  # the filament recipe at 32^3 with 8^3-coarse boxes (16^3 fine)
        base, boxes, ff, ef = streamer_composite(32, seed=3, box=8)
        return amr.Composite(base, boxes, ff, ef, "amr_streamer32")
    raise IndexError(k)


CASES = [0, 1, 2]


class _Gpu:
    def __init__(self, comp, rtol=1e-12, max_cycles=300):
        q = comp.base
        self.comp = comp
        self.desc = mg.mg_desc_default(q.nx, q.ny, q.nz, q.h, rtol=rtol, max_cycles=max_cycles)
        self.ctx = mg.mga_create(self.desc, comp.boxes)
        eb = dev(q.eps) if q.eps is not None else None
        ef = [dev(e) for e in comp.eps_fine] if comp.eps_fine is not None else None
        if eb is None and ef is not None:  # beta = 1 on the base, given on the boxes
            eb = torch.ones(q.shape, dtype=torch.float64, device="cuda")
        if ef is None and eb is not None:
            ef = [torch.ones(f.shape, dtype=torch.float64, device="cuda") for f in comp.f_fine]
        mg.mga_set_coeffs(self.ctx, eb, ef, q.a, mg.make_bcs(q.bc_types(), q.bc_values()))

    def solve(self, guess=None):
        q, comp = self.comp.base, self.comp
        xb = dev(guess[0]) if guess else torch.zeros(q.shape, dtype=torch.float64, device="cuda")
        xf = [dev(a) for a in guess[1]] if guess else [torch.zeros(f.shape, dtype=torch.float64, device="cuda")
                                                        for f in comp.f_fine]
        rc, st = mg.mga_solve(self.ctx, dev(q.f), [dev(f) for f in comp.f_fine], xb, xf,
                              mg.MG_GUESS if guess else 0)
        torch.cuda.synchronize()
        return rc, st, xb.cpu().numpy(), [a.cpu().numpy() for a in xf]

    def apply(self, ub, uf):
        yb = torch.empty(ub.shape, dtype=torch.float64, device="cuda")
        yf = [torch.empty(a.shape, dtype=torch.float64, device="cuda") for a in uf]
        mg.mga_apply(self.ctx, dev(ub), [dev(a) for a in uf], yb, yf)
        torch.cuda.synchronize()
        return yb.cpu().numpy(), [a.cpu().numpy() for a in yf]

    def close(self):
        mg.mga_destroy(self.ctx)


def _unknowns(comp, ub, uf):
    mask = amr.coverage(comp.base.nx, comp.base.ny, comp.base.nz, comp.boxes) < 0
    return np.concatenate([ub[mask]] + [a.ravel() for a in uf])


@pytest.mark.parametrize("k", CASES)
def test_apply_matches_oracle(k):
    comp = _case(k)
    print(f"amr apply case {comp.name} boxes={comp.boxes}", flush=True)
    rng = np.random.default_rng(100 + k)
    ub = rng.standard_normal(comp.base.shape)
    uf = [rng.standard_normal(f.shape) for f in comp.f_fine]
    want_b, want_f = amr.apply(comp, ub, uf)
    g = _Gpu(comp)
    try:
        got_b, got_f = g.apply(ub, uf)
    finally:
        g.close()
    scale = max(np.abs(want_b).max(), max(np.abs(a).max() for a in want_f))
    assert np.abs(got_b - want_b).max() <= 1e-12 * scale
    for a, b in zip(got_f, want_f):
        assert np.abs(a - b).max() <= 1e-12 * scale


@pytest.mark.parametrize("k", CASES)
def test_solve_matches_oracle(k):
    comp = _case(k)
    print(f"amr solve case {comp.name} boxes={comp.boxes}", flush=True)
    want_b, want_f = amr.solve(comp)
    zb = np.zeros(comp.base.shape)
    assert abs(_weighted_rhs_norm(comp) - amr.residual(comp, zb, [np.zeros(f.shape) for f in comp.f_fine])[1]) \
        <= 1e-12 * _weighted_rhs_norm(comp)
    g = _Gpu(comp, rtol=1e-12)
    try:
        rc, st, ub, uf = g.solve()
    finally:
        g.close()
    assert rc == mg.MG_OK, st.as_dict()
    rn, bn = amr.residual(comp, ub, uf)
    assert rn <= 2e-12 * bn, (rn / bn, st.as_dict())
    assert abs(st.rel_res - rn / bn) <= 1e-3 * st.rel_res + 1e-15
    assert rel_l2(_unknowns(comp, ub, uf), _unknowns(comp, want_b, want_f)) <= 1e-8
    # covered base cells: the mean of their eight children
    for (lo, hi), a in zip(comp.boxes, uf):
        avg = a.reshape(a.shape[0] // 2, 2, a.shape[1] // 2, 2, a.shape[2] // 2, 2).mean(axis=(1, 3, 5))
        cov = ub[lo[2] // 2:hi[2] // 2, lo[1] // 2:hi[1] // 2, lo[0] // 2:hi[0] // 2]
        assert np.abs(cov - avg).max() <= 1e-14 * max(np.abs(avg).max(), 1e-300)


def test_without_boxes_is_the_single_grid_solve():
    p = synth.random_problem(24, 16, 20, 7)
    comp = amr.Composite(p, [], [], None if p.eps is None else [], "amr_nobox")
    print("amr no-box case", flush=True)
    g = _Gpu(comp, rtol=1e-12)
    try:
        rc, st, ub, _ = g.solve()
    finally:
        g.close()
    assert rc == mg.MG_OK
    want, _ = amr.solve(comp)
    assert rel_l2(ub, want) <= 1e-8


def test_guess_at_the_solution_stops_at_once():
    comp = _case(0)
    want_b, want_f = amr.solve(comp)
    g = _Gpu(comp, rtol=1e-10)
    try:
        rc, st, ub, uf = g.solve(guess=(want_b, want_f))
    finally:
        g.close()
    assert rc == mg.MG_OK and st.cycles == 0 and st.rel_res0 <= 1e-10


def test_full_size_sampled_residual():
    base, boxes, ff, ef = streamer_composite(256, seed=0)
    comp = amr.Composite(base, boxes, ff, ef, "amr_streamer256")
    print(f"amr full-size case boxes={boxes}", flush=True)
    g = _Gpu(comp, rtol=1e-10, max_cycles=100)
    try:
        rc, st, ub, uf = g.solve()
    finally:
        g.close()
    assert rc == mg.MG_OK, st.as_dict()
    # sampled rows: random uncovered base cells, random fine cells, and the
    # cells on both sides of each box's faces (edges and corners included)
    rng = np.random.default_rng(1)
    mask = amr.coverage(base.nx, base.ny, base.nz, boxes)
    cells = []
    while len(cells) < 60:
        I, J, K = (int(v) for v in rng.integers(0, 256, 3))
        if mask[K, J, I] < 0:
            cells.append(("c", I, J, K))
    for p, (lo, hi) in enumerate(boxes):
        for _ in range(20):
            cells.append(("f", p, *(int(rng.integers(lo[d], hi[d])) for d in range(3))))
        for d in range(3):
            for side in (lo[d], hi[d] - 1):
                for t in range(8):
                    c = [int(rng.integers(lo[e], hi[e])) if t & (1 << e) else (lo[e] if t & 4 else hi[e] - 1)
                         for e in range(3)]
                    c[d] = side
                    cells.append(("f", p, *c))
                    C = [v // 2 for v in c]
                    C[d] += 1 if side == hi[d] - 1 else -1
                    cells.append(("c", *C))
    r = amr.residual_at(comp, ub, uf, cells)
    w = np.array([comp.base.h ** 3 if c[0] == "c" else (comp.base.h / 2) ** 3 for c in cells])
    bnorm = _weighted_rhs_norm(comp)
    assert np.all(np.sqrt(w) * np.abs(r) <= 1.01 * st.rel_res * bnorm + 1e-300), (r, st.as_dict())


def _weighted_rhs_norm(comp):
    """||b|| of the composite problem (volume-weighted), from the source and
    the Dirichlet faces (the rows' right-hand sides) without assembling A."""
    q = comp.base
    mask = amr.coverage(q.nx, q.ny, q.nz, comp.boxes) < 0
    b = np.array(q.f, dtype=np.float64, copy=True)
    beta = np.ones(q.shape) if q.eps is None else np.asarray(q.eps)
    ic2 = 1.0 / q.h ** 2
    for d, (t, v) in enumerate(q.bc):
        if t != "D":
            continue
        axis, hi = 2 - d // 2, d % 2
        sl = [slice(None)] * 3
        sl[axis] = -1 if hi else 0
        b[tuple(sl)] += 2.0 * beta[tuple(sl)] * ic2 * v
    s = q.h ** 3 * np.sum(b[mask] ** 2) + (q.h / 2) ** 3 * sum(np.sum(f ** 2) for f in comp.f_fine)
    return float(np.sqrt(s))
