"""mg_residual_noalloc (no context, no device allocation, reductions on the
library's static scratch array) against mg_residual on the same inputs:
the same kernels and the same reduction order, so r and both norms agree
bit for bit.  Two calls in a row, the second on a smaller grid (the scratch
keeps the first call's contents)."""
import numpy as np
import pytest

import synth
from tests.gpu_util import dev, make_solver

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1809_08857_amd import mg  # noqa: E402


def _check(p, seed):
    rng = np.random.default_rng(seed)
    u = dev(rng.standard_normal(p.shape))
    f = dev(p.f)
    eps = dev(p.eps) if p.eps is not None else None
    s = make_solver(p)
    try:
        r_ref = torch.empty(p.shape, dtype=torch.float64, device="cuda")
        rn_ref, bn_ref = s.residual(f, u, r_ref)
    finally:
        s.close()
    desc = mg.mg_desc_default(p.nx, p.ny, p.nz, p.h)
    bcs = mg.make_bcs(p.bc_types(), p.bc_values())
    r = torch.full(p.shape, 7.0, dtype=torch.float64, device="cuda")
    rn, bn = mg.mg_residual_noalloc(desc, eps, p.a, bcs, f, u, r)
    torch.cuda.synchronize()
    print(p.name, rn, rn_ref, bn, bn_ref, flush=True)
    assert torch.equal(r, r_ref)
    assert rn == rn_ref and bn == bn_ref
    rn2, bn2 = mg.mg_residual_noalloc(desc, eps, p.a, bcs, f, u)  # norms only
    assert rn2 == rn_ref and bn2 == bn_ref


def test_noalloc_residual_matches_mg_residual_twice():
    _check(synth.streamer_set(96, 64, 80, seed=1)[0], 1)           # cell eps, Dirichlet values
    _check(synth.random_problem(40, 24, 20, 2, variable_eps=False), 2)  # smaller, beta = 1


def test_noalloc_residual_rejects_bad_input():
    p = synth.random_problem(16, 16, 16, 3)
    desc = mg.mg_desc_default(16, 16, 16, p.h)
    bcs = mg.make_bcs(p.bc_types(), p.bc_values())
    f, u = dev(p.f), dev(np.zeros(p.shape))
    bad = p.eps.copy()
    bad[2, 3, 4] = -1.0
    with pytest.raises(mg.MgError):
        mg.mg_residual_noalloc(desc, dev(bad), p.a, bcs, f, u)
    desc.nx = 0
    with pytest.raises(mg.MgError):
        mg.mg_residual_noalloc(desc, dev(p.eps), p.a, bcs, f, u)
