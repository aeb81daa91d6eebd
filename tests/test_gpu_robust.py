"""Failure handling and range of the engine, through the C ABI:

- divergence: a residual that keeps growing is reported as MG_EDIVERGED
  within a few cycles (single and batched solves); the growth is forced from
  the host by over-weighting the coarse-grid correction
  (MG_OPT_CORRECTION_WEIGHT), every kernel still runs its normal bounded
  loops;
- the FP32 / BF16 inner cycles of the refinement forms on operators and
  right-hand sides outside the FP32 range (coefficients near 1e30 or 1e-30,
  sources scaled by 1e-35 or 1e35): the inner problem is scaled by powers of
  two, and the solves reach the oracle's solution as for unscaled data;
  coefficient ranges beyond 2^70 are rejected for those forms;
- x-y planes wider than the reductions' 2048 partial sums (768 x 768): the
  reducing kernels then cover several tiles per workgroup."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import dev, gpu_solve, make_solver, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
from paper_1809_08857_amd import mg  # noqa: E402


def _rtol(p):
    return 1e-11 if p.a == 0.0 else 1e-10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_growing_residual_is_diverged(prec):
    p = synth.streamer_set(64, seed=3)[1]
    print(f"divergence {prec}", flush=True)
    s = make_solver(p, precision=prec, rtol=1e-10)
    try:
        f = dev(p.f)
        x = torch.zeros(p.shape, dtype=torch.float64, device="cuda")
        mg.mg_set_option(s.ctx, mg.MG_OPT_CORRECTION_WEIGHT, 3.5)
        with pytest.raises(mg.MgError) as ei:
            s.solve(f, x)
        assert ei.value.code == mg.MG_EDIVERGED
        print(mg.mg_last_error(), flush=True)
        # the plain weight converges again on the same context
        mg.mg_set_option(s.ctx, mg.MG_OPT_CORRECTION_WEIGHT, 1.0)
        x.zero_()
        rc, st = s.solve(f, x)
        assert rc == mg.MG_OK and st.rel_res <= 1e-10
        with pytest.raises(mg.MgError):
            mg.mg_set_option(s.ctx, mg.MG_OPT_CORRECTION_WEIGHT, 0.0)
        with pytest.raises(mg.MgError):
            mg.mg_set_option(s.ctx, 99, 1.0)
    finally:
        s.close()


def test_stall_at_rounding_floor_is_not_diverged():
    """A tolerance below the FP64 floor: the residual stalls and wobbles,
    which must end as MG_NOT_CONVERGED, not as a divergence."""
    p = synth.streamer_set(32, seed=4)[2]
    x, rc, st = gpu_solve(p, rtol=1e-18, max_cycles=30)
    assert rc == mg.MG_NOT_CONVERGED and st["cycles"] == 30
    assert st["rel_res"] < 1e-13


def test_batched_divergence_stops_that_problem_only():
    probs = synth.streamer_set(32, seed=5)[1:3] + synth.streamer_set(48, 32, 32, seed=6)[1:2]
    solvers = [make_solver(p, precision="fp32", rtol=1e-10) for p in probs]
    try:
        mg.mg_set_option(solvers[1].ctx, mg.MG_OPT_CORRECTION_WEIGHT, 3.5)
        fs = [dev(p.f) for p in probs]
        xs = [torch.zeros(p.shape, dtype=torch.float64, device="cuda") for p in probs]
        import ctypes
        n = len(probs)
        P = ctypes.c_void_p
        st = (mg.MgStats * n)()
        rc = mg.load().mg_solve_batched(n, (P * n)(*[s.ctx.value for s in solvers]),
                                        (P * n)(*[f.data_ptr() for f in fs]),
                                        (P * n)(*[x.data_ptr() for x in xs]), 0, st)
        print(rc, mg.mg_last_error(), [s.as_dict() for s in st], flush=True)
        assert rc == mg.MG_EDIVERGED
        assert st[1].cycles < 20
        for k in (0, 2):
            assert st[k].rel_res <= 1e-10
            assert rel_l2(xs[k].cpu().numpy(), oracle.solve_reference(probs[k])) <= 1e-9
    finally:
        for s in solvers:
            s.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("eps_scale", [1e30, 1e-30])
def test_lowp_coefficients_outside_fp32_range(prec, eps_scale):
    """The potential with its permittivity scaled by 1e30 or 1e-30 (the
    FP32 copies would overflow or underflow without the scaling): the same
    solution as the oracle's, to 1e-9."""
    p = synth.streamer_set(64, seed=7)[0]
    p.eps = p.eps * eps_scale
    p.f = p.f * eps_scale
    print(f"{prec} eps x {eps_scale:g}", flush=True)
    x, rc, st = gpu_solve(p, precision=prec, rtol=1e-11)
    print(st, flush=True)
    assert rc == mg.MG_OK
    ref = oracle.solve_reference(p)
    assert rel_l2(x, ref) <= 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("f_scale", [1e-35, 1e35])
def test_lowp_sources_outside_fp32_range(prec, f_scale):
    p = synth.streamer_set(64, seed=8)[1]
    p.f = p.f * f_scale
    print(f"{prec} f x {f_scale:g}", flush=True)
    x, rc, st = gpu_solve(p, precision=prec, rtol=1e-10)
    x_u, rc_u, st_u = gpu_solve(synth.streamer_set(64, seed=8)[1], precision=prec, rtol=1e-10)
    print(st, st_u, flush=True)
    assert rc == mg.MG_OK and rc_u == mg.MG_OK
    assert abs(st["cycles"] - st_u["cycles"]) <= 1
    assert rel_l2(x, oracle.solve_reference(p)) <= 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_lowp_rejects_coefficient_range_beyond_2_70(prec):
    p = synth.streamer_set(32, seed=9)[0]
    p.eps = np.where(p.eps > 2.0, 1e-15, 1e10)  # ratio 1e25
    with pytest.raises(mg.MgError) as ei:
        make_solver(p, precision=prec)
    assert ei.value.code == mg.MG_EINVAL
    x, rc, st = gpu_solve(p, rtol=1e-10)  # FP64 takes it
    assert rc == mg.MG_OK


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_wide_planes_768(prec):
    """768 x 768 x 64: more column tiles per plane than a reduction has
    partial sums; the strongly screened photon group (fast to converge, so
    the oracle can finish from the GPU's answer)."""
    p = synth.streamer_set(768, 768, 64, seed=10)[3]
    print(f"wide planes {prec}", flush=True)
    x, rc, st = gpu_solve(p, precision=prec, rtol=1e-10)
    print(st, flush=True)
    assert rc == mg.MG_OK
    _, rn, bn = oracle.residual(p, x)
    assert rn / bn <= 1e-10 * 1.001
    ref, cyc, rel = oracle.solve_vcycle(p, rtol=1e-13, max_cycles=20, u0=x)
    assert rel <= 1e-13
    assert rel_l2(x, ref) <= 1e-9
