"""What the trained network gains: at 128^3, on unseen filament sources
(test seeds), the three photon-group solves started from the U-net guess
need fewer V-cycles than from zero, no guess is rejected, and the solutions
still agree with the FP64 oracle to 1e-9 relative L2 at relative residual
1e-10.  Weights: paper_1809_08857_amd/weights/unet128.mglw, trained by
paper_1809_08857_amd.train_guess on seeds 0..1999."""
import os
import time

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import rel_l2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1809_08857_amd import learned as L  # noqa: E402
from paper_1809_08857_amd import mg  # noqa: E402
from paper_1809_08857_amd.train_guess import TEST_SEED0, helmholtz_solvers  # noqa: E402

N = 128
WEIGHTS = os.path.join(L.WEIGHTS_DIR, f"unet{N}.mglw")


@pytest.fixture(scope="module")
def setup():
    if not os.path.exists(WEIGHTS):
        pytest.fail(f"trained weights missing: {WEIGHTS}")
    solvers, k2 = helmholtz_solvers(N)
    net = L.mgl_create(N, N, N)
    L.mgl_load(net, WEIGHTS)
    yield solvers, k2, net
    for s in solvers:
        s.close()
    L.mgl_destroy(net)


def _set(solvers, k2, net, s, learned):
    xs = [torch.zeros((N, N, N), dtype=torch.float64, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if learned:
        L.mgl_predict(net, s, k2, xs)
    stats = []
    for sv, x in zip(solvers, xs):
        rc, st = sv.solve(s, x, mg.MG_GUESS if learned else 0)
        assert rc == mg.MG_OK
        stats.append(st.as_dict())
    torch.cuda.synchronize()
    return xs, stats, time.perf_counter() - t0


def test_learned_guess_saves_cycles(setup):
    solvers, k2, net = setup
    seeds = range(TEST_SEED0, TEST_SEED0 + 4)
    saved, t_plain, t_learned = [], 0.0, 0.0
    for seed in seeds:
        s = torch.from_numpy(synth.filament_source(N, N, N, seed)).cuda()
        _set(solvers, k2, net, s, True)  # warm-up
        x0, st0, dt0 = _set(solvers, k2, net, s, False)
        x1, st1, dt1 = _set(solvers, k2, net, s, True)
        t_plain += dt0
        t_learned += dt1
        for a, b in zip(st0, st1):
            assert b["fell_back"] == 0
            assert b["rel_res"] <= 1e-10 and a["rel_res"] <= 1e-10
        saved.append([a["cycles"] - b["cycles"] for a, b in zip(st0, st1)])
        # the guesses themselves are within a few per cent of the solution
        g = [torch.zeros_like(x0[0]) for _ in range(3)]
        L.mgl_predict(net, s, k2, g)
        for gi, xi in zip(g, x0):
            assert (torch.linalg.norm(gi - xi) / torch.linalg.norm(xi)).item() < 0.05
    saved = np.array(saved)
    print("cycles saved per solve", saved.mean(axis=0), f"set time plain {t_plain / 4 * 1e3:.2f} ms, "
          f"learned {t_learned / 4 * 1e3:.2f} ms (inference included)", flush=True)
    assert saved.min() >= 0
    assert saved.sum(axis=1).mean() >= 3


def test_learned_solutions_match_oracle(setup):
    solvers, k2, net = setup
    seed = TEST_SEED0 + 7
    probs = synth.streamer_set(N, seed=seed)[1:]
    s = torch.from_numpy(probs[0].f).cuda()
    xs, st, _ = _set(solvers, k2, net, s, True)
    for p, x, sti in zip(probs, xs, st):
        ref = oracle.solve_reference(p)
        assert rel_l2(x.cpu().numpy(), ref) <= 1e-9, (p.name, sti)
