"""Benchmark of the multigrid engine on one MI355X.

Workload (one "step"): the four elliptic solves of one field update at
256^3 — the variable-permittivity potential (dielectric slab + seeded
streamer filament) and the three screened photon-group equations
(kappa_i h = 0.05, 0.3, 1.5) — each from a zero guess to relative residual
1e-10, in FP64 V-cycles.  Inputs are generated once on the host, copied to
HBM, and stay resident; the timed region covers whole solves only.

Prints one JSON line:  solves/s (value), DoF/s, ms per step, the roofline of
the dominant kernel (the finest-level red-black smoother of the potential,
timed live with HIP events inside the library) and the CPU oracle timed on
a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    return ap.parse_args()


def cpu_baseline(n: int, seed: int):
    """The oracle as it stands: lexicographic Gauss-Seidel V(2,2) cycles on
    the host, timed on the potential solve of the same 256^3 set (one solve:
    a bounded sample of the four-solve step)."""
    import oracle
    import synth
    p = synth.streamer_set(n, seed=seed)[0]
    oracle.build(force=False)
    t = time.perf_counter()
    _, cycles, rel = oracle.solve_vcycle(p, rtol=1e-10, max_cycles=50)
    dt = time.perf_counter() - t
    return {"value": 1.0 / dt, "unit": "solves/s", "cores": oracle.threads(), "kind": "oracle",
            "sample": f"1 of the 4 solves (potential, seed {seed}) at {n}^3, lexicographic GS V(2,2) "
                      f"to rel. residual 1e-10: {cycles} cycles, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not part of this build",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_1809_08857_amd import mg

    torch.cuda.set_device(0)
    n = args.n
    probs = synth.streamer_set(n, seed=args.seed)
    f_dev = torch.from_numpy(probs[0].f).cuda()  # the same source drives all four
    ctxs, xs = [], []
    for p in probs:
        eps = torch.from_numpy(p.eps).cuda() if p.eps is not None else None
        # the potential is solved one decade tighter: its error/residual
        # ratio is ~10-25, and the 1e-9 agreement with the oracle must hold
        rtol = 1e-11 if p.a == 0.0 else 1e-10
        s = mg.Solver(p.nx, p.ny, p.nz, p.h, eps=eps, a=p.a, bc_types=p.bc_types(), bc_values=p.bc_values(),
                      precision=args.precision, rtol=rtol)
        ctxs.append(s)
        xs.append(torch.zeros(p.shape, dtype=torch.float64, device="cuda"))
        del eps
    if args.autotune:
        for s in ctxs:
            mg.mg_autotune(s.ctx, 3)
    torch.cuda.synchronize()

    def step():
        cyc = []
        for s, x in zip(ctxs, xs):
            rc, st = s.solve(f_dev, x)
            if rc != mg.MG_OK:
                raise RuntimeError(f"solve did not converge: {st.as_dict()}")
            cyc.append(st.cycles)
        return cyc

    for _ in range(args.warmup):
        step()
    mg.mg_timing(ctxs[0].ctx, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cycles = []
    for _ in range(args.steps):
        cycles.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kern_ms, kname, bytes_per_launch = mg.mg_timing_read(ctxs[0].ctx)
    mg.mg_timing(ctxs[0].ctx, 0)

    solves = 4 * args.steps
    value = solves / dt
    cells = n**3
    roof = None
    if launches > 0:
        avg_s = kern_ms / launches / 1e3
        achieved = bytes_per_launch / avg_s / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": kname,
                "avg_us": round(avg_s * 1e6, 2), "launches": launches,
                "algorithmic_bytes_per_launch": bytes_per_launch}
    out = {
        "metric": "elliptic solves/s (Poisson+3 Helmholtz) & DoF/s at 256^3, rel-residual 1e-10",
        "value": round(value, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else f"f64+{args.precision}",
        "data": "synthetic",
        "config": {"workload": f"streamer field update: potential (eps slab) + 3 photon groups at {n}^3, "
                               f"zero guess to rel. residual 1e-10 (potential 1e-11)", "grid": [n, n, n],
                   "solves_per_step": 4, "precision": args.precision,
                   "cycles_per_solve": [int(c) for c in np.mean(np.array(cycles), axis=0).round()]},
        "dof_per_s": round(value * cells, 1),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n, args.seed)
    for s in ctxs:
        s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
