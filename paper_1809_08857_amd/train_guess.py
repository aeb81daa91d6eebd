"""Train the learned initial guess of the three photon-group solves.

Data: for each seed, the streamer source s of the seeded filament generator
and the three converged screened solutions Psi_i of (kappa_i^2 - lap) Psi_i
= s (homogeneous Dirichlet faces, kappa_i h = 0.05, 0.3, 1.5), solved by
this package's multigrid engine in FP64 to relative residual 1e-10.  The
network learns t_i = kappa_i^2 Psi_i / (max|s| scale_i) with the mgl_*
kernels (mean-squared error, Adam, cosine learning-rate decay).

    python -m paper_1809_08857_amd.train_guess --n 128 --train 2000 --val 200 \
        --epochs 8 --out paper_1809_08857_amd/weights/unet128.mglw

Seeds: training 0 .. train-1, validation 2000 .. 2000+val-1 (test seeds
3000+ are left for evaluation).  Every sample stays resident on the GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

VAL_SEED0 = 2000
TEST_SEED0 = 3000


def _source(args):
    n, seed = args
    from synth.problems import filament_source
    return seed, filament_source(n, n, n, seed)


def helmholtz_solvers(n: int, precision: str = "fp64"):
    """The three photon-group operators at n^3 (coefficients independent of
    the source): returns (solvers, kappa2)."""
    import synth
    from paper_1809_08857_amd import mg
    probs = synth.streamer_set(n, seed=0)[1:]
    solvers = [mg.Solver(p.nx, p.ny, p.nz, p.h, eps=None, a=p.a, bc_types=p.bc_types(), bc_values=p.bc_values(),
                         precision=precision, rtol=1e-10) for p in probs]
    return solvers, [p.a for p in probs]


def generate(n: int, seeds, solvers, kappa2, net, pool, log=print):
    """Sources and targets of the given seeds, on the device."""
    import torch
    from paper_1809_08857_amd import learned as L, mg
    S, T = [], []
    t0 = time.time()
    for k, (seed, s) in enumerate(pool.imap(_source, [(n, int(q)) for q in seeds], chunksize=2)):
        sd = torch.from_numpy(s).cuda()
        psi = [torch.zeros((n, n, n), dtype=torch.float64, device="cuda") for _ in range(3)]
        for sv, x in zip(solvers, psi):
            rc, st = sv.solve(sd, x)
            if rc != mg.MG_OK:
                raise RuntimeError(f"seed {seed}: solve failed {st.as_dict()}")
        t = torch.empty((n, n, n, 3), dtype=torch.float32, device="cuda")
        L.mgl_make_target(net, sd, psi, kappa2, t)
        S.append(sd)
        T.append(t)
        if (k + 1) % 200 == 0:
            log(f"  generated {k + 1}/{len(seeds)} ({time.time() - t0:.0f} s)")
    return S, T


def fit_scales(n, solvers, kappa2, net, pool, count=32):
    """scale_i = mean over `count` training sources of max|kappa_i^2 Psi_i| / max|s|."""
    from paper_1809_08857_amd import learned as L
    import torch
    L.mgl_set_scales(net, (1.0, 1.0, 1.0))
    acc = np.zeros(3)
    for seed, s in pool.imap(_source, [(n, q) for q in range(count)]):
        sd = torch.from_numpy(s).cuda()
        psi = [torch.zeros((n, n, n), dtype=torch.float64, device="cuda") for _ in range(3)]
        for sv, x in zip(solvers, psi):
            sv.solve(sd, x)
        t = torch.empty((n, n, n, 3), dtype=torch.float32, device="cuda")
        acc += np.array(L.mgl_make_target(net, sd, psi, kappa2, t, want_max=True))
    return tuple(float(a) for a in acc / count)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--train", type=int, default=2000)
    ap.add_argument("--val", type=int, default=200)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-min", type=float, default=2e-5)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", required=True)
    ap.add_argument("--log", default=None)
    args = ap.parse_args(argv)

    logf = open(args.log, "a") if args.log else None

    def log(msg):
        print(msg, flush=True)
        if logf:
            logf.write(msg + "\n")
            logf.flush()

    pool = mp.get_context("spawn").Pool(args.workers)
    import torch
    from paper_1809_08857_amd import learned as L
    torch.cuda.set_device(0)
    n = args.n
    solvers, kappa2 = helmholtz_solvers(n)
    net = L.mgl_create(n, n, n)
    L.mgl_init_params(net, args.seed)
    scales = fit_scales(n, solvers, kappa2, net, pool)
    L.mgl_set_scales(net, scales)
    log(f"scales {scales}")
    t0 = time.time()
    S, T = generate(n, range(args.train), solvers, kappa2, net, pool, log)
    VS, VT = generate(n, range(VAL_SEED0, VAL_SEED0 + args.val), solvers, kappa2, net, pool, log)
    pool.close()
    log(f"data: {len(S)} train, {len(VS)} val pairs in {time.time() - t0:.0f} s")

    def val_loss():
        return float(np.mean([L.mgl_eval_loss(net, s, t) for s, t in zip(VS, VT)]))

    rng = np.random.default_rng(args.seed)
    steps_per_epoch = len(S) // args.batch
    total = steps_per_epoch * args.epochs
    step = 0
    log(f"epoch 0 val {val_loss():.4e}")
    best = math.inf
    history = []
    for ep in range(args.epochs):
        order = rng.permutation(len(S))
        t1 = time.time()
        run = 0.0
        for b in range(steps_per_epoch):
            idx = order[b * args.batch:(b + 1) * args.batch]
            lr = args.lr_min + 0.5 * (args.lr - args.lr_min) * (1 + math.cos(math.pi * step / total))
            run += L.mgl_train_step(net, [S[i] for i in idx], [T[i] for i in idx], lr=lr)
            step += 1
            if (b + 1) % 100 == 0:
                log(f"  epoch {ep + 1} step {b + 1}/{steps_per_epoch} train {run / (b + 1):.4e} lr {lr:.2e}")
        v = val_loss()
        history.append({"epoch": ep + 1, "train": run / steps_per_epoch, "val": v, "s": time.time() - t1})
        log(f"epoch {ep + 1} train {run / steps_per_epoch:.4e} val {v:.4e} ({time.time() - t1:.0f} s)")
        if v < best:
            best = v
            os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
            L.mgl_save(net, args.out)
    log(json.dumps({"scales": scales, "best_val": best, "history": history}))
    for sv in solvers:
        sv.close()
    L.mgl_destroy(net)


if __name__ == "__main__":
    main()
