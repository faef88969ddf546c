"""Training of the learned initial guess on trajectories the solver produces.

Everything numeric runs in the library (time steps, features, network,
gradients, Adam); this module only schedules it: it runs a set of seeded 2D
evaporation runs, keeps every state vector in device memory, draws training
crops (step triples n-2, n-1, n of one run, random crop origins), and calls
chm_net_train_step.  The run parameters follow the workload the guess is for:
a 2D unit square of n x n squares, the Flory-Huggins free energy with chi_pn
drawn per run, solvent removed per step at a per-run rate until the solvent
fraction has dropped by 0.5.

Command line (writes the FP32 parameters as a .npy file):

    python -m paper_2204_03575_amd.guess_train --n 256 --runs 40 --steps 500 \\
        --iters 4000 --out paper_2204_03575_amd/weights/guess256.npy
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def run_params(n: int, k: int, seed: int, chi_range=(0.6, 1.4), evap_range=(1e-3, 5e-3), **extra):
    """Parameters of run k: chi_pn and the evaporation rate drawn from the
    seeded stream, initial noise seed seed + k."""
    sys.path.insert(0, ROOT)
    import synthetic as S
    u = S.uniform01(seed + 7919 * (k + 1), 2)
    chi = chi_range[0] + (chi_range[1] - chi_range[0]) * u[0]
    evap = evap_range[0] + (evap_range[1] - evap_range[0]) * u[1]
    p = S.preset("square512", n=(n, n), chi_pn=float(chi), evap_ds=float(evap),
                 evap_steps=int(round(0.5 / evap)), **extra)
    return p, seed + k


def generate(n: int, runs: int, steps: int, seed: int, precision: str = "fp64", log=print):
    """Solutions of every step's solve (before solvent removal) of every run: a
    list of CUDA tensors [steps + 1, 4 (n+1)^2] (row 0: the initial state)."""
    import torch
    import synthetic as S
    from .chm import Solver
    trajs = []
    co, ce = S.make_mesh(S.preset("square512", n=(n, n)))
    nv = co.shape[0]
    t0 = time.perf_counter()
    for k in range(runs):
        p, s = run_params(n, k, seed)
        g = Solver(co, ce, dict(p, precision=precision))
        php, phn, _ = S.initial_fractions(nv, p["mean_p"], p["mean_n"], seed=s)
        g.set_fields(php, phn)
        X = torch.empty((steps + 1, 4 * nv), dtype=torch.float64, device="cuda")
        X[0] = g.get_state(solution=True)
        for i in range(steps):
            g.step(1)
            X[i + 1] = g.get_state(solution=True)
        trajs.append(X)
        del g
        log(f"# run {k + 1}/{runs} (chi_pn {p['chi_pn']:.3f}, evaporation {p['evap_ds']:.4f}/step): "
            f"{steps} steps, {time.perf_counter() - t0:.1f} s so far")
    return trajs


def train(net, trajs, H: int, W: int, iters: int, batch: int = 32, crop: int = 64,
          lr: float = 1e-3, lr_min: float = 1e-5, seed: int = 1, log=print, log_every: int = 200,
          smooth: float = 0.0):
    """Adam on random crops; cosine step-size decay from lr to lr_min."""
    rng = np.random.default_rng(seed)
    crop_h, crop_w = min(crop, H), min(crop, W)
    losses = []
    t0 = time.perf_counter()
    for it in range(iters):
        a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * it / max(1, iters)))
        r = rng.integers(0, len(trajs), batch)
        steps = [trajs[i].shape[0] for i in r]
        nn = [int(rng.integers(2, s)) for s in steps]
        x2 = [trajs[i][m - 2] for i, m in zip(r, nn)]
        x1 = [trajs[i][m - 1] for i, m in zip(r, nn)]
        x0 = [trajs[i][m] for i, m in zip(r, nn)]
        oy = rng.integers(0, H - crop_h + 1, batch)
        ox = rng.integers(0, W - crop_w + 1, batch)
        loss = net.train_step(H, W, crop_h, crop_w, x2, x1, x0, oy, ox, a, smooth)
        losses.append(loss)
        if log_every and ((it + 1) % log_every == 0 or it == 0):
            log(f"# train {it + 1}/{iters}: loss {np.mean(losses[-log_every:]):.4e} "
                f"(lr {a:.2e}, {time.perf_counter() - t0:.1f} s)")
    return losses


def evaluate(net, n: int, run_ids, steps: int, seed: int, modes=("previous", "linear", "learned"),
             precision: str = "fp64", log=print):
    """Runs run_ids (the same seeded runs as generate) with each start mode:
    mean FGMRES iterations per species and step, geometric mean of the
    starting relative residual, how often each start was chosen, time per step."""
    import torch
    import synthetic as S
    from .chm import Solver
    co, ce = S.make_mesh(S.preset("square512", n=(n, n)))
    nv = co.shape[0]
    H = W = n + 1
    out = {}
    for mode in modes:
        its, r0, used, ms = [], [], np.zeros(3), 0.0
        for k in run_ids:
            p, s = run_params(n, k, seed)
            g = Solver(co, ce, dict(p, precision=precision))
            php, phn, _ = S.initial_fractions(nv, p["mean_p"], p["mean_n"], seed=s)
            g.set_fields(php, phn)
            g.set_guess(mode, net if mode == "learned" else None, H, W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = g.step(steps)
            torch.cuda.synchronize()
            ms += 1e3 * (time.perf_counter() - t0) / steps / len(run_ids)
            for x in st:
                its += list(x["iters"])
                r0 += list(x["res0"])
                for u in x["guess_used"]:
                    used[u] += 1
            del g
        out[mode] = {"iters_per_species_step": float(np.mean(its)),
                     "res0_geomean": float(np.exp(np.mean(np.log(np.maximum(r0, 1e-300))))),
                     "start_chosen": {"previous": int(used[0]), "linear": int(used[1]),
                                      "learned": int(used[2])},
                     "ms_per_step": ms}
        log(f"# {mode}: {out[mode]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--runs", type=int, default=40)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--iters", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--crop", type=int, default=64)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--smooth", type=float, default=0.0,
                    help="weight of the neighbour-difference term of the loss")
    ap.add_argument("--seed", type=int, default=20220500)
    ap.add_argument("--holdout", type=int, default=2, help="runs kept out of training")
    ap.add_argument("--out", default=os.path.join(HERE, "weights", "guess256.npy"))
    args = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    import synthetic as S
    from .chm import Net
    torch.cuda.init()
    log = lambda s: print(s, file=sys.stderr, flush=True)
    H = W = args.n + 1
    trajs = generate(args.n, args.runs + args.holdout, args.steps, args.seed, log=log)
    train_set, hold = trajs[:args.runs], trajs[args.runs:]
    net = Net(max(args.batch * args.crop * args.crop, H * W))
    net.set_params(S.net_init(seed=args.seed, zero_last=True))
    t0 = time.perf_counter()
    losses = train(net, train_set, H, W, args.iters, args.batch, args.crop, args.lr, log=log,
                   smooth=args.smooth)
    t_train = time.perf_counter() - t0
    del trajs, train_set, hold
    torch.cuda.empty_cache()
    quality = evaluate(net, args.n, range(args.runs, args.runs + args.holdout), args.steps,
                       args.seed, log=log)
    flat = net.get_params(flat=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out, flat)
    summary = {"n": args.n, "runs": args.runs, "steps": args.steps, "snapshots": args.runs * (args.steps + 1),
               "iters": args.iters, "batch": args.batch, "crop": args.crop, "lr": args.lr,
               "smooth": args.smooth,
               "seed": args.seed, "train_seconds": t_train,
               "loss_first_200": float(np.mean(losses[:200])), "loss_last_200": float(np.mean(losses[-200:])),
               "holdout": quality, "out": args.out}
    print(json.dumps(summary), flush=True)


if __name__ == "__main__":
    main()
