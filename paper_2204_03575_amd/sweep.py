"""Parameter sweep of many independent 2D runs on one GPU.

Runs are grouped by mesh size; each group is one batched solver
(chm_create_batch): its runs share the assembled matrices and both AMG
hierarchies, every kernel launch of a time step covers all of them, and the
SELL-64 and coarsest-level kernels serve several runs per lane (each matrix
entry a lane loads is used for runs_per_lane runs).  The groups advance
concurrently (chm_step_many): each on its own HIP stream, driven by its own
host thread, so the latency-bound launches of one group overlap the others.
An autotuner picks, per group, the runs per lane and then the preconditioner
settings (Chebyshev degree and interval of the As hierarchy, CG steps per As
solve), each with the shortest time per step measured on the group itself,
from the same state, at the same residual tolerance.  All
computation runs in the library; this module only schedules it.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SIZES = (128, 192, 256, 384, 512)
# The tuner starts from the workload's own settings (the 512x512 preset: As
# smoother of degree 7 over [rho/5, rho], 2 CG steps per As solve; 2 runs per
# lane), then tries the other runs per lane, then the other As settings with
# the best runs per lane; a candidate replaces the best only when it is at
# least TUNE_MARGIN faster (timing noise must not pick a worse setting).
TUNE_PREC = [dict(cheb_degree=d, schur_pcg=k, cheb_ratio=r)
             for (d, k, r) in ((7, 2, 5.0), (6, 2, 5.0), (5, 2, 8.0), (4, 2, 15.0))]
TUNE_RB = (2, 1, 4)
TUNE_MARGIN = 0.03
TUNE_WARMUP, TUNE_STEPS = 2, 3


def draw_runs(count: int = 64, seed: int = 20220700):
    """count runs: mesh size uniform in SIZES, chi_pn uniform in [0.6, 1.4], solvent
    removal uniform in [1e-3, 5e-3] per step until the solvent fraction has dropped
    by 0.5, initial-noise seed per run."""
    sys.path.insert(0, ROOT)
    import synthetic as S
    u = S.uniform01(seed, 3 * count).reshape(count, 3)
    runs = []
    for k in range(count):
        n = SIZES[min(int(u[k, 0] * len(SIZES)), len(SIZES) - 1)]
        evap = 1e-3 + 4e-3 * u[k, 2]
        runs.append(dict(n=n, chi_pn=0.6 + 0.8 * u[k, 1], evap_ds=evap,
                         evap_steps=int(round(0.5 / evap)), seed=seed + 1 + k))
    return runs


def groups(runs):
    out = {}
    for r in runs:
        out.setdefault(r["n"], []).append(r)
    return dict(sorted(out.items()))


def make_group(n: int, runs, base: dict, stream=None):
    """The batched solver of one group (on `stream`, a torch stream, or the
    current one), every run set to its initial state."""
    import synthetic as S
    from .chm import Solver
    p = dict(S.preset("square512", n=(n, n)), **base)
    co, ce = S.make_mesh(p)
    rl = [dict(chi_pn=r["chi_pn"], evap_ds=r["evap_ds"], evap_steps=r["evap_steps"]) for r in runs]
    g = Solver(co, ce, p, runs=rl, stream=None if stream is None else stream.cuda_stream)
    for i, r in enumerate(runs):
        php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"], seed=r["seed"])
        g.set_fields(php, phn, run=i)
    return g, co.shape[0]


def timed_steps(g, steps: int):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = g.step(steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st


def timed_many(gs, steps: int):
    """`steps` time steps of every solver of gs, concurrently (chm_step_many)."""
    import torch
    from .chm import step_many
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = step_many(gs, steps)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, st


def _time_candidate(n, runs, base, cand, steps, log):
    g, _ = make_group(n, runs, dict(base, **cand))
    g.step(TUNE_WARMUP)
    dt, _ = timed_steps(g, steps)
    del g
    log(f"#   {n}x{n} {cand}: {1e3 * dt / steps:.2f} ms/step")
    return dt


def autotune(n: int, runs, base: dict, steps: int = TUNE_STEPS, log=print):
    """Per group, the settings with the shortest time per step (TUNE_WARMUP
    warm-up steps, then `steps` timed ones, from the group's initial state
    each time): runs per lane first (TUNE_RB, with the first TUNE_PREC
    entry, the workload's own), then the As settings (TUNE_PREC) with the
    best runs per lane."""
    best = dict(TUNE_PREC[0], runs_per_lane=TUNE_RB[0])
    best_t = _time_candidate(n, runs, base, best, steps, log)

    def trial(cand):
        nonlocal best, best_t
        dt = _time_candidate(n, runs, base, cand, steps, log)
        if dt < (1.0 - TUNE_MARGIN) * best_t:
            best, best_t = cand, dt

    if len(runs) > 1:
        for rb in TUNE_RB[1:]:
            trial(dict(best, runs_per_lane=rb))
    for prec in TUNE_PREC[1:]:
        trial(dict(prec, runs_per_lane=best["runs_per_lane"]))
    return best


def iters_of(stats, batched: bool):
    flat = [s for step in stats for s in (step if batched else [step])]
    return sum(s["iters"][0] + s["iters"][1] for s in flat)
