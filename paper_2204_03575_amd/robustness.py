"""The paper's solver-robustness experiments (Section 4), run on the GPU.

The paper solves the first 20 time steps of its film problem with MINRES and
Algorithm 1 (AMG solves to a relative residual of 1e-4, MINRES to 1e-7) and
reports, per time step, the larger iteration count of the two species and
the time per linear system, for: 2D meshes of 100 x 50 up to 3200 x 1600
points on the 10 x 2.5 rectangle; 3D meshes of 30 x 15 x 30 up to
160 x 80 x 160 points on the 10 x 2.5 x 10 box; the interface parameter eps
from 1e-4 to 10 and the time step tau from 1e-7 to 1e-4 on the 800 x 400
mesh.  This module runs the same sweeps (polynomial potential, evaporation
inflow on the top, patterned substrate at the bottom, phi_p = phi_n = 0.35
+- 0.01) with three solver variants:

  paper   MINRES, stationary AMG solves to 1e-4 (at most 30 cycles);
  minres  MINRES, two stationary V-cycles per AMG solve (a fixed operator);
  fgmres  the production setting: FGMRES(30), CG steps per As solve chosen
          at setup from the measured V-cycle contraction (2 up to 0.3, 4 up
          to 0.6, else 6), HIP graphs.

Each case prints one JSON line: mesh, parameters, the worst (over species)
iteration count of every step, the time per step (both species, measured
around each step with the device synchronised), and the setup time.  The
paper's own figures (its CPU, per linear system) are in PAPER_FIGURES for
context.  With --after N every variant starts from the state after N time
steps of the production solver (the same state for all three, fields and
chemical potentials), as in the paper's runs after 1000 steps on the 2D
meshes (Section 4, Fig. 2).  All computation runs in the library.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

MESHES_2D = [(100, 50), (200, 100), (400, 200), (800, 400), (1600, 800), (3200, 1600)]
MESHES_3D = [(30, 15, 30), (40, 20, 40), (60, 30, 60), (80, 40, 80), (120, 60, 120),
             (160, 80, 160)]
EPS = [1e-4, 1e-3, 1e-2, 1e-1, 1.0, 10.0]
TAU = [1e-7, 1e-6, 1e-5, 1e-4]
SWEEP_MESH = (800, 400)

# The paper's figures: worst iteration count over the 20 steps and seconds per
# linear system (one species) on its 6-core desktop CPU.
PAPER_FIGURES = {
    "mesh2d": {(100, 50): (15, 0.089), (200, 100): (14, 0.23), (400, 200): (14, 1.03),
               (800, 400): (13, 4.06), (1600, 800): (12, 18.8), (3200, 1600): (10, 84.3)},
    "mesh3d": {(30, 15, 30): (8, 0.136), (40, 20, 40): (10, 0.32), (60, 30, 60): (12, 1.43),
               (80, 40, 80): (12, 3.16), (120, 60, 120): (12, 13.3),
               (160, 80, 160): (12, 30.5)},
    "eps": {1e-4: (17, 4.82), 1e-3: (13, 4.06), 1e-2: (10, 3.35), 1e-1: (9, 3.49),
            1.0: (8, 3.92), 10.0: (7, 4.15)},
    "tau": {1e-7: (10, 2.32), 1e-6: (11, 2.83), 1e-5: (12, 3.44), 1e-4: (13, 4.0)},
    # steps 1001 to 1020 (Fig. 2)
    "mesh2d_after1000": {(100, 50): (15, 0.086), (200, 100): (16, 0.27), (400, 200): (15, 1.06),
                         (800, 400): (14, 4.42), (1600, 800): (13, 20.3)},
}

VARIANTS = {
    "paper": dict(krylov="minres", schur_pcg=0, amg_cycles=30, amg_tol=1e-4, use_graphs=0),
    "minres": dict(krylov="minres", schur_pcg=0, amg_cycles=2, amg_tol=0.0, use_graphs=0),
    "fgmres": dict(krylov="fgmres", schur_pcg=-1, amg_cycles=2, amg_tol=0.0, use_graphs=1),
}


def case_params(points, variant: str, **kw) -> dict:
    """The film problem on a mesh of `points` (vertices per direction)."""
    sys.path.insert(0, ROOT)
    import synthetic as S
    dim = len(points)
    extent = (10.0, 2.5) if dim == 2 else (10.0, 2.5, 10.0)
    cells = tuple(int(q) - 1 for q in points)
    p = S.preset("paper2d", dim=dim, n=cells, extent=extent, rtol=1e-7, max_iters=1000,
                 coarse_max=2048)
    p.update(VARIANTS[variant])
    p.update(kw)
    return p


def advance(points, nsteps: int, log=None, chunk: int = 100, **kw):
    """The state after `nsteps` time steps of the production solver from the
    seeded initial state: (phi_p, phi_n, mu_p, mu_n) as host arrays."""
    import torch
    import synthetic as S
    from .chm import Solver
    p = case_params(points, "fgmres", **kw)
    co, ce = S.make_mesh(p)
    g = Solver(co, ce, p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    t0 = time.perf_counter()
    done = 0
    while done < nsteps:
        k = min(chunk, nsteps - done)
        st = g.step(k)      # raises on a failed step
        done += k
        if log:
            torch.cuda.synchronize()
            log(f"# advance {tuple(points)}: {done} of {nsteps} steps, "
                f"{time.perf_counter() - t0:.1f} s, last iterations {st[-1]['iters']}")
    f = g.get_fields()
    del g
    return f["phi_p"], f["phi_n"], f["mu_p"], f["mu_n"]


def run_case(points, variant: str, steps: int = 20, log=None, start=None, **kw) -> dict:
    import numpy as np
    import torch
    import synthetic as S
    from .chm import ChmError, Solver
    p = case_params(points, variant, **kw)
    tm = time.perf_counter()
    co, ce = S.make_mesh(p)
    t0 = time.perf_counter()
    g = Solver(co, ce, p)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    if start is None:
        php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
        g.set_fields(php, phn)
    else:
        g.set_fields(*start)
    if log:
        log(f"# {variant} {tuple(points)}: mesh {t0 - tm:.2f} s, setup {setup_s:.2f} s, "
            f"initial state {time.perf_counter() - t0 - setup_s:.2f} s")
    iters, times, status = [], [], "ok"
    for k in range(steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        try:
            st = g.step(1)[0]
        except ChmError as e:
            status = f"stopped: {e}"
            break
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        iters.append(max(st["iters"]))
        if log:
            log(f"# {variant} {tuple(points)} step {k}: iterations {st['iters']}, "
                f"{times[-1]:.4f} s")
    tf = time.perf_counter()
    f = g.get_fields()
    k_cg, rho = g.schur_info()
    out = dict(points=list(points), vertices=int(co.shape[0]), unknowns=int(4 * co.shape[0]),
               variant=variant, eps=p["eps"], tau=p["tau"], steps=len(iters), status=status,
               schur_pcg=k_cg, vcycle_contraction=round(rho, 4),
               worst_iters=iters, max_iters=max(iters) if iters else None,
               s_per_step=[round(x, 6) for x in times],
               median_s_per_step=float(np.median(times)) if times else None,
               setup_s=round(setup_s, 3),
               phi_range=[float(min(f["phi_p"].min(), f["phi_n"].min())),
                          float(max(f["phi_p"].max(), f["phi_n"].max()))])
    del g
    if log:
        log(f"# {variant} {tuple(points)}: fields and teardown {time.perf_counter() - tf:.2f} s")
    return out


def _count(pts) -> int:
    v = 1
    for q in pts:
        v *= q
    return v


def cases(sweep: str, max_vertices: int):
    def fits(pts):
        return _count(pts) <= max_vertices
    if sweep == "mesh2d":
        return [(m, {}, ("mesh2d", m)) for m in MESHES_2D if fits(m)]
    if sweep == "mesh3d":
        return [(m, {}, ("mesh3d", m)) for m in MESHES_3D if fits(m)]
    if sweep == "eps":
        return [(SWEEP_MESH, dict(eps=e), ("eps", e)) for e in EPS]
    if sweep == "tau":
        return [(SWEEP_MESH, dict(tau=t), ("tau", t)) for t in TAU]
    raise ValueError(sweep)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--sweep", default="mesh2d", choices=["mesh2d", "mesh3d", "eps", "tau"])
    ap.add_argument("--variants", default="paper,minres,fgmres")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--max-vertices", type=int, default=6_000_000)
    ap.add_argument("--min-vertices", type=int, default=0)
    ap.add_argument("--after", type=int, default=0, metavar="N",
                    help="start every variant from the state after N production steps")
    ap.add_argument("--progress", action="store_true", help="log every step on stderr")
    a = ap.parse_args(argv)
    log = (lambda m: print(m, file=sys.stderr, flush=True)) if a.progress else None
    for pts, kw, key in cases(a.sweep, a.max_vertices):
        if _count(pts) < a.min_vertices:
            continue
        fig = key[0] + (f"_after{a.after}" if a.after else "")
        ref = PAPER_FIGURES.get(fig, {}).get(key[1])
        start = advance(pts, a.after, log=log, **kw) if a.after else None
        for v in a.variants.split(","):
            r = run_case(pts, v, a.steps, log=log, start=start, **kw)
            r["sweep"] = a.sweep
            r["after_steps"] = a.after
            r["paper_worst_iters"], r["paper_s_per_system"] = ref if ref else (None, None)
            print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
