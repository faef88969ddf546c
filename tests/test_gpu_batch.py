"""GPU: batched solvers (several runs on one mesh sharing matrices and AMG
hierarchies, every launch covering all runs).

Each run of a batch performs, per run, exactly the operations of a solver
that holds that run alone (same kernels, same per-run partial-sum grids and
summation orders, its own Krylov control), so its trajectory must equal the
single-run trajectory bitwise: fields, iteration counts and residuals.  The
single-run solver is itself checked against the oracle elsewhere; one batched
run is also compared with the oracle directly here (1e-10, equal iterations).
"""
import numpy as np
import pytest

import synthetic as S
from oracle import Oracle

pytestmark = pytest.mark.gpu

FIELDS = ("phi_p", "phi_n", "mu_p", "mu_n")


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_03575_amd import library
    library()


def case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def run_list(k, seed=5):
    rng = np.random.default_rng(seed)
    return [dict(chi_pn=float(rng.uniform(0.6, 1.4)), evap_ds=float(rng.uniform(1e-3, 5e-3)),
                 evap_steps=int(rng.integers(1, 4))) for _ in range(k)]


def initial(nv, r, p):
    return S.initial_fractions(nv, p["mean_p"], p["mean_n"], seed=S.BASE_SEED + 100 + r)[:2]


# the preconditioner settings of the 512x512 workload (Chebyshev mass solve,
# 2 CG steps of degree-6 V-cycles over [rho/5, rho])
W512 = dict(mass_solver="chebyshev", cheb_degree_mass=5, cheb_degree=6, cheb_ratio=5.0,
            schur_pcg=2)


BOX = dict(dim=3, n=(6, 5, 4), extent=(1.0, 1.0, 0.8))


@pytest.mark.parametrize("runs,precision,guess,extra", [
    (1, "fp64", "previous", {}), (5, "fp64", "previous", {}), (7, "fp32", "previous", {}),
    (4, "fp64", "linear", {}), (3, "fp32", "linear", W512),
    (5, "fp64", "previous", dict(runs_per_lane=1)), (5, "fp64", "linear", dict(runs_per_lane=4)),
    (6, "fp32", "linear", dict(W512, runs_per_lane=4)), (7, "fp32", "previous", dict(runs_per_lane=4)),
    (3, "fp64", "previous", dict(BOX, runs_per_lane=4)), (5, "fp32", "previous", dict(BOX)),
    (5, "fp64", "linear", dict(ortho="cgs2")), (4, "fp32", "previous", dict(BOX, ortho="cgs2"))],
    ids=["1-fp64", "5-fp64", "7-fp32", "4-fp64-linear", "3-fp32-linear-w512", "5-fp64-rb1",
         "5-fp64-linear-rb4", "6-fp32-linear-w512-rb4", "7-fp32-rb4", "3-fp64-3d-rb4",
         "5-fp32-3d", "5-fp64-linear-cgs2", "4-fp32-3d-cgs2"])
def test_batch_runs_equal_single_runs_bitwise(runs, precision, guess, extra):
    case("batch vs single runs", runs=runs, precision=precision, guess=guess, **extra)
    from paper_2204_03575_amd import Solver
    p = dict(S.preset("square32", n=(24, 20)), precision=precision, **extra)
    co, ce = S.make_mesh(p)
    nv = co.shape[0]
    rl = run_list(runs)
    steps = 4
    b = Solver(co, ce, p, runs=rl)
    for r in range(runs):
        b.set_fields(*initial(nv, r, p), run=r)
    b.set_guess(guess, None, 21, 25)
    bst = b.step(steps)
    for r in range(runs):
        s = Solver(co, ce, dict(p, **rl[r]))
        s.set_fields(*initial(nv, r, p))
        s.set_guess(guess, None, 21, 25)
        sst = s.step(steps)
        for k in range(steps):
            got = bst[k] if runs == 1 else bst[k][r]
            for key in ("iters", "relres", "res0", "guess_used", "status"):
                assert got[key] == sst[k][key], (r, k, key, got[key], sst[k][key])
        fb, fs = b.get_fields(run=r), s.get_fields()
        for f in FIELDS:
            assert np.array_equal(fb[f], fs[f]), (r, f)
        print(f"run {r}: iterations {[x['iters'] for x in sst]}", flush=True)
        del s


def test_batched_run_matches_oracle():
    case("one run of a batch of 3 against the oracle")
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=(20, 18))
    co, ce = S.make_mesh(p)
    nv = co.shape[0]
    rl = [dict(chi_pn=0.8, evap_ds=0.0), dict(chi_pn=1.3, evap_ds=0.002, evap_steps=5),
          dict(chi_pn=1.0, evap_ds=0.0)]
    b = Solver(co, ce, p, runs=rl)
    for r in range(3):
        b.set_fields(*initial(nv, r, p), run=r)
    o = Oracle(co, ce, dict(p, **rl[1]))
    php, phn = initial(nv, 1, p)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros(nv), mu_n=np.zeros(nv))
    for k in range(3):
        bs = b.step(1)[0][1]
        st = o.step(st)
        got = b.get_fields(run=1)
        assert bs["iters"] == st["stats"]["iters"], (k, bs, st["stats"])
        for f in FIELDS:
            e = np.linalg.norm(got[f] - st[f]) / np.linalg.norm(st[f])
            assert e <= 1e-10, (k, f, e)


def test_nan_in_one_run_commits_no_run():
    case("a NaN in one run of four")
    from paper_2204_03575_amd import ChmError, Solver
    p = S.preset("square32", n=(12, 10))
    co, ce = S.make_mesh(p)
    nv = co.shape[0]
    b = Solver(co, ce, p, runs=run_list(4))
    for r in range(4):
        php, phn = initial(nv, r, p)
        if r == 2:
            php = php.copy()
            php[7] = np.nan
        b.set_fields(php, phn, run=r)
    before = [b.get_fields(run=r) for r in range(4)]
    with pytest.raises(ChmError) as e:
        b.step(1)
    assert "run 2" in str(e.value)
    for r in range(4):
        after = b.get_fields(run=r)
        for f in ("phi_p", "phi_n"):
            assert np.array_equal(after[f], before[r][f], equal_nan=True)


def test_batch_argument_checks():
    case("batch argument checks")
    from paper_2204_03575_amd import ChmError, Solver
    p = S.preset("square32", n=(6, 6))
    co, ce = S.make_mesh(p)
    with pytest.raises(ChmError):
        Solver(co, ce, p, runs=[{}] * 65)
    with pytest.raises(ChmError):
        Solver(co, ce, p, runs=[dict(evap_ds=-1.0)])
    b = Solver(co, ce, p, runs=[{}, {}])
    with pytest.raises(ChmError):
        b.set_fields(np.zeros(49), np.zeros(49), run=2)
    assert b.lib.chm_batch_size(b.h) == 2


def test_step_many_equals_separate_steps():
    """chm_step_many: solvers on their own streams, advanced concurrently by one
    host thread each, take the iterates they take when stepped one by one."""
    case("chm_step_many vs separate chm_step")
    import torch

    from paper_2204_03575_amd import Solver, step_many
    cfgs = [(dict(S.preset("square32", n=(24, 20))), 3), (dict(S.preset("square32", n=(30, 28)), precision="fp32"), 4),
            (dict(S.preset("square32", n=(16, 16))), 1)]

    def make(p, runs, stream=None):
        co, ce = S.make_mesh(p)
        nv = co.shape[0]
        g = Solver(co, ce, p, runs=run_list(runs) if runs > 1 else None,
                   stream=None if stream is None else stream.cuda_stream)
        for r in range(runs):
            g.set_fields(*initial(nv, r, p), run=r)
        return g

    streams = [torch.cuda.Stream() for _ in cfgs]
    many = [make(p, r, st) for (p, r), st in zip(cfgs, streams)]
    got = step_many(many, 3)
    torch.cuda.synchronize()
    for k, (p, runs) in enumerate(cfgs):
        one = make(p, runs)
        ref = one.step(3)
        keys = ("iters", "relres", "status")
        for i in range(3):
            a = [got[k][i]] if runs == 1 else got[k][i]
            b = [ref[i]] if runs == 1 else ref[i]
            assert [[x[q] for q in keys] for x in a] == [[x[q] for q in keys] for x in b], (k, i)
        for r in range(runs):
            fa, fb = many[k].get_fields(run=r), one.get_fields(run=r)
            for f in FIELDS:
                assert np.array_equal(fa[f], fb[f]), (k, r, f)


def test_step_many_failure_stays_in_its_solver():
    """A solver whose step fails (here: no convergence within 2 iterations) reports
    its error code and keeps its state; the other solvers of the same call
    advance as if stepped alone."""
    case("chm_step_many with one failing solver")
    import torch

    from paper_2204_03575_amd import ChmError, Solver, step_many
    from paper_2204_03575_amd.chm import CHM_ENOCONV
    good_p = dict(S.preset("square32", n=(24, 20)))
    bad_p = dict(S.preset("square32", n=(20, 18)), max_iters=2)

    def make(p, stream=None):
        co, ce = S.make_mesh(p)
        g = Solver(co, ce, p, stream=None if stream is None else stream.cuda_stream)
        g.set_fields(*initial(co.shape[0], 0, p))
        return g

    streams = [torch.cuda.Stream() for _ in range(2)]
    good, bad = make(good_p, streams[0]), make(bad_p, streams[1])
    before = bad.get_fields()
    with pytest.raises(ChmError) as err:
        step_many([good, bad], 1)
    assert err.value.code == CHM_ENOCONV
    torch.cuda.synchronize()
    after = bad.get_fields()
    for f in FIELDS:
        assert np.array_equal(before[f], after[f]), f
    ref = make(good_p)
    ref.step(1)
    fa, fb = good.get_fields(), ref.get_fields()
    for f in FIELDS:
        assert np.array_equal(fa[f], fb[f]), f

