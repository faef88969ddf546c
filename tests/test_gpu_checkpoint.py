"""GPU: exact checkpoint and resume, and per-run history in a batch.

A solver stopped after k steps is checkpointed with chm_get_fields_run and
chm_get_history; a fresh solver restored with chm_set_fields_run and
chm_set_history must then take the uninterrupted solver's iterates bit for
bit: the same fields, iteration counts, residuals and choices of start, in
every start mode (previous state, linear extrapolation, the network's guess)
and with the solvent removal switching off inside the resumed part (the step
counter is part of the checkpoint).  In a batch, setting one run's fields
starts a new history for that run only: the other runs go on exactly as they
would alone.
"""
import os

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu

FIELDS = ("phi_p", "phi_n", "mu_p", "mu_n")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2204_03575_amd", "weights", "guess256.npy")


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_03575_amd import library
    library()


def case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def same_stats(a, b):
    for x, y in zip(a, b):
        assert x["iters"] == y["iters"] and x["relres"] == y["relres"], (x, y)
        assert x["guess_used"] == y["guess_used"], (x, y)


def same_fields(a, b):
    for f in FIELDS:
        assert np.array_equal(a[f], b[f]), f


@pytest.mark.parametrize("mode,precision", [("previous", "fp64"), ("linear", "fp64"),
                                            ("learned", "fp64"), ("linear", "fp32"),
                                            ("learned", "fp32")])
def test_resume_is_bitwise(mode, precision):
    case("checkpoint/resume", mode=mode, precision=precision)
    from paper_2204_03575_amd import Net, Solver
    nx, ny = 24, 20
    p = dict(S.preset("square32", n=(nx, ny)), precision=precision, evap_ds=3e-3, evap_steps=5)
    co, ce = S.make_mesh(p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    H, W = ny + 1, nx + 1
    net = None
    if mode == "learned":
        net = Net(H * W)
        net.set_params(np.load(WEIGHTS))
    a = Solver(co, ce, p)
    a.set_fields(php, phn)
    a.set_guess(mode, net, H, W)
    a.step(3)
    ckpt_f = a.get_fields()
    ckpt_h = a.get_history()
    assert ckpt_h["steps"] == 3 and ckpt_h["valid"] == 2
    rest_a = a.step(4)   # steps 4..7: the removal stops after step 5
    b = Solver(co, ce, p)
    b.set_fields(ckpt_f["phi_p"], ckpt_f["phi_n"], ckpt_f["mu_p"], ckpt_f["mu_n"])
    b.set_history(ckpt_h)
    b.set_guess(mode, net, H, W)
    rest_b = b.step(4)
    same_stats(rest_a, rest_b)
    same_fields(a.get_fields(), b.get_fields())
    if mode != "previous":
        assert any(s["guess_used"] != (0, 0) for s in rest_a)   # the history is used
    # without the history the resumed solver departs (its first step starts
    # from the previous state and the removal counter restarts)
    c = Solver(co, ce, p)
    c.set_fields(ckpt_f["phi_p"], ckpt_f["phi_n"], ckpt_f["mu_p"], ckpt_f["mu_n"])
    c.set_guess(mode, net, H, W)
    c.step(4)
    fc = c.get_fields()
    assert any(not np.array_equal(fc[f], a.get_fields()[f]) for f in FIELDS)


def test_history_roundtrip_and_checks():
    case("history get/set round trip and argument checks")
    from paper_2204_03575_amd import Solver
    from paper_2204_03575_amd.chm import ChmError
    p = S.preset("square32", n=(8, 6))
    co, ce = S.make_mesh(p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g = Solver(co, ce, p)
    h0 = g.get_history()
    assert h0["valid"] == 0 and h0["steps"] == 0
    g.set_fields(php, phn)
    h1 = g.get_history()
    assert h1["valid"] == 1 and h1["y2"] is None
    st = g.get_state().cpu().numpy()
    assert np.array_equal(h1["y1"].cpu().numpy(), st)
    g.step(2)
    h2 = g.get_history()
    assert h2["valid"] == 2 and h2["steps"] == 2
    assert np.array_equal(h2["y1"].cpu().numpy(), g.get_state(solution=True).cpu().numpy())
    g.set_history(dict(h2, steps=7))
    assert g.get_history()["steps"] == 7
    with pytest.raises(ChmError):
        g.set_history(dict(h2, valid=3))
    with pytest.raises(ChmError):
        g.set_history(dict(h2, y2=None))
    with pytest.raises(ChmError):
        g.set_history(dict(h2, steps=-1))
    with pytest.raises(ChmError):
        g.get_history(run=1)


def test_setting_one_run_keeps_the_others_history():
    case("batch: set_fields_run resets only that run")
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=(16, 12))
    co, ce = S.make_mesh(p)
    nv = co.shape[0]
    runs = [dict(chi_pn=0.8, evap_ds=2e-3, evap_steps=4), dict(chi_pn=1.2, evap_ds=4e-3, evap_steps=6),
            dict(chi_pn=1.0, evap_ds=1e-3, evap_steps=2)]
    init = [S.initial_fractions(nv, p["mean_p"], p["mean_n"], seed=S.BASE_SEED + 200 + r)[:2]
            for r in range(3)]
    new = S.initial_fractions(nv, 0.12, 0.09, seed=S.BASE_SEED + 300)[:2]
    bat = Solver(co, ce, p, runs=runs)
    bat.set_guess("linear")
    for r in range(3):
        bat.set_fields(*init[r], run=r)
    bat.step(3)
    bat.set_fields(*new, run=1)
    tail = bat.step(3)
    for r in range(3):
        one = Solver(co, ce, dict(p, **runs[r]))
        one.set_guess("linear")
        one.set_fields(*init[r])
        one.step(3)
        if r == 1:
            one.set_fields(*new)
        t1 = one.step(3)
        same_stats([s[r] for s in tail], t1)
        same_fields(bat.get_fields(run=r), one.get_fields())
