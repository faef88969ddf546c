"""GPU: the volume fractions leaving [0, 1], the paper's eps = 1e-4 failure.

The paper records that its film run diverges at eps = 1e-4 (Section 4,
Fig. 4).  On the 100 x 50 film the state leaves [0, 1] within 40 steps; every
step reports how many vertices are outside, and that count must equal the
oracle's at every step (the fields agree to 1e-10, so a vertex would have to
sit within that of 0 or 1 to flip).  With range_check = 1 the first such step
fails with CHM_EDOMAIN and leaves the state as it was.
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


def film(**kw):
    from paper_2204_03575_amd import robustness as R
    p = R.case_params((100, 50), "fgmres", eps=1e-4, schur_pcg=2, **kw)
    co, ce = S.make_mesh(p)
    return p, co, ce


def test_outside_count_matches_oracle_until_divergence():
    print("\n[case] film 100x50, eps 1e-4, out-of-range counts vs oracle", flush=True)
    from paper_2204_03575_amd import Solver
    p, co, ce = film()
    g, o = Solver(co, ce, p), Oracle(co, ce, p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    first = None
    for k in range(40):
        gs = g.step(1)[0]
        st = o.step(st)
        assert gs["iters"] == st["stats"]["iters"], (k, gs["iters"], st["stats"]["iters"])
        assert gs["outside"] == st["stats"]["outside"], (k, gs["outside"], st["stats"]["outside"])
        g.set_fields(st["phi_p"], st["phi_n"], st["mu_p"], st["mu_n"])
        if gs["outside"]:
            first = k
            break
    print("first step outside [0, 1]:", first, flush=True)
    assert first is not None


def test_range_check_stops_and_keeps_the_state():
    print("\n[case] film 100x50, eps 1e-4, range_check = 1", flush=True)
    from paper_2204_03575_amd import Solver
    from paper_2204_03575_amd.chm import CHM_EDOMAIN, ChmError
    p, co, ce = film()
    free_run = Solver(co, ce, p)
    checked = Solver(co, ce, dict(p, range_check=1))
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    free_run.set_fields(php, phn)
    checked.set_fields(php, phn)
    for k in range(40):
        before = checked.get_fields()
        a = free_run.step(1)[0]
        if a["outside"]:
            with pytest.raises(ChmError) as e:
                checked.step(1)
            assert e.value.code == CHM_EDOMAIN
            assert e.value.stats[0]["outside"] == a["outside"]
            after = checked.get_fields()
            for f in FIELDS:
                assert np.array_equal(after[f], before[f]), f
            return
        b = checked.step(1)[0]
        assert b["iters"] == a["iters"] and b["outside"] == 0
    pytest.fail("the state did not leave [0, 1] within 40 steps")
