"""GPU: the automatic inner CG steps (schur_pcg = -1).

The library measures the As-norm contraction of one V-cycle at setup (power
iteration from a seeded start) and picks 2, 4 or 6 CG steps per As solve;
the oracle does the same from its own hierarchy.  The contraction must agree
to rounding, the chosen count exactly, and the steps that follow must match
the oracle's (iteration counts equal, fields to 1e-10).  Cases on the
paper's film problem (Section 4) with a stiffness-dominated As (eps 10, large
tau) so that both counts occur.
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


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def maxrel(a, b):
    mb = np.abs(b).max()
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0)


@pytest.mark.parametrize("tau,k_expected", [(1e-2, 2), (1e-1, 4)])
def test_automatic_steps_match_oracle(tau, k_expected):
    print(f"\n[case] automatic inner CG steps, film 40x22, eps 10, tau {tau}", flush=True)
    from paper_2204_03575_amd import Solver
    from paper_2204_03575_amd import robustness as R
    p = R.case_params((40, 22), "fgmres", eps=10.0, tau=tau, coarse_max=16, schur_pcg=-1)
    co, ce = S.make_mesh(p)
    g, o = Solver(co, ce, p), Oracle(co, ce, p)
    kg, rg = g.schur_info()
    ko, ro = o.schur_info()
    print("gpu", kg, rg, "oracle", ko, ro, flush=True)
    assert kg == ko == k_expected
    assert rg == pytest.approx(ro, rel=1e-9)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    for k in range(2):
        gs = g.step(1)[0]
        st = o.step(st)
        assert gs["iters"] == st["stats"]["iters"], (k, gs, st["stats"])
        got = g.get_fields()
        for f in FIELDS:
            assert rel(got[f], st[f]) <= 1e-10, (k, f)
            assert maxrel(got[f], st[f]) <= 1e-10, (k, f, "elementwise")
        g.set_fields(st["phi_p"], st["phi_n"], st["mu_p"], st["mu_n"])


def test_fixed_steps_report_no_measurement():
    from paper_2204_03575_amd import Solver
    from paper_2204_03575_amd.chm import ChmError
    p = S.preset("square32", n=(10, 9))
    co, ce = S.make_mesh(p)
    assert Solver(co, ce, p).schur_info() == (p["schur_pcg"], 0.0)
    with pytest.raises(ChmError):
        Solver(co, ce, dict(p, schur_pcg=-1, krylov="minres"))
