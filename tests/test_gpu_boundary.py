"""GPU: the boundary terms of eq. chternary:2 (evaporation inflow on the
top, patterned substrate at the bottom) against the oracle: the boundary
vector of a state (1e-13, a few ulps of sums of a few facet contributions),
time steps on the paper's 10 x 2.5 film in 2D and a 3D box (1e-10 per field,
identical iteration counts), and a batch with boundary terms against single
runs (bitwise)."""
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


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


CASES = [dict(n=(12, 6)), dict(n=(13, 5), bc_pattern=0, bc_h=(0.2, 0.4)),
         dict(dim=3, n=(4, 2, 3), extent=(10.0, 2.5, 6.0))]


@pytest.mark.parametrize("kw", CASES, ids=["2d-pattern", "2d-ragged-h", "3d"])
def test_boundary_vector_matches_oracle(kw):
    case("boundary vector", **kw)
    from paper_2204_03575_amd import Solver
    p = S.preset("paper2d", **kw)
    co, ce = S.make_mesh(p)
    g = Solver(co, ce, p)
    o = Oracle(co, ce, p)
    rng = np.random.default_rng(3)
    php = 0.35 + 0.05 * rng.standard_normal(co.shape[0])
    phn = 0.3 + 0.05 * rng.standard_normal(co.shape[0])
    g.set_fields(php, phn)
    gp, gn = g.boundary()
    op, on = o.boundary(php, phn)
    assert rel(gp, op) <= 1e-13 and rel(gn, on) <= 1e-13
    assert np.array_equal(gp != 0, op != 0)
    b0, b1 = o.rhs(php, phn)
    assert np.abs(op).sum() > 0


@pytest.mark.parametrize("kw", [dict(n=(24, 12)), dict(dim=3, n=(6, 3, 4), extent=(10.0, 2.5, 6.0))],
                         ids=["2d-24x12", "3d-6x3x4"])
def test_steps_with_boundary_match_oracle(kw):
    case("steps with boundary terms", **kw)
    from paper_2204_03575_amd import Solver
    p = S.preset("paper2d", **kw)
    co, ce = S.make_mesh(p)
    g = Solver(co, ce, p)
    o = Oracle(co, ce, p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    for k in range(3):
        gs = g.step(1)[0]
        st = o.step(st)
        got = g.get_fields()
        print(f"step {k}: {gs['iters']} oracle {st['stats']['iters']}", flush=True)
        assert gs["iters"] == st["stats"]["iters"]
        for f in FIELDS:
            assert rel(got[f], st[f]) <= 1e-10, (k, f, rel(got[f], st[f]))


def test_batch_with_boundary_equals_single_runs():
    case("batch of 3 with boundary terms")
    from paper_2204_03575_amd import Solver
    p = S.preset("paper2d", n=(18, 6))
    co, ce = S.make_mesh(p)
    nv = co.shape[0]
    rl = [dict(chi_pn=0.7), dict(chi_pn=1.1), dict(chi_pn=1.3)]
    inits = [S.initial_fractions(nv, 0.35, 0.35, seed=S.BASE_SEED + 50 + r)[:2] for r in range(3)]
    b = Solver(co, ce, p, runs=rl)
    for r in range(3):
        b.set_fields(*inits[r], run=r)
    bst = b.step(2)
    for r in range(3):
        s = Solver(co, ce, dict(p, **rl[r]))
        s.set_fields(*inits[r])
        sst = s.step(2)
        for k in range(2):
            assert bst[k][r]["iters"] == sst[k]["iters"]
        fb, fs = b.get_fields(run=r), s.get_fields()
        for f in FIELDS:
            assert np.array_equal(fb[f], fs[f]), (r, f)
