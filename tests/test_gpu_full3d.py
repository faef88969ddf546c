"""GPU: the 3D workload at full size (96x96x48 hexahedra cut into Kuhn
tetrahedra on a 1 x 1 x 0.5 box, 461,041 vertices), one time step, against the
oracle.  The oracle's step takes about a minute on one core, so it runs once
for both tests.

  * FP64 path: the same FGMRES iteration counts and fields within 1e-10
    relative (the per-step parity bar);
  * FP32 preconditioner: FP64 true residual <= rtol (plus 1 %) by the oracle's
    operator, at most a few extra iterations, fields within 1e-6 of the FP64
    oracle (see the module docstring of the mixed-precision tests).
"""
import numpy as np
import pytest

import synthetic as S
from oracle import Oracle

pytestmark = pytest.mark.gpu

FIELDS = ("phi_p", "phi_n", "mu_p", "mu_n")


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)

def maxrel(a, b):
    """elementwise: max |a - b| over max |b| (a single bad vertex cannot hide
    in a 2-norm over many)"""
    mb = np.abs(b).max()
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0)


@pytest.fixture(scope="module")
def box():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_03575_amd import library
    library()
    print("\n[case] box96 oracle setup and one step", flush=True)
    p = S.preset("box96")
    co, ce = S.make_mesh(p)
    o = Oracle(co, ce, p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    st0 = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    st1 = o.step(dict(st0))
    print("oracle:", st1["stats"], flush=True)
    return p, co, ce, o, st0, st1


def run_gpu(p, co, ce, st0, precision):
    from paper_2204_03575_amd import Solver
    g = Solver(co, ce, dict(p, precision=precision))
    g.set_fields(st0["phi_p"], st0["phi_n"])
    gs = g.step(1)[0]
    return gs, g.get_fields()


def test_box96_fp64_one_step_matches_oracle(box):
    p, co, ce, o, st0, st1 = box
    print("[case] box96 fp64 one step", flush=True)
    gs, got = run_gpu(p, co, ce, st0, "fp64")
    print("gpu:", gs, flush=True)
    assert gs["iters"] == st1["stats"]["iters"]
    for f in FIELDS:
        e, em = relerr(got[f], st1[f]), maxrel(got[f], st1[f])
        print(f, e, em, flush=True)
        assert e <= 1e-10, (f, e)
        assert em <= 1e-10, (f, "elementwise", em)


def test_box96_fp32_preconditioner_one_step(box):
    p, co, ce, o, st0, st1 = box
    print("[case] box96 fp32 preconditioner one step", flush=True)
    gs, got = run_gpu(p, co, ce, st0, "fp32")
    b = o.rhs(st0["phi_p"], st0["phi_n"])
    for s, (ph, mu) in enumerate((("phi_p", "mu_p"), ("phi_n", "mu_n"))):
        x = np.concatenate([got[ph], got[mu]])
        res = np.linalg.norm(b[s] - o.apply_saddle(s, x)) / np.linalg.norm(b[s])
        print(f"species {s}: iters {gs['iters'][s]} (fp64 oracle {st1['stats']['iters'][s]}), "
              f"true relres {res:.3e}", flush=True)
        assert res <= 1.01 * p["rtol"]
        assert gs["iters"][s] <= st1["stats"]["iters"][s] + 3
    for f in FIELDS:
        e = relerr(got[f], st1[f])
        print(f"{f} difference from the FP64 oracle {e:.3e}", flush=True)
        assert e <= 1e-6, (f, e)
