"""GPU: a 3D box large enough that its second AMG level has more than 131,072
rows (192x192x96 cubes, 3.6 M vertices; level 1 has 135,084 rows with about 40
entries per row).  There the level's A takes the CSR layout (its rows are long)
while its prolongator, with 1 to 9 entries per row, takes SELL-64.  The fused
prolongation-and-smoothing launch reads P's CSR values in the preconditioner's
precision, which the FP32 copies hold only for a CSR-layout P, so the V-cycle
must take the two separate launches on such a level.  A regression test: one
step in FP64 and one with the FP32 preconditioner from the same state, which
must agree to the mixed-precision bound with at most a few more iterations."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu

FIELDS = ("phi_p", "phi_n", "mu_p", "mu_n")


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_03575_amd import library
    library()


def test_large_level_with_csr_a_and_sell_p():
    print("\n[case] box 192x192x96, FP64 and FP32 preconditioner, one step", flush=True)
    from paper_2204_03575_amd import Solver
    p = S.preset("box96", n=(192, 192, 96))
    co, ce = S.make_mesh(p)
    nv = co.shape[0]
    php, phn, _ = S.initial_fractions(nv, p["mean_p"], p["mean_n"])
    out = {}
    for prec in ("fp64", "fp32"):
        g = Solver(co, ce, dict(p, precision=prec))
        assert g.num_levels(1) >= 3
        lanes, _ = g.layout(1, 1)
        assert lanes > 0                       # level 1's A in the CSR layout
        g.set_fields(php, phn)
        st = g.step(1)[0]
        print(prec, st["iters"], st["relres"], flush=True)
        out[prec] = (st, g.get_fields())
        del g
    s64, f64 = out["fp64"]
    s32, f32 = out["fp32"]
    assert max(s64["relres"]) <= p["rtol"] and max(s32["relres"]) <= p["rtol"]
    assert all(b <= a + 3 for a, b in zip(s64["iters"], s32["iters"]))
    for f in FIELDS:
        e = np.linalg.norm(f32[f] - f64[f]) / np.linalg.norm(f64[f])
        assert e <= 1e-6, (f, e)
