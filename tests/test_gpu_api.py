"""GPU: the field calls of the C-ABI with host pointers (on_device = 0)
against the device-pointer path the binding uses: the same state in, the same
fields out, bit for bit, with phi_s = 1 - phi_p - phi_n (Section 2)."""
import ctypes as C

import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu_available():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2204_03575_amd import library
    library()


def ptr(a):
    return a.ctypes.data_as(C.c_void_p)


@pytest.mark.parametrize("runs", [1, 3])
def test_host_pointer_fields_round_trip(runs):
    print(f"\n[case] host-pointer fields, runs={runs}", flush=True)
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=(23, 17))
    co, ce = S.make_mesh(p)
    nv = co.shape[0]
    g = Solver(co, ce, p, runs=[{}] * runs if runs > 1 else None)
    rng = np.random.default_rng(4)
    for r in range(runs):
        php, phn = rng.uniform(0.05, 0.4, nv), rng.uniform(0.05, 0.4, nv)
        mup, mun = rng.standard_normal(nv), rng.standard_normal(nv)
        rc = g.lib.chm_set_fields_run(g.h, r, ptr(php), ptr(phn), ptr(mup), ptr(mun), 0)
        assert rc == 0
        out = {k: np.full(nv, np.nan) for k in ("phi_p", "phi_n", "phi_s", "mu_p", "mu_n")}
        rc = g.lib.chm_get_fields_run(g.h, r, *(ptr(out[k]) for k in
                                                ("phi_p", "phi_n", "phi_s", "mu_p", "mu_n")), 0)
        assert rc == 0
        dev = g.get_fields(run=r)
        for k, ref in (("phi_p", php), ("phi_n", phn), ("mu_p", mup), ("mu_n", mun)):
            assert np.array_equal(out[k], ref), k
            assert np.array_equal(dev[k], ref), k
        assert np.array_equal(out["phi_s"], 1.0 - php - phn)
        assert np.array_equal(dev["phi_s"], out["phi_s"])
    # mu omitted: set to zero
    php, phn = rng.uniform(0.05, 0.4, nv), rng.uniform(0.05, 0.4, nv)
    assert g.lib.chm_set_fields_run(g.h, 0, ptr(php), ptr(phn), None, None, 0) == 0
    f = g.get_fields()
    assert not np.any(f["mu_p"]) and not np.any(f["mu_n"])
    assert np.array_equal(f["phi_p"], php)
