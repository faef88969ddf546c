"""GPU: value tables.  Where a fine-level SELL matrix has few distinct values
(uniform meshes), the kernels read a 2-byte index per entry into the table of
those values instead of the value itself.  The table holds the same values,
so every product, and with it every step, is bitwise the same as reading the
values directly (values_direct = 1); the tables must also be in use on the
uniform meshes of the workloads."""
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


def case(name, **kw):
    print(f"\n[case] {name} {kw}", flush=True)


def run(p, steps, runs=None):
    from paper_2204_03575_amd import Solver
    co, ce = S.make_mesh(p)
    g = Solver(co, ce, p, runs=runs)
    nv = co.shape[0]
    for r in range(len(runs) if runs else 1):
        php, phn, _ = S.initial_fractions(nv, p["mean_p"], p["mean_n"], seed=S.BASE_SEED + r)
        g.set_fields(php, phn, run=r)
    st = g.step(steps)
    return g, st


SMALL = [
    ("square32", dict(n=(40, 36))),
    ("square32", dict(n=(40, 36), precision="fp32")),
    ("square32", dict(dim=3, n=(12, 10, 8), extent=(1.0, 1.0, 0.8))),
    ("square32", dict(dim=3, n=(12, 10, 8), extent=(1.0, 1.0, 0.8), precision="fp32",
                      mass_solver="chebyshev", cheb_degree_mass=3)),
    ("square32", dict(n=(40, 36), ortho="cgs2", mass_solver="chebyshev", cheb_degree_mass=5)),
]


@pytest.mark.parametrize("name,kw", SMALL, ids=["2d", "2d-fp32", "3d", "3d-fp32-masscheb",
                                                 "2d-cgs2-masscheb"])
def test_tables_give_the_same_bits(name, kw):
    case("value tables vs direct values", **kw)
    # meshes this small keep their hierarchy levels in the CSR layout, so the
    # tables in use are those of the solver's M and K (the product with M in
    # Algorithm 1 and in the right-hand side); the next test covers a SELL
    # fine level
    p = S.preset(name, **kw)
    g1, s1 = run(p, 3)
    g0, s0 = run(dict(p, values_direct=1), 3)
    assert g0.value_table(-1, 0) == 0 and g0.value_table(-1, 1) == 0
    assert g1.value_table(-1, 0) > 0 and g1.value_table(-1, 1) > 0
    for k in range(3):
        assert s1[k]["iters"] == s0[k]["iters"], k
        assert s1[k]["relres"] == s0[k]["relres"], k
    f1, f0 = g1.get_fields(), g0.get_fields()
    for f in FIELDS:
        assert np.array_equal(f1[f], f0[f]), f


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tables_on_sell_fine_level_same_bits(precision):
    """A mesh large enough for the SELL-64 fine level (131,072 rows and up),
    so the V-cycle smoother and residual read their values through the table."""
    case("SELL fine level with value tables", precision=precision)
    p = S.preset("square32", n=(400, 360), precision=precision, mass_solver="chebyshev",
                 cheb_degree_mass=5, cheb_degree=6, cheb_ratio=5.0, schur_pcg=2,
                 cheb_degree_coarse=4, coarse_max=2048)
    g1, s1 = run(p, 2)
    g0, s0 = run(dict(p, values_direct=1), 2)
    assert g1.layout(1, 0)[0] == 0          # SELL-64 on the fine As level
    assert g1.value_table(1, 0) > 0 and g1.value_table(0, 0) > 0
    assert g0.value_table(1, 0) == 0 and g0.value_table(0, 0) == 0
    for k in range(2):
        assert s1[k]["iters"] == s0[k]["iters"], k
        assert s1[k]["relres"] == s0[k]["relres"], k
    f1, f0 = g1.get_fields(), g0.get_fields()
    for f in FIELDS:
        assert np.array_equal(f1[f], f0[f]), f


def test_tables_in_a_batch_same_bits():
    case("batch of 3 runs, value tables vs direct values")
    rng = np.random.default_rng(7)
    runs = [dict(chi_pn=float(rng.uniform(0.6, 1.4))) for _ in range(3)]
    p = S.preset("square32", n=(36, 30), runs_per_lane=2)
    g1, s1 = run(p, 2, runs)
    g0, s0 = run(dict(p, values_direct=1), 2, runs)
    for r in range(3):
        f1, f0 = g1.get_fields(run=r), g0.get_fields(run=r)
        for f in FIELDS:
            assert np.array_equal(f1[f], f0[f]), (r, f)


def layered_box(nx, ny, nz):
    """Kuhn box of [0,1/32]^2 x [0,0.5] whose nz cell layers all differ in
    thickness (nearly cubic cells on 8 x 8 x 64): every layer adds its own
    element values, so the assembled M and K hold between 1,025 and 2,048
    distinct values (about 1,300 each) and their tables take the largest
    staging path (up to 8 entries per thread of a 256-thread block)."""
    co, ce = S.mesh_box_3d(nx, ny, nz, 1.0 / 32, 1.0 / 32, 1.0)
    t = 1.0 + 0.125 * np.arange(nz)
    zs = np.concatenate([[0.0], np.cumsum(t)]) / np.sum(t) * 0.5
    k = np.rint(co[:, 2] * nz).astype(int)
    co = co.copy()
    co[:, 2] = zs[k]
    return co, ce


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tables_of_more_than_1024_values_same_bits(precision):
    case("tables of 1,025-2,048 values vs direct values", precision=precision)
    from paper_2204_03575_amd import Solver
    co, ce = layered_box(8, 8, 64)
    p = S.preset("square32", dim=3, n=(8, 8, 64), extent=(1.0 / 32, 1.0 / 32, 0.5),
                 precision=precision)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"], seed=S.BASE_SEED)
    out = []
    for direct in (0, 1):
        g = Solver(co, ce, dict(p, values_direct=direct))
        g.set_fields(php, phn)
        out.append((g, g.step(2)))
    (g1, s1), (g0, s0) = out
    m_m, m_k = g1.value_table(-1, 0), g1.value_table(-1, 1)
    print(f"[tables] M {m_m} K {m_k}", flush=True)
    assert 1024 < max(m_m, m_k) <= 2048 and min(m_m, m_k) > 0
    assert g0.value_table(-1, 0) == 0 and g0.value_table(-1, 1) == 0
    for k in range(2):
        assert s1[k]["iters"] == s0[k]["iters"], k
        assert s1[k]["relres"] == s0[k]["relres"], k
    f1, f0 = g1.get_fields(), g0.get_fields()
    for f in FIELDS:
        assert np.array_equal(f1[f], f0[f]), f
