"""GPU: the SELL-64 matrices of the solve with 16-bit column offsets.

With wide_index = 0 (the default) a square SELL matrix whose entries all lie
within 32767 of the diagonal stores each column as an offset from its row
(2 B per entry in the kernels' traffic instead of 4).  The kernels then add
the same products in the same order, so the results are bitwise those of
wide_index = 1: checked over two time steps in FP64 and FP32 on a mesh large
enough for the fine levels to take the SELL layout (400 x 400, 160,801
vertices).  A mesh whose vertex numbering is shuffled has offsets beyond
16 bits; the library keeps 32-bit columns for it, and a step matches the
oracle as every other step does.  Strips whose largest offset is exactly
32767 and 32768 pin the limit."""
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


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)

def maxrel(a, b):
    """elementwise: max |a - b| over max |b| (a single bad vertex cannot hide
    in a 2-norm over many)"""
    mb = np.abs(b).max()
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_offsets_give_the_wide_columns_results_bitwise(prec):
    case("16-bit offsets vs 32-bit columns, 400x400, 2 steps", prec=prec)
    from paper_2204_03575_amd import Solver
    p = S.preset("square512", n=(400, 400), precision=prec)
    co, ce = S.make_mesh(p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    out = {}
    for wide in (0, 1):
        g = Solver(co, ce, dict(p, wide_index=wide))
        want = 4 if wide else 2
        # the fine level of both hierarchies and M's pattern use SELL-64
        assert g.layout(-1) == (0, want)
        assert g.layout(0, 0) == (0, want)
        assert g.layout(1, 0) == (0, want)
        # coarse levels keep the CSR layout (32-bit columns)
        assert g.layout(1, 1)[0] > 0 and g.layout(1, 1)[1] == 4
        g.set_fields(php, phn)
        st = g.step(2)
        out[wide] = ([x["iters"] for x in st], [x["relres"] for x in st], g.get_fields())
        print(wide, out[wide][0], flush=True)
        del g
    assert out[0][0] == out[1][0]
    assert out[0][1] == out[1][1]
    for f in FIELDS:
        assert np.array_equal(out[0][2][f], out[1][2][f]), f


def shuffled_mesh(p, seed):
    """The mesh of p with its vertices renumbered by a seeded permutation."""
    co, ce = S.make_mesh(p)
    perm = np.random.default_rng(seed).permutation(co.shape[0])   # old -> new
    co2 = np.empty_like(co)
    co2[perm] = co
    return co2, perm[ce].astype(ce.dtype)


def test_offsets_that_do_not_fit_keep_wide_columns():
    case("shuffled 200x200 mesh: offsets beyond 16 bits")
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=(200, 200))
    co, ce = S.make_mesh(p)
    assert Solver(co, ce, p).layout(-1) == (0, 2)      # natural numbering: offsets <= 202
    co, ce = shuffled_mesh(p, 5)
    g, o = Solver(co, ce, p), Oracle(co, ce, p)
    assert g.layout(-1) == (0, 4)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    gs = g.step(1)[0]
    st = o.step(st)
    assert gs["iters"] == st["stats"]["iters"], (gs, st["stats"])
    got = g.get_fields()
    for f in FIELDS:
        assert relerr(got[f], st[f]) <= 1e-10, f
        assert maxrel(got[f], st[f]) <= 1e-10, (f, "elementwise")


@pytest.mark.parametrize("nx,fits", [(32765, True), (32766, False)])
def test_offsets_at_the_16_bit_limit(nx, fits):
    """A strip of nx x 1 unit squares: its largest column offset is nx + 2,
    32767 (the largest that fits) or 32768 (the first that does not)."""
    case("strip at the 16-bit offset limit", nx=nx)
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=(nx, 1), extent=(float(nx), 1.0))
    co, ce = S.make_mesh(p)
    assert np.abs(ce[:, :, None] - ce[:, None, :]).max() == (32767 if fits else 32768)
    g, o = Solver(co, ce, p), Oracle(co, ce, p)
    assert g.layout(-1) == (0, 2 if fits else 4)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    gs = g.step(1)[0]
    st = o.step(st)
    assert gs["iters"] == st["stats"]["iters"], (gs, st["stats"])
    got = g.get_fields()
    for f in FIELDS:
        assert relerr(got[f], st[f]) <= 1e-10, f
        assert maxrel(got[f], st[f]) <= 1e-10, (f, "elementwise")


def test_wide_index_argument_check():
    case("wide_index must be 0 or 1; layout of a level that does not exist")
    from paper_2204_03575_amd import ChmError, Solver
    p = S.preset("square32", n=(4, 4), wide_index=2)
    co, ce = S.make_mesh(p)
    with pytest.raises(ChmError):
        Solver(co, ce, p)
    g = Solver(co, ce, dict(p, wide_index=0))
    for hier, lev in ((2, 0), (1, g.num_levels(1)), (0, -1)):
        with pytest.raises(ChmError):
            g.layout(hier, lev)
