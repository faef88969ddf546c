"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Every stage is compared on the same seeded inputs: assembled matrices, the AMG
hierarchy (integer structure bit-exact, values to rounding), one V-cycle, the
CG-accelerated As solve, the saddle-point operator, Algorithm 1, the
right-hand side, one time step and short trajectories.  Tolerances:
  * integer data (patterns, aggregates, iteration counts): exact;
  * matrices and hierarchy values: 1e-13 relative to the largest entry (a few
    ulps of sums of tens of products);
  * linear operators and preconditioner: 1e-12 relative (the V-cycle chains
    tens of SpMVs with different summation order and FMA contraction);
  * fields after a time step: 1e-10 relative per field, in the 2-norm.
"""
import math

import numpy as np
import pytest

import synthetic as S
from oracle import Oracle, OracleError

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


def make(n=(32, 32), dim=2, extent=None, **kw):
    from paper_2204_03575_amd import Solver
    p = S.preset("square32", n=n, dim=dim, **kw)
    if extent is not None:
        p["extent"] = extent
    elif dim == 3:
        p["extent"] = (1.0, 1.0, 1.0)
    co, ce = S.make_mesh(p)
    return p, co, ce, Solver(co, ce, p), Oracle(co, ce, p)


def relerr(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)

def maxrel(a, b):
    """elementwise: max |a - b| over max |b| (a single bad vertex cannot hide
    in a 2-norm over many)"""
    mb = np.abs(b).max()
    return np.abs(a - b).max() / (mb if mb > 0 else 1.0)


MESHES = [
    dict(n=(32, 32)),                                   # the 32x32 square
    dict(n=(37, 23), extent=(2.0, 0.75)),               # ragged slices, anisotropic cells
    dict(n=(6, 5, 4), dim=3),                           # Kuhn tetrahedra
    dict(n=(1, 1)),                                     # 4 vertices: a single coarse level
    dict(n=(2, 1)),
]


@pytest.mark.parametrize("mesh", MESHES, ids=lambda m: "x".join(map(str, m["n"])))
def test_matrices_match(mesh):
    case("matrices", **mesh)
    p, co, ce, g, o = make(**mesh)
    for which, ow in (("M", "M"), ("K", "K"), ("As", "As0")):
        grp, gci, gv = g.matrix(which)
        orp, oci, ov = o.matrix(ow)
        assert np.array_equal(grp, orp) and np.array_equal(gci, oci), which
        scale = np.abs(ov).max()
        assert np.abs(gv - ov).max() <= 1e-13 * scale, (which, np.abs(gv - ov).max() / scale)


@pytest.mark.parametrize("mesh", MESHES[:3], ids=lambda m: "x".join(map(str, m["n"])))
@pytest.mark.parametrize("hier", [0, 1])
def test_hierarchy_matches(mesh, hier):
    case("hierarchy", hier=hier, **mesh)
    p, co, ce, g, o = make(coarse_max=20, **mesh)
    assert g.num_levels(hier) == o.num_levels(hier)
    for lev in range(o.num_levels(hier)):
        gl, ol = g.level(hier, lev), o.level(hier, lev)
        assert gl["n"] == ol["n"]
        assert abs(gl["rho"] - ol["rho"]) <= 1e-13 * ol["rho"]
        assert np.array_equal(gl["A"][0], ol["A"][0]) and np.array_equal(gl["A"][1], ol["A"][1])
        sc = np.abs(ol["A"][2]).max()
        assert np.abs(gl["A"][2] - ol["A"][2]).max() <= 1e-12 * sc, (lev, "A")
        if "agg" in ol:
            assert np.array_equal(gl["agg"], ol["agg"]), (lev, "aggregates")
            assert np.array_equal(gl["P"][0], ol["P"][0]) and np.array_equal(gl["P"][1], ol["P"][1])
            sp_ = np.abs(ol["P"][2]).max()
            assert np.abs(gl["P"][2] - ol["P"][2]).max() <= 1e-13 * sp_, (lev, "P")


@pytest.mark.parametrize("mesh", MESHES, ids=lambda m: "x".join(map(str, m["n"])))
def test_vcycle_and_schur_solve_match(mesh):
    case("vcycle", **mesh)
    p, co, ce, g, o = make(coarse_max=20, **mesh)
    rng = np.random.default_rng(11)
    b0, b1 = rng.standard_normal(o.nv), rng.standard_normal(o.nv)
    for hier in (0, 1):
        x0, x1 = g.vcycle(hier, b0, b1)
        assert relerr(x0, o.vcycle(hier, b0)) <= 1e-12, hier
        assert relerr(x1, o.vcycle(hier, b1)) <= 1e-12, hier
    x0, x1 = g.schur_solve(b0, b1)
    assert relerr(x0, o.schur_solve(0, b0)) <= 1e-12
    assert relerr(x1, o.schur_solve(1, b1)) <= 1e-12


@pytest.mark.parametrize("mesh", MESHES[:3], ids=lambda m: "x".join(map(str, m["n"])))
def test_operator_preconditioner_rhs_match(mesh):
    case("operators", **mesh)
    p, co, ce, g, o = make(**mesh)
    rng = np.random.default_rng(5)
    v0, v1 = rng.standard_normal(2 * o.nv), rng.standard_normal(2 * o.nv)
    y0, y1 = g.apply_saddle(v0, v1)
    assert relerr(y0, o.apply_saddle(0, v0)) <= 1e-13
    assert relerr(y1, o.apply_saddle(1, v1)) <= 1e-13
    w0, w1 = g.apply_prec(v0, v1)
    assert relerr(w0, o.apply_prec(0, v0)) <= 1e-12
    assert relerr(w1, o.apply_prec(1, v1)) <= 1e-12
    php, phn, _ = S.initial_fractions(o.nv, 0.1, 0.1)
    g.set_fields(php, phn)
    b0, b1 = g.rhs()
    r0, r1 = o.rhs(php, phn)
    assert relerr(b0, r0) <= 1e-13 and relerr(b1, r1) <= 1e-13


@pytest.mark.parametrize("mesh", MESHES[:3], ids=lambda m: "x".join(map(str, m["n"])))
def test_rhs_over_the_range_of_the_logarithm(mesh):
    """f' of Flory-Huggins (N_p = N_n = 20) for states whose quadrature values span
    the logarithm's arguments.  State A: phi_p and phi_n log-uniform in
    [1e-14, 0.45] (below the 1e-12 floor they are clamped), so phi_s >= 0.1.
    State B: phi_p in [0.55, 0.98] or [1.02, 1.5] and phi_n in [1e-14, 0.01], so
    phi_s is at least 0.01 or negative (clamped) at every vertex.  phi_s =
    1 - phi_p - phi_n loses the digits of the sum where it is small, so states
    with phi_s just above the floor at a vertex are left out: there the
    right-hand side is as sensitive to the rounding of phi_p + phi_n as to the
    logarithm."""
    case("rhs over the logarithm's range", **mesh)
    p, co, ce, g, o = make(**mesh)
    nv = co.shape[0]
    rng = np.random.default_rng(11)
    u = rng.uniform(size=(4, nv))
    side = rng.integers(0, 2, nv)
    states = [
        (10.0 ** (-14 + 13.65 * u[0]), 10.0 ** (-14 + 13.65 * u[1])),
        (np.where(side == 0, 0.55 + 0.43 * u[2], 1.02 + 0.48 * u[2]), 10.0 ** (-14 + 12 * u[3])),
    ]
    for php, phn in states:
        g.set_fields(php, phn)
        b0, b1 = g.rhs()
        r0, r1 = o.rhs(php, phn)
        assert relerr(b0, r0) <= 1e-13 and relerr(b1, r1) <= 1e-13
        assert maxrel(b0, r0) <= 1e-12 and maxrel(b1, r1) <= 1e-12


def run_pair(p, co, ce, g, o, steps, php=None, phn=None):
    if php is None:
        php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    for k in range(steps):
        gs = g.step(1)[0]
        st = o.step(st)
        got = g.get_fields()
        assert gs["iters"] == st["stats"]["iters"], (k, gs, st["stats"])
        for f in FIELDS:
            e = relerr(got[f], st[f])
            assert e <= 1e-10, (k, f, e)
            e = maxrel(got[f], st[f])
            assert e <= 1e-10, (k, f, "elementwise", e)
        assert np.allclose(got["phi_s"], 1 - got["phi_p"] - got["phi_n"], atol=1e-15)
        # hand the oracle's state back so each step starts from identical inputs
        g.set_fields(st["phi_p"], st["phi_n"], st["mu_p"], st["mu_n"])
    return st


def test_square32_five_step_trajectory():
    case("square32 trajectory (5 steps, rtol 1e-8)")
    p = S.preset("square32")
    co, ce = S.make_mesh(p)
    from paper_2204_03575_amd import Solver
    run_pair(p, co, ce, Solver(co, ce, p), Oracle(co, ce, p), p["steps"])


def test_square32_free_running_trajectory():
    """Five steps with no state hand-back: errors must stay at rounding level."""
    case("square32 free-running")
    p = S.preset("square32")
    co, ce = S.make_mesh(p)
    from paper_2204_03575_amd import Solver
    g, o = Solver(co, ce, p), Oracle(co, ce, p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    g.set_fields(php, phn)
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros_like(php), mu_n=np.zeros_like(php))
    stats = g.step(p["steps"])
    for _ in range(p["steps"]):
        st = o.step(st)
    got = g.get_fields()
    for f in FIELDS:
        assert relerr(got[f], st[f]) <= 1e-10, f
        assert maxrel(got[f], st[f]) <= 1e-10, (f, "elementwise")
    assert all(s["relres"][0] <= p["rtol"] and s["relres"][1] <= p["rtol"] for s in stats)


@pytest.mark.parametrize("variant", [
    dict(potential="polynomial", mean=(0.35, 0.35)),
    dict(smoother="jacobi", cheb_degree=3, cheb_degree_mass=2),
    dict(schur_pcg=0, amg_cycles=2),
    dict(restart=5),                                  # forces restarts
    dict(tau=1e-6, eps=1e-2, mobility=2.0),
    dict(potential="none"),
    dict(mass_solver="chebyshev", cheb_degree_mass=5),
    dict(mass_solver="chebyshev", cheb_degree_mass=4, smoother="jacobi", cheb_degree=3),
    dict(mass_solver="chebyshev", cheb_degree_mass=5, krylov="minres", schur_pcg=0,
         amg_cycles=2),
    dict(cheb_degree=1, cheb_degree_mass=1),          # one smoothing step: no fused first steps
    dict(cheb_degree=2, cheb_degree_mass=2, mass_solver="chebyshev"),   # the fused steps only
    dict(cheb_degree=4, cheb_degree_coarse=1, coarse_max=12),     # coarse levels of degree 1
    dict(cheb_degree=6, cheb_degree_coarse=3, coarse_max=12, cheb_ratio=5.0,
         mass_solver="chebyshev", cheb_degree_mass=5, schur_pcg=2),
    dict(smoother="jacobi", cheb_degree=3, cheb_degree_coarse=1, coarse_max=12),
    dict(ortho="cgs2"),                               # both Gram-Schmidt passes in one iteration
    dict(ortho="cgs2", restart=5),
    dict(restart=2),                                  # a cycle of two: one delayed pass
    dict(ortho="cgs2", cheb_degree=6, cheb_degree_coarse=3, coarse_max=12, cheb_ratio=5.0,
         mass_solver="chebyshev", cheb_degree_mass=5, schur_pcg=2),
], ids=["poly", "jacobi", "stationary", "restart5", "tau-eps-mob", "nopot", "mass-cheb",
        "mass-jacobi", "mass-cheb-minres", "degree1", "degree2", "coarse1", "coarse3",
        "jacobi-coarse1", "cgs2", "cgs2-restart5", "restart2", "cgs2-coarse3"])
def test_step_variants(variant):
    v = dict(variant)
    mean = v.pop("mean", (0.1, 0.1))
    case("step variant", **v)
    p, co, ce, g, o = make(n=(20, 17), **v)
    php, phn, _ = S.initial_fractions(o.nv, *mean)
    run_pair(p, co, ce, g, o, 2, php, phn)


@pytest.mark.parametrize("mass", ["amg", "chebyshev"])
def test_3d_box_steps(mass):
    case("3d box 6x6x4, 2 steps", mass_solver=mass)
    p, co, ce, g, o = make(n=(6, 6, 4), dim=3, extent=(1.0, 1.0, 0.5), mass_solver=mass,
                           cheb_degree_mass=5 if mass == "chebyshev" else 2)
    run_pair(p, co, ce, g, o, 2)


@pytest.mark.parametrize("ortho", ["cgs2", "dcgs2"])
def test_3d_box_coarse_degree_steps(ortho):
    """the 3D box workload's setting: coarse levels smoothed with one step"""
    case("3d box 10x9x6, coarse degree 1, 2 steps", ortho=ortho)
    p, co, ce, g, o = make(n=(10, 9, 6), dim=3, extent=(1.0, 1.0, 0.5), mass_solver="chebyshev",
                           cheb_degree_mass=5, schur_pcg=1, cheb_degree_coarse=1, coarse_max=30,
                           ortho=ortho)
    assert g.num_levels(1) >= 3
    run_pair(p, co, ce, g, o, 2)


@pytest.mark.parametrize("mass", ["chebyshev"])
def test_preconditioner_with_chebyshev_mass_matches(mass):
    case("Algorithm 1 with the Chebyshev mass solve")
    p, co, ce, g, o = make(n=(23, 19), mass_solver=mass, cheb_degree_mass=5)
    rng = np.random.default_rng(12)
    v0, v1 = rng.standard_normal(2 * o.nv), rng.standard_normal(2 * o.nv)
    w0, w1 = g.apply_prec(v0, v1)
    assert relerr(w0, o.apply_prec(0, v0)) <= 1e-12
    assert relerr(w1, o.apply_prec(1, v1)) <= 1e-12


def test_evaporation_steps():
    case("evaporation 0.01 per step for 2 steps, then none")
    p, co, ce, g, o = make(n=(16, 16), evap_ds=0.01, steps=2)
    run_pair(p, co, ce, g, o, 3)


def test_nonconvergence_keeps_state():
    case("max_iters = 2")
    from paper_2204_03575_amd.chm import CHM_ENOCONV, ChmError
    p, co, ce, g, o = make(n=(10, 10), max_iters=2)
    php, phn, _ = S.initial_fractions(o.nv, 0.1, 0.1)
    g.set_fields(php, phn)
    with pytest.raises(ChmError) as ei:
        g.step(1)
    assert ei.value.code == CHM_ENOCONV
    got = g.get_fields()
    assert np.array_equal(got["phi_p"], php) and np.array_equal(got["phi_n"], phn)
    with pytest.raises(OracleError):
        o.step(dict(phi_p=php, phi_n=phn, mu_p=0 * php, mu_n=0 * php))


def test_nan_is_reported():
    case("NaN in phi_p")
    from paper_2204_03575_amd.chm import CHM_ENAN, ChmError
    p, co, ce, g, o = make(n=(6, 6))
    php, phn, _ = S.initial_fractions(o.nv, 0.1, 0.1)
    php[3] = np.nan
    g.set_fields(php, phn)
    with pytest.raises(ChmError) as ei:
        g.step(1)
    assert ei.value.code == CHM_ENAN


@pytest.mark.parametrize("ortho", ["cgs2", "dcgs2"])
def test_graph_replays_match_eager_bitwise(ortho):
    """Each FGMRES iteration captured as a HIP graph and replayed over several
    steps (with eager right-hand sides and host synchronisation in between)
    gives the eager kernels' results bit for bit, step by step."""
    case("graphs vs eager, 28x26, 4 steps", ortho=ortho)
    runs = []
    for graphs in (0, 1):
        p, co, ce, g, o = make(n=(28, 26), use_graphs=graphs, ortho=ortho)
        php, phn, _ = S.initial_fractions(o.nv, 0.1, 0.1)
        g.set_fields(php, phn)
        per_step = []
        for k in range(4):
            st = g.step(1)[0]
            per_step.append((st["iters"], g.get_fields()))
        runs.append(per_step)
    for k in range(4):
        (it0, f0), (it1, f1) = runs[0][k], runs[1][k]
        assert it0 == it1, k
        for f in FIELDS:
            assert np.array_equal(f0[f], f1[f]), (k, f)


def test_runs_are_bitwise_deterministic():
    case("determinism 24x24, 2 steps, two solvers")
    outs = []
    for rep in range(2):
        p, co, ce, g, o = make(n=(24, 24))
        php, phn, _ = S.initial_fractions(o.nv, 0.1, 0.1)
        g.set_fields(php, phn)
        for k in range(2):
            st = g.step(1)[0]
            print(f"solver {rep} step {k}: {st}", flush=True)
        outs.append(g.get_fields())
        del g
    for f in FIELDS:
        assert np.array_equal(outs[0][f], outs[1][f]), f


def test_square512_one_step_full_size():
    """The 512x512 workload of the benchmark, one step, against the oracle."""
    case("square512 one step (full size)")
    p = S.preset("square512")
    co, ce = S.make_mesh(p)
    from paper_2204_03575_amd import Solver
    g = Solver(co, ce, p)
    o = Oracle(co, ce, p)
    php, phn, _ = S.initial_fractions(co.shape[0], p["mean_p"], p["mean_n"])
    run_pair(p, co, ce, g, o, 1, php, phn)
