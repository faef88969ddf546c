"""Host logic of the robustness sweeps: the cases and parameters follow the
paper's Section 4 experiments (film 10 x 2.5 or box 10 x 2.5 x 10, meshes
given in points, MINRES to 1e-7 with AMG solves to 1e-4, polynomial
potential, boundary terms)."""
from paper_2204_03575_amd import robustness as R


def test_case_params_follow_the_paper():
    p = R.case_params((800, 400), "paper")
    assert p["n"] == (799, 399) and p["extent"] == (10.0, 2.5) and p["dim"] == 2
    assert p["krylov"] == "minres" and p["schur_pcg"] == 0
    assert p["amg_tol"] == 1e-4 and p["rtol"] == 1e-7
    assert p["potential"] == "polynomial" and p["boundary"] == 1 and p["bc_pattern"] == 1
    assert p["eps"] == 1e-3 and p["tau"] == 1e-4
    assert p["mean_p"] == p["mean_n"] == 0.35
    q = R.case_params((30, 15, 30), "fgmres", eps=0.1)
    assert q["dim"] == 3 and q["n"] == (29, 14, 29) and q["extent"] == (10.0, 2.5, 10.0)
    assert q["krylov"] == "fgmres" and q["eps"] == 0.1


def test_sweeps_cover_the_papers_figures():
    assert [c[0] for c in R.cases("mesh2d", 10 ** 9)] == R.MESHES_2D
    assert [c[0] for c in R.cases("mesh3d", 10 ** 9)] == R.MESHES_3D
    assert [c[1]["eps"] for c in R.cases("eps", 10 ** 9)] == R.EPS
    assert [c[1]["tau"] for c in R.cases("tau", 10 ** 9)] == R.TAU
    assert [c[0] for c in R.cases("mesh2d", 400_000)] == R.MESHES_2D[:4]
    for fig, figs in R.PAPER_FIGURES.items():
        if fig == "mesh2d_after1000":   # Fig. 2: the 2D meshes up to 1600 x 800
            assert sorted(figs) == sorted(R.MESHES_2D[:5])
            continue
        assert len(figs) == len(R.cases(fig, 10 ** 9))
