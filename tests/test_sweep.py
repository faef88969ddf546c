"""The sweep's run draw and grouping (host logic): seeded, the stated
distributions, every run in exactly one group of its mesh size."""
from paper_2204_03575_amd import sweep as W


def test_draw_is_seeded_and_in_range():
    a, b = W.draw_runs(64), W.draw_runs(64)
    assert a == b
    for r in a:
        assert r["n"] in W.SIZES
        assert 0.6 <= r["chi_pn"] <= 1.4
        assert 1e-3 <= r["evap_ds"] <= 5e-3
        assert abs(r["evap_steps"] * r["evap_ds"] - 0.5) <= r["evap_ds"]
    assert len({r["seed"] for r in a}) == 64
    assert len({r["n"] for r in a}) == len(W.SIZES)


def test_groups_partition_by_size():
    runs = W.draw_runs(64)
    g = W.groups(runs)
    assert sum(len(v) for v in g.values()) == 64
    for n, rs in g.items():
        assert all(r["n"] == n for r in rs)
    assert list(g) == sorted(g)
