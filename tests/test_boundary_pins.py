"""Pins of the oracle's boundary terms (eq. chternary:2 with the coefficients
of Section 4): the edge rule against closed forms, the boundary vector of
constant and linear states against integrals computed independently, the
substrate patterning, and the mass balance of a step, which with no flux
through the sides changes the integral of each phase by tau times the
boundary inflow."""
import numpy as np
import pytest
from scipy.integrate import quad

import synthetic as S
from oracle import Oracle
from oracle import oracle as O


def test_edge_rule_is_exact_to_degree_five():
    bary, w = O.quadrature(1)
    t = bary[:, 1]
    for k in range(6):
        assert np.isclose(np.dot(w, t ** k), 1.0 / (k + 1), rtol=1e-14)
    assert not np.isclose(np.dot(w, t ** 6), 1.0 / 7, rtol=1e-9)


def paper(n=(12, 6), **kw):
    p = S.preset("paper2d", n=n, **kw)
    co, ce = S.make_mesh(p)
    return p, co, ce, Oracle(co, ce, p)


def test_constant_state_inflow_and_substrate_totals():
    p, co, ce, o = paper()
    nv = co.shape[0]
    a, c = 0.3, 0.25
    gp, gn = o.boundary(np.full(nv, a), np.full(nv, c))
    Lx = 10.0
    top = np.isclose(co[:, 1], 2.5)
    bot = np.isclose(co[:, 1], 0.0)
    k = p["bc_k"]
    # the top takes k a (1 - a - c) per unit length, split to vertices by the hat functions
    assert np.isclose(gp[top].sum(), k * a * (1 - a - c) * Lx, rtol=1e-13)
    assert np.isclose(gn[top].sum(), k * c * (1 - a - c) * Lx, rtol=1e-13)
    hx = Lx / 12
    interior_top = top & (co[:, 0] > 1e-9) & (co[:, 0] < Lx - 1e-9)
    assert np.allclose(gp[interior_top], k * a * (1 - a - c) * hx, rtol=1e-13)
    # patterned substrate: p_p = 1 on half of the bottom (12 cells: two per sixth)
    assert np.isclose(gp[bot].sum(), 0.01 * Lx / 2, rtol=1e-13)
    assert np.isclose(gn[bot].sum(), 0.01 * Lx / 2, rtol=1e-13)
    # the first sixth prefers the polymer: its vertices carry no acceptor flux
    first = bot & (co[:, 0] < Lx / 6 - 1e-9)
    assert np.all(gn[first] == 0.0) and np.all(gp[first] > 0.0)
    # no flux through the sides or the interior
    assert np.all(gp[~(top | bot)] == 0.0) and np.all(gn[~(top | bot)] == 0.0)


def test_linear_state_matches_independent_integration():
    p, co, ce, o = paper(n=(6, 3), bc_pattern=0, bc_h=(0.3, 0.7))
    nv = co.shape[0]
    php = 0.2 + 0.02 * co[:, 0] + 0.01 * co[:, 1]
    phn = 0.3 - 0.015 * co[:, 0]
    gp, gn = o.boundary(php, phn)
    k = p["bc_k"]
    xs = np.unique(co[:, 0])
    for y, top in ((2.5, True), (0.0, False)):
        idx = [int(np.flatnonzero(np.isclose(co[:, 0], x) & np.isclose(co[:, 1], y))[0]) for x in xs]
        for j, v in enumerate(idx):
            ref_p = ref_n = 0.0
            for e in (j - 1, j):   # the two edges around vertex j
                if e < 0 or e + 1 >= len(xs):
                    continue
                x0, x1 = xs[e], xs[e + 1]
                a0, a1, b0, b1 = php[idx[e]], php[idx[e + 1]], phn[idx[e]], phn[idx[e + 1]]
                lam = (lambda x: (x1 - x) / (x1 - x0)) if e == j else (lambda x: (x - x0) / (x1 - x0))
                fp = lambda x: a0 + (a1 - a0) * (x - x0) / (x1 - x0)
                fn = lambda x: b0 + (b1 - b0) * (x - x0) / (x1 - x0)
                if top:
                    gpx = lambda x: k * fp(x) * (1 - fp(x) - fn(x))
                    gnx = lambda x: k * fn(x) * (1 - fp(x) - fn(x))
                else:
                    gpx = lambda x: 0.01 + 2 * 0.3 * fp(x)
                    gnx = lambda x: 0.01 + 2 * 0.7 * fn(x)
                ref_p += quad(lambda x: gpx(x) * lam(x), x0, x1, epsabs=1e-15)[0]
                ref_n += quad(lambda x: gnx(x) * lam(x), x0, x1, epsabs=1e-15)[0]
            assert np.isclose(gp[v], ref_p, rtol=1e-12, atol=1e-16), (y, j)
            assert np.isclose(gn[v], ref_n, rtol=1e-12, atol=1e-16), (y, j)


def test_3d_top_face_total():
    p = S.preset("paper2d", dim=3, n=(4, 2, 3), extent=(10.0, 2.5, 6.0), bc_pattern=0)
    co, ce = S.make_mesh(p)
    o = Oracle(co, ce, p)
    nv = co.shape[0]
    gp, gn = o.boundary(np.full(nv, 0.3), np.full(nv, 0.3))
    top = np.isclose(co[:, 1], 2.5)
    assert np.isclose(gp[top].sum(), p["bc_k"] * 0.3 * 0.4 * 60.0, rtol=1e-13)
    assert np.isclose(gp[~top].sum(), 0.01 * 60.0, rtol=1e-13)


def test_step_mass_balance_equals_boundary_inflow():
    p, co, ce, o = paper(n=(18, 6))
    nv = co.shape[0]
    php, phn, _ = S.initial_fractions(nv, p["mean_p"], p["mean_n"])
    M = o.scipy_matrix("M")
    st = dict(phi_p=php, phi_n=phn, mu_p=np.zeros(nv), mu_n=np.zeros(nv))
    gp, gn = o.boundary(php, phn)
    new = o.step(st)
    ones = np.ones(nv)
    for a, b, g in ((php, new["phi_p"], gp), (phn, new["phi_n"], gn)):
        change = ones @ (M @ (b - a))
        assert np.isclose(change, p["tau"] * g.sum(), rtol=1e-6), (change, p["tau"] * g.sum())
        assert change != 0.0


def test_boundary_off_is_zero_and_changes_nothing():
    p, co, ce, o = paper(n=(6, 3), boundary=0)
    nv = co.shape[0]
    gp, gn = o.boundary(np.full(nv, 0.3), np.full(nv, 0.3))
    assert np.all(gp == 0.0) and np.all(gn == 0.0)
