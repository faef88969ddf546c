"""Pins of the oracle's discrete Ginzburg-Landau energy (eq. ginzburglandau,
Section 2, without the substrate term): E(phi) = sum over the species of the
integral of the bulk density f(phi_p,h, phi_n,h) plus (eps_i / 2) times the
integral of |grad phi_i,h|^2.

Each test compares the oracle with a value fixed independently of it: a hand
value of the polynomial density for a constant state, the closed-form
Dirichlet integral of a smooth field with its O(h^2) convergence, and exact
integrals over single simplices by SciPy's adaptive quadrature.  A factor
eps in place of eps/2, a dropped quadrature weight or cell volume, or a
missing species fails at least one of them.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import synthetic as S
from oracle import Oracle


def _oracle(co, ce, **kw):
    p = S.preset("square32", n=(1, 1), **kw)
    return Oracle(co, ce, p)


def test_constant_state_gives_area_times_density():
    """K 1 = 0, so a constant state has no gradient energy and E = |Omega| f.
    Polynomial density at phi_p = 0.2, phi_n = 0.3 (phi_s = 0.5), by hand:
    3.5 * 0.04 * 0.09 + 0.1 * 0.25 = 0.0376."""
    co, ce = S.mesh_rect_2d(7, 5, 2.0, 0.75)
    o = _oracle(co, ce, potential="polynomial")
    one = np.ones(o.nv)
    E = o.energy(0.2 * one, 0.3 * one)
    assert E == pytest.approx(2.0 * 0.75 * 0.0376, rel=1e-13)
    # 3D: a 1 x 1 x 0.5 box, Kuhn tetrahedra
    co, ce = S.mesh_box_3d(3, 2, 2, 1.0, 1.0, 0.5)
    o = _oracle(co, ce, potential="polynomial")
    one = np.ones(o.nv)
    assert o.energy(0.2 * one, 0.3 * one) == pytest.approx(0.5 * 0.0376, rel=1e-13)
    # no bulk density: zero for any constant state
    co, ce = S.mesh_rect_2d(4, 4)
    o = _oracle(co, ce, potential="none")
    assert abs(o.energy(0.4 * np.ones(o.nv), 0.1 * np.ones(o.nv))) < 1e-16


def test_dirichlet_integral_of_a_cosine_mode():
    """f = 0: E = (eps/2) int |grad phi|^2.  For phi = cos(pi x) cos(pi y) on
    the unit square the integral is pi^2 / 2, so E -> eps pi^2 / 4 for the
    polymer field alone; the nodal interpolant's energy converges at O(h^2).
    The acceptor field 0.5 phi adds a quarter of that with its own eps."""
    eps_p, eps_n = 2e-3, 5e-3
    exact = 0.5 * eps_p * math.pi ** 2 / 2 + 0.5 * eps_n * 0.25 * math.pi ** 2 / 2
    errs = []
    for n in (8, 16, 32):
        co, ce = S.mesh_rect_2d(n, n)
        o = _oracle(co, ce, potential="none", eps=(eps_p, eps_n))
        u = np.cos(math.pi * co[:, 0]) * np.cos(math.pi * co[:, 1])
        errs.append(abs(o.energy(u, 0.5 * u) - exact) / exact)
    assert errs[-1] < 5e-3
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    assert all(1.8 < r < 2.2 for r in rates), (errs, rates)


def _triangle_integral(fun, xv):
    """integral over the triangle with vertices xv (3 x 2) of fun(x, y)"""
    a, b, c = xv
    J = np.column_stack([b - a, c - a])
    det = abs(np.linalg.det(J))

    def g(t, s):   # reference coordinates (s, t), 0 <= t <= 1 - s
        x, y = a + J @ np.array([s, t])
        return fun(x, y)
    val, _ = integrate.dblquad(g, 0.0, 1.0, 0.0, lambda s: 1.0 - s, epsabs=1e-15, epsrel=1e-13)
    return det * val


def test_linear_fields_on_one_triangle_integrate_exactly():
    """Linear fields make the polynomial density a quartic, which the degree-5
    rule integrates exactly; the gradient term is |grad phi|^2 |T|."""
    xv = np.array([[0.1, 0.2], [0.9, 0.35], [0.3, 0.8]])
    ce = np.array([[0, 1, 2]], dtype=np.int32)
    eps = 3e-3
    o = _oracle(xv, ce, potential="polynomial", eps=eps)
    php = np.array([0.15, 0.3, 0.22])
    phn = np.array([0.4, 0.12, 0.25])
    # the linear interpolants in closed form: phi(x) = c0 + g . x
    A = np.column_stack([np.ones(3), xv])
    cp, cn = np.linalg.solve(A, php), np.linalg.solve(A, phn)

    def dens(x, y):
        p = cp[0] + cp[1] * x + cp[2] * y
        q = cn[0] + cn[1] * x + cn[2] * y
        return 3.5 * p * p * q * q + 0.1 * (1.0 - p - q) ** 2
    area = 0.5 * abs(np.linalg.det(np.column_stack([xv[1] - xv[0], xv[2] - xv[0]])))
    grad = 0.5 * eps * (cp[1] ** 2 + cp[2] ** 2 + cn[1] ** 2 + cn[2] ** 2) * area
    exact = _triangle_integral(dens, xv) + grad
    assert o.energy(php, phn) == pytest.approx(exact, rel=1e-12)


def test_linear_fields_on_one_tetrahedron_integrate_exactly():
    xv = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.2, 0.9, 0.1], [0.1, 0.3, 0.7]])
    ce = np.array([[0, 1, 2, 3]], dtype=np.int32)
    eps = 4e-3
    o = _oracle(xv, ce, potential="polynomial", eps=eps)
    php = np.array([0.15, 0.3, 0.22, 0.05])
    phn = np.array([0.4, 0.12, 0.25, 0.33])
    A = np.column_stack([np.ones(4), xv])
    cp, cn = np.linalg.solve(A, php), np.linalg.solve(A, phn)
    J = (xv[1:] - xv[0]).T
    det = abs(np.linalg.det(J))

    def g(u, t, s):   # reference coordinates (s, t, u) of the unit tetrahedron
        x = xv[0] + J @ np.array([s, t, u])
        p = cp[0] + cp[1:] @ x
        q = cn[0] + cn[1:] @ x
        return 3.5 * p * p * q * q + 0.1 * (1.0 - p - q) ** 2
    val, _ = integrate.tplquad(g, 0.0, 1.0, 0.0, lambda s: 1.0 - s, 0.0,
                               lambda s, t: 1.0 - s - t, epsabs=1e-15, epsrel=1e-12)
    grad = 0.5 * eps * (cp[1:] @ cp[1:] + cn[1:] @ cn[1:]) * det / 6.0
    assert o.energy(php, phn) == pytest.approx(det * val + grad, rel=1e-11)
