"""Pins of the oracle's Chebyshev mass solve (the alternative to AMG for the
mass block of Algorithm 1 that Section 3 names, after Wathen and Rees): from
x = 0, d Chebyshev steps on D^-1 M over [rho/ratio, rho] give
x_d = (I - R_d(D^-1 M)) M^-1 b with the scaled Chebyshev residual polynomial
R_d(l) = T_d((theta - l)/delta) / T_d(theta/delta); d damped-Jacobi sweeps
give x_d = (I - (I - w D^-1 M)^d) M^-1 b.  Both closed forms are evaluated
here by a dense eigendecomposition, independently of the oracle's
recurrence."""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

import synthetic as S
from oracle import Oracle


def setup(dim=2, n=(7, 6), **kw):
    extent = (1.0, 1.0) if dim == 2 else (1.0, 1.0, 1.0)
    p = S.preset("square32", dim=dim, n=n, extent=extent, mass_solver="chebyshev", **kw)
    co, ce = S.make_mesh(p)
    return p, Oracle(co, ce, p)


def closed_form(M, b, poly):
    """(I - poly(D^-1 M)) M^-1 b, poly applied through D^-1/2 M D^-1/2."""
    d = np.diag(M)
    Sm = M / np.sqrt(np.outer(d, d))
    lam, Q = np.linalg.eigh(Sm)
    R = (Q * poly(lam)) @ Q.T
    Rd = (R * np.sqrt(d)[None, :]) / np.sqrt(d)[:, None]   # D^-1/2 R D^1/2
    y = np.linalg.solve(M, b)
    return y - Rd @ y


@pytest.mark.parametrize("dim,n", [(2, (7, 6)), (3, (3, 3, 2))], ids=["2d", "3d"])
@pytest.mark.parametrize("deg", [1, 2, 5])
def test_chebyshev_mass_solve_is_the_scaled_chebyshev_polynomial(dim, n, deg):
    p, o = setup(dim, n, cheb_degree_mass=deg, cheb_ratio_mass=4.0)
    M = o.scipy_matrix("M").toarray()
    rho = np.max(np.abs(M).sum(axis=1) / np.diag(M))       # Gershgorin bound of D^-1 M
    lmax, lmin = rho, rho / 4.0
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    Td = lambda t: C.chebval(t, [0] * deg + [1])
    poly = lambda lam: Td((theta - lam) / delta) / Td(theta / delta)
    rng = np.random.default_rng(deg + 10 * dim)
    b = rng.standard_normal(o.nv)
    w = o.apply_prec(0, np.concatenate([b, np.zeros(o.nv)]))[: o.nv]
    ref = closed_form(M, b, poly)
    assert np.linalg.norm(w - ref) <= 1e-12 * np.linalg.norm(ref)
    # on [lmin, lmax] the residual polynomial is at most 1/T_d(theta/delta)
    lam = np.linalg.eigvalsh(M / np.sqrt(np.outer(np.diag(M), np.diag(M))))
    assert lam.max() <= lmax + 1e-12


@pytest.mark.parametrize("deg", [1, 3])
def test_jacobi_mass_solve_is_the_damped_jacobi_polynomial(deg):
    p, o = setup(smoother="jacobi", cheb_degree_mass=deg)
    M = o.scipy_matrix("M").toarray()
    rho = np.max(np.abs(M).sum(axis=1) / np.diag(M))
    w_ = 4.0 / (3.0 * rho)
    b = np.random.default_rng(3).standard_normal(o.nv)
    w = o.apply_prec(1, np.concatenate([b, np.zeros(o.nv)]))[: o.nv]
    ref = closed_form(M, b, lambda lam: (1.0 - w_ * lam) ** deg)
    assert np.linalg.norm(w - ref) <= 1e-12 * np.linalg.norm(ref)


def test_chebyshev_mass_solve_converges_with_degree():
    errs = []
    for deg in (2, 4, 8):
        p, o = setup(n=(9, 9), cheb_degree_mass=deg)
        M = o.scipy_matrix("M").toarray()
        b = np.random.default_rng(0).standard_normal(o.nv)
        w = o.apply_prec(0, np.concatenate([b, np.zeros(o.nv)]))[: o.nv]
        y = np.linalg.solve(M, b)
        errs.append(np.linalg.norm(w - y) / np.linalg.norm(y))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-3


def test_unknown_mass_solver_is_rejected():
    import ctypes
    import oracle as O
    p = S.preset("square32", n=(4, 4))
    co, ce = S.make_mesh(p)
    co = np.ascontiguousarray(co, dtype=np.float64)
    ce = np.ascontiguousarray(ce, dtype=np.int32)
    lib = O.load_library()
    for bad in (2, -1):
        prm = O.oracle_params(p)
        prm.mass_solver = bad
        h = ctypes.c_void_p()
        rc = lib.orc_create(2, co.shape[0], co.ctypes.data_as(ctypes.c_void_p), ce.shape[0],
                            ce.ctypes.data_as(ctypes.c_void_p), ctypes.byref(prm),
                            ctypes.byref(h))
        assert rc != 0 and not h.value
