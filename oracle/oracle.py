"""ctypes wrapper of the C oracle (TEST INFRASTRUCTURE ONLY).

``build_oracle()`` compiles ``chm_oracle.c`` with gcc into ``liboracle.so``
next to this file.  ``Oracle`` owns one ``orc_solver_t``: mesh and parameters
in, FP64 fields per time step out, plus inspection calls (matrices, AMG
levels, one V-cycle, Algorithm 1, the saddle-point operator, one FGMRES solve)
for the parity tests.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "chm_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

POTENTIALS = {"flory_huggins": 0, "polynomial": 1, "none": 2}
SMOOTHERS = {"chebyshev": 0, "jacobi": 1}
CODES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -4: "ENOCONV", -5: "ENAN", -6: "EDOMAIN"}


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {CODES.get(code, code)}")
        self.code = code


class orc_params_t(C.Structure):
    _fields_ = [
        ("tau", C.c_double), ("eps", C.c_double * 2), ("mobility", C.c_double * 2),
        ("potential", C.c_int32), ("Np", C.c_double), ("Nn", C.c_double), ("Ns", C.c_double),
        ("chi_pn", C.c_double), ("chi_ps", C.c_double), ("chi_ns", C.c_double),
        ("log_floor", C.c_double), ("evap_ds", C.c_double), ("evap_steps", C.c_int32),
        ("rtol", C.c_double), ("restart", C.c_int32), ("max_iters", C.c_int32),
        ("amg_cycles", C.c_int32), ("schur_pcg", C.c_int32), ("smoother", C.c_int32),
        ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double),
        ("cheb_degree_mass", C.c_int32), ("cheb_ratio_mass", C.c_double),
        ("coarse_max", C.c_int32), ("max_levels", C.c_int32),
        ("boundary", C.c_int32), ("bc_k", C.c_double), ("bc_g", C.c_double * 2),
        ("bc_h", C.c_double * 2), ("bc_pattern", C.c_int32), ("krylov", C.c_int32),
        ("amg_tol", C.c_double), ("mass_solver", C.c_int32), ("cheb_degree_coarse", C.c_int32),
        ("range_check", C.c_int32),
    ]


class orc_stats_t(C.Structure):
    _fields_ = [("iters", C.c_int32 * 2), ("relres", C.c_double * 2),
                ("status", C.c_int32), ("clamped", C.c_int32), ("outside", C.c_int32)]


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2; OpenMP only splits row loops
    over host threads, see orc_threads)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
                        "-fopenmp", "-Wall", "-Wno-unused-function", "-o", tmp, SRC, "-lm"],
                       check=True)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def load_library():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build_oracle()
        lib = C.CDLL(LIB)
        P = C.POINTER
        d, i32, i64 = C.c_double, C.c_int32, C.c_int64
        vp = C.c_void_p
        lib.orc_element_matrices.argtypes = [C.c_int, vp, vp, vp, P(d)]
        lib.orc_quadrature.argtypes = [C.c_int, P(C.c_int), vp, vp]
        lib.orc_potential.argtypes = [P(orc_params_t), d, d, P(d), P(d), P(d)]
        lib.orc_create.argtypes = [C.c_int, i64, vp, i64, vp, P(orc_params_t), P(vp)]
        lib.orc_destroy.argtypes = [vp]
        lib.orc_destroy.restype = None
        lib.orc_nnz.argtypes = [vp]
        lib.orc_nnz.restype = i64
        lib.orc_get_matrix.argtypes = [vp, C.c_int, vp, vp, vp]
        lib.orc_num_levels.argtypes = [vp, C.c_int]
        lib.orc_level_info.argtypes = [vp, C.c_int, C.c_int, P(i64), P(i64), P(i64), P(d)]
        lib.orc_level_get.argtypes = [vp, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp]
        lib.orc_amg_solve.argtypes = [vp, C.c_int, vp, vp]
        lib.orc_vcycle.argtypes = [vp, C.c_int, vp, vp]
        lib.orc_schur_solve.argtypes = [vp, C.c_int, vp, vp]
        lib.orc_smooth.argtypes = [vp, C.c_int, C.c_int, vp, vp]
        lib.orc_apply_saddle.argtypes = [vp, C.c_int, vp, vp]
        lib.orc_apply_prec.argtypes = [vp, C.c_int, vp, vp]
        lib.orc_rhs.argtypes = [vp, vp, vp, vp, vp]
        lib.orc_boundary.argtypes = [vp, vp, vp, vp, vp]
        lib.orc_minres.argtypes = [vp, C.c_int, vp, vp, P(i32), P(d)]
        lib.orc_fgmres.argtypes = [vp, C.c_int, vp, vp, P(i32), P(d)]
        lib.orc_step.argtypes = [vp, vp, vp, vp, vp, P(orc_stats_t)]
        lib.orc_energy.argtypes = [vp, vp, vp]
        lib.orc_energy.restype = d
        lib.orc_schur_info.argtypes = [vp, P(i32), P(d)]
        lib.orc_threads.argtypes = [C.c_int]
        lib.orc_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def oracle_params(p: dict) -> orc_params_t:
    """Fill the oracle's parameter struct from a preset dict."""
    s = orc_params_t()
    s.tau = p["tau"]
    eps = p["eps"] if isinstance(p["eps"], (list, tuple)) else (p["eps"], p["eps"])
    mob = p["mobility"] if isinstance(p["mobility"], (list, tuple)) else (p["mobility"],) * 2
    s.eps[0], s.eps[1] = eps
    s.mobility[0], s.mobility[1] = mob
    s.potential = POTENTIALS[p["potential"]]
    for k in ("Np", "Nn", "Ns", "chi_pn", "chi_ps", "chi_ns", "log_floor", "rtol"):
        setattr(s, k, p[k])
    s.evap_ds = p.get("evap_ds", 0.0)
    if s.evap_ds > 0.0:
        s.evap_steps = int(p.get("evap_steps", p.get("steps", 0)))
    else:
        s.evap_steps = 0
    for k in ("restart", "max_iters", "amg_cycles", "schur_pcg", "cheb_degree",
              "cheb_degree_mass", "coarse_max", "max_levels"):
        setattr(s, k, int(p[k]))
    s.smoother = SMOOTHERS[p["smoother"]]
    s.cheb_ratio = p["cheb_ratio"]
    s.cheb_ratio_mass = p["cheb_ratio_mass"]
    s.boundary = int(p.get("boundary", 0))
    s.bc_k = float(p.get("bc_k", 0.0))
    g = p.get("bc_g", (0.0, 0.0))
    h = p.get("bc_h", (0.0, 0.0))
    s.bc_g[0], s.bc_g[1] = g
    s.bc_h[0], s.bc_h[1] = h
    s.bc_pattern = int(p.get("bc_pattern", 0))
    s.krylov = {"fgmres": 0, "minres": 1}[p.get("krylov", "fgmres")]
    s.amg_tol = float(p.get("amg_tol", 0.0))
    s.mass_solver = {"amg": 0, "chebyshev": 1}[p.get("mass_solver", "amg")]
    s.cheb_degree_coarse = int(p.get("cheb_degree_coarse", 0))
    s.range_check = int(p.get("range_check", 0))
    return s


def element_matrices(xv: np.ndarray):
    lib = load_library()
    xv = np.ascontiguousarray(xv, dtype=np.float64)
    dim = xv.shape[1]
    nl = dim + 1
    MT = np.zeros((nl, nl))
    KT = np.zeros((nl, nl))
    vol = C.c_double()
    rc = lib.orc_element_matrices(dim, _ptr(xv), _ptr(MT), _ptr(KT), C.byref(vol))
    if rc:
        raise OracleError(rc, "orc_element_matrices")
    return MT, KT, vol.value


def quadrature(dim: int):
    """The rule on the reference simplex of dimension dim (1: edges)."""
    lib = load_library()
    bary = np.zeros((64, dim + 1))
    w = np.zeros(64)
    n = C.c_int()
    rc = lib.orc_quadrature(dim, C.byref(n), _ptr(bary), _ptr(w))
    if rc:
        raise OracleError(rc, "orc_quadrature")
    return bary[: n.value].copy(), w[: n.value].copy()


def potential(p: dict, php: float, phn: float):
    lib = load_library()
    prm = oracle_params(p)
    f, fp, fn = C.c_double(), C.c_double(), C.c_double()
    rc = lib.orc_potential(C.byref(prm), php, phn, C.byref(f), C.byref(fp), C.byref(fn))
    if rc:
        raise OracleError(rc, "orc_potential")
    return f.value, fp.value, fn.value


def threads(n: int = 0) -> int:
    """Host threads of the oracle's row loops (n > 0 sets them); the results
    are bitwise the same for any count."""
    return load_library().orc_threads(int(n))


class Oracle:
    """One oracle solver instance."""

    def __init__(self, coords: np.ndarray, cells: np.ndarray, params: dict):
        self.lib = load_library()
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        self.cells = np.ascontiguousarray(cells, dtype=np.int32)
        self.dim = self.coords.shape[1]
        self.nv = self.coords.shape[0]
        self.params = dict(params)
        self._prm = oracle_params(params)
        h = C.c_void_p()
        rc = self.lib.orc_create(self.dim, self.nv, _ptr(self.coords), self.cells.shape[0],
                                 _ptr(self.cells), C.byref(self._prm), C.byref(h))
        if rc:
            raise OracleError(rc, "orc_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # --- matrices and hierarchy -------------------------------------
    def matrix(self, which: str):
        """CSR (rowptr, col, val) of 'M', 'K', 'As0' or 'As1'."""
        idx = {"M": 0, "K": 1, "As0": 2, "As1": 3}[which]
        nnz = self.lib.orc_nnz(self.h)
        rp = np.zeros(self.nv + 1, np.int32)
        ci = np.zeros(nnz, np.int32)
        v = np.zeros(nnz)
        rc = self.lib.orc_get_matrix(self.h, idx, _ptr(rp), _ptr(ci), _ptr(v))
        if rc:
            raise OracleError(rc, "orc_get_matrix")
        return rp, ci, v

    def scipy_matrix(self, which: str):
        import scipy.sparse as sp
        rp, ci, v = self.matrix(which)
        return sp.csr_matrix((v, ci, rp), shape=(self.nv, self.nv))

    def num_levels(self, hier: int) -> int:
        return self.lib.orc_num_levels(self.h, hier)

    def level(self, hier: int, lev: int) -> dict:
        n, na, npp = C.c_int64(), C.c_int64(), C.c_int64()
        rho = C.c_double()
        rc = self.lib.orc_level_info(self.h, hier, lev, C.byref(n), C.byref(na), C.byref(npp),
                                     C.byref(rho))
        if rc:
            raise OracleError(rc, "orc_level_info")
        n, na, npp = n.value, na.value, npp.value
        Arp = np.zeros(n + 1, np.int32)
        Aci = np.zeros(na, np.int32)
        Av = np.zeros(na)
        agg = np.full(n, -1, np.int32)
        Prp = np.zeros(n + 1, np.int32)
        Pci = np.zeros(npp, np.int32)
        Pv = np.zeros(npp)
        rc = self.lib.orc_level_get(self.h, hier, lev, _ptr(Arp), _ptr(Aci), _ptr(Av), _ptr(agg),
                                    _ptr(Prp), _ptr(Pci), _ptr(Pv))
        if rc:
            raise OracleError(rc, "orc_level_get")
        out = dict(n=n, rho=rho.value, A=(Arp, Aci, Av))
        if npp:
            out.update(agg=agg, P=(Prp, Pci, Pv), nc=int(agg.max()) + 1)
        return out

    def amg_solve(self, hier: int, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        rc = self.lib.orc_amg_solve(self.h, hier, _ptr(b), _ptr(x))
        if rc:
            raise OracleError(rc, "orc_amg_solve")
        return x

    def vcycle(self, hier: int, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        rc = self.lib.orc_vcycle(self.h, hier, _ptr(b), _ptr(x))
        if rc:
            raise OracleError(rc, "orc_vcycle")
        return x

    def smooth(self, hier: int, lev: int, b: np.ndarray, x: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x, dtype=np.float64, copy=True)
        rc = self.lib.orc_smooth(self.h, hier, lev, _ptr(b), _ptr(x))
        if rc:
            raise OracleError(rc, "orc_smooth")
        return x

    def schur_solve(self, species: int, b: np.ndarray) -> np.ndarray:
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros_like(b)
        rc = self.lib.orc_schur_solve(self.h, species, _ptr(b), _ptr(x))
        if rc:
            raise OracleError(rc, "orc_schur_solve")
        return x

    # --- operators and solves ----------------------------------------
    def apply_saddle(self, species: int, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(x)
        rc = self.lib.orc_apply_saddle(self.h, species, _ptr(x), _ptr(y))
        if rc:
            raise OracleError(rc, "orc_apply_saddle")
        return y

    def apply_prec(self, species: int, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.float64)
        w = np.zeros_like(v)
        rc = self.lib.orc_apply_prec(self.h, species, _ptr(v), _ptr(w))
        if rc:
            raise OracleError(rc, "orc_apply_prec")
        return w

    def rhs(self, php: np.ndarray, phn: np.ndarray):
        php = np.ascontiguousarray(php, dtype=np.float64)
        phn = np.ascontiguousarray(phn, dtype=np.float64)
        bp = np.zeros(2 * self.nv)
        bn = np.zeros(2 * self.nv)
        rc = self.lib.orc_rhs(self.h, _ptr(php), _ptr(phn), _ptr(bp), _ptr(bn))
        if rc:
            raise OracleError(rc, "orc_rhs")
        return bp, bn

    def boundary(self, php: np.ndarray, phn: np.ndarray):
        """The boundary vectors (G_p, G_n) of eq. chternary:2 for the state."""
        php = np.ascontiguousarray(php, dtype=np.float64)
        phn = np.ascontiguousarray(phn, dtype=np.float64)
        gp, gn = np.zeros(self.nv), np.zeros(self.nv)
        rc = self.lib.orc_boundary(self.h, _ptr(php), _ptr(phn), _ptr(gp), _ptr(gn))
        if rc:
            raise OracleError(rc, "orc_boundary")
        return gp, gn

    def minres(self, species: int, b: np.ndarray, x0: np.ndarray, allow_noconv: bool = False):
        """MINRES from x0; with allow_noconv the iterate after max_iters is
        returned instead of an error."""
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, copy=True)
        it = C.c_int32()
        rr = C.c_double()
        rc = self.lib.orc_minres(self.h, species, _ptr(b), _ptr(x), C.byref(it), C.byref(rr))
        if rc and not (allow_noconv and rc == -4):
            raise OracleError(rc, "orc_minres")
        return x, it.value, rr.value

    def fgmres(self, species: int, b: np.ndarray, x0: np.ndarray):
        b = np.ascontiguousarray(b, dtype=np.float64)
        x = np.array(x0, dtype=np.float64, copy=True)
        it = C.c_int32()
        rr = C.c_double()
        rc = self.lib.orc_fgmres(self.h, species, _ptr(b), _ptr(x), C.byref(it), C.byref(rr))
        if rc:
            raise OracleError(rc, "orc_fgmres")
        return x, it.value, rr.value

    def step(self, state: dict) -> dict:
        """One time step on a state dict with phi_p, phi_n, mu_p, mu_n (copied)."""
        php = np.array(state["phi_p"], dtype=np.float64, copy=True)
        phn = np.array(state["phi_n"], dtype=np.float64, copy=True)
        mup = np.array(state["mu_p"], dtype=np.float64, copy=True)
        mun = np.array(state["mu_n"], dtype=np.float64, copy=True)
        st = orc_stats_t()
        rc = self.lib.orc_step(self.h, _ptr(php), _ptr(phn), _ptr(mup), _ptr(mun), C.byref(st))
        stats = dict(iters=(st.iters[0], st.iters[1]), relres=(st.relres[0], st.relres[1]),
                     status=st.status, clamped=st.clamped, outside=st.outside)
        if rc:
            raise OracleError(rc, f"orc_step (stats {stats})")
        return dict(phi_p=php, phi_n=phn, mu_p=mup, mu_n=mun, stats=stats)

    def schur_info(self):
        """(CG steps per As solve in use, measured V-cycle contraction or 0)."""
        k, rho = C.c_int32(), C.c_double()
        rc = self.lib.orc_schur_info(self.h, C.byref(k), C.byref(rho))
        if rc:
            raise OracleError(rc, "orc_schur_info")
        return k.value, rho.value

    def energy(self, php: np.ndarray, phn: np.ndarray) -> float:
        php = np.ascontiguousarray(php, dtype=np.float64)
        phn = np.ascontiguousarray(phn, dtype=np.float64)
        return self.lib.orc_energy(self.h, _ptr(php), _ptr(phn))
