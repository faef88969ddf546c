"""Python binding of the C ABI in include/chm.h (argument marshalling only).

Every function here forwards to the same-named symbol of ``libchm.so``; the
computation runs in the library's HIP kernels.  PyTorch supplies device memory
(``tensor.data_ptr()``) and the HIP stream.  If the library is not built the
import fails loudly: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libchm.so")

CHM_OK, CHM_EINVAL, CHM_ENOMEM, CHM_EHIP, CHM_ENOCONV, CHM_ENAN = 0, -1, -2, -3, -4, -5
CHM_EDOMAIN = -6
CODES = {0: "CHM_OK", -1: "CHM_EINVAL", -2: "CHM_ENOMEM", -3: "CHM_EHIP", -4: "CHM_ENOCONV",
         -5: "CHM_ENAN", -6: "CHM_EDOMAIN"}
POTENTIALS = {"flory_huggins": 0, "polynomial": 1, "none": 2}
SMOOTHERS = {"chebyshev": 0, "jacobi": 1}

# exported entry points (must match include/chm.h)
ENTRY_POINTS = [
    "chm_create", "chm_set_fields", "chm_step", "chm_get_fields", "chm_destroy",
    "chm_last_error", "chm_nnz", "chm_get_matrix", "chm_num_levels", "chm_level_info",
    "chm_level_get", "chm_vcycle", "chm_schur_solve", "chm_apply_saddle", "chm_apply_prec",
    "chm_rhs", "chm_quadrature", "chm_timer_enable", "chm_timer_read", "chm_setup_info",
    "chm_net_create", "chm_net_destroy", "chm_net_last_error", "chm_net_set_params",
    "chm_net_get_params", "chm_net_features", "chm_net_forward", "chm_net_gradients",
    "chm_net_adam", "chm_net_guess", "chm_net_train_step", "chm_set_guess", "chm_get_state",
    "chm_create_batch", "chm_batch_size", "chm_set_fields_run", "chm_get_fields_run",
    "chm_boundary", "chm_level_layout", "chm_get_history", "chm_set_history", "chm_value_table",
    "chm_net_guess_noalloc", "chm_step_many", "chm_schur_info",
]

NET_LAYERS = ((8, 32), (32, 32), (32, 32), (32, 4))
NET_NPARAMS = sum(9 * ci * co + co for ci, co in NET_LAYERS)
GUESS_MODES = {"previous": 0, "linear": 1, "learned": 2}


class ChmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{CODES.get(code, code)}: {msg}")
        self.code = code


class chm_mesh_t(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int64), ("coords", C.c_void_p),
                ("n_cells", C.c_int64), ("cells", C.c_void_p)]


class chm_params_t(C.Structure):
    _fields_ = [
        ("tau", C.c_double), ("eps", C.c_double * 2), ("mobility", C.c_double * 2),
        ("potential", C.c_int32), ("Np", C.c_double), ("Nn", C.c_double), ("Ns", C.c_double),
        ("chi_pn", C.c_double), ("chi_ps", C.c_double), ("chi_ns", C.c_double),
        ("log_floor", C.c_double), ("evap_ds", C.c_double), ("evap_steps", C.c_int32),
        ("rtol", C.c_double), ("restart", C.c_int32), ("max_iters", C.c_int32),
        ("amg_cycles", C.c_int32), ("schur_pcg", C.c_int32), ("smoother", C.c_int32),
        ("cheb_degree", C.c_int32), ("cheb_ratio", C.c_double),
        ("cheb_degree_mass", C.c_int32), ("cheb_ratio_mass", C.c_double),
        ("coarse_max", C.c_int32), ("max_levels", C.c_int32), ("use_graphs", C.c_int32),
        ("precision", C.c_int32),
        ("boundary", C.c_int32), ("bc_k", C.c_double), ("bc_g", C.c_double * 2),
        ("bc_h", C.c_double * 2), ("bc_pattern", C.c_int32), ("krylov", C.c_int32),
        ("amg_tol", C.c_double), ("mass_solver", C.c_int32), ("wide_index", C.c_int32),
        ("runs_per_lane", C.c_int32), ("cheb_degree_coarse", C.c_int32),
        ("range_check", C.c_int32), ("ortho", C.c_int32), ("values_direct", C.c_int32),
    ]


class chm_run_t(C.Structure):
    _fields_ = [("chi_pn", C.c_double), ("chi_ps", C.c_double), ("chi_ns", C.c_double),
                ("evap_ds", C.c_double), ("evap_steps", C.c_int32)]


class chm_stats_t(C.Structure):
    _fields_ = [("iters", C.c_int32 * 2), ("relres", C.c_double * 2), ("status", C.c_int32),
                ("clamped", C.c_int32), ("t_step_ms", C.c_double), ("guess_used", C.c_int32 * 2),
                ("res0", C.c_double * 2), ("outside", C.c_int32)]


_lib = None


def library():
    """Load libchm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        lib = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        P = C.POINTER
        sig = {
            "chm_create": ([P(chm_mesh_t), P(chm_params_t), vp, P(vp)], C.c_int),
            "chm_set_fields": ([vp, vp, vp, vp, vp, i32], C.c_int),
            "chm_step": ([vp, i32, P(chm_stats_t)], C.c_int),
            "chm_get_fields": ([vp, vp, vp, vp, vp, vp, i32], C.c_int),
            "chm_destroy": ([vp], C.c_int),
            "chm_last_error": ([vp], C.c_char_p),
            "chm_nnz": ([vp], i64),
            "chm_get_matrix": ([vp, i32, vp, vp, vp], C.c_int),
            "chm_num_levels": ([vp, i32], C.c_int),
            "chm_level_info": ([vp, i32, i32, P(i64), P(i64), P(i64), P(d)], C.c_int),
            "chm_level_layout": ([vp, i32, i32, P(i32), P(i32)], C.c_int),
            "chm_value_table": ([vp, i32, i32, P(i32)], C.c_int),
            "chm_level_get": ([vp, i32, i32, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "chm_vcycle": ([vp, i32, vp, vp], C.c_int),
            "chm_schur_solve": ([vp, vp, vp], C.c_int),
            "chm_apply_saddle": ([vp, vp, vp], C.c_int),
            "chm_apply_prec": ([vp, vp, vp], C.c_int),
            "chm_rhs": ([vp, vp], C.c_int),
            "chm_quadrature": ([i32, P(i32), vp, vp], C.c_int),
            "chm_timer_enable": ([vp, i32, i32], C.c_int),
            "chm_timer_read": ([vp, P(i64), P(d), P(i64)], C.c_int),
            "chm_setup_info": ([vp, P(d), P(i64), P(i64)], C.c_int),
            "chm_net_create": ([i64, vp, P(vp)], C.c_int),
            "chm_net_destroy": ([vp], C.c_int),
            "chm_net_last_error": ([vp], C.c_char_p),
            "chm_net_set_params": ([vp, vp], C.c_int),
            "chm_net_get_params": ([vp, vp], C.c_int),
            "chm_net_features": ([vp, i32, i32, vp, vp, vp, vp], C.c_int),
            "chm_net_forward": ([vp, i32, i32, i32, vp, vp], C.c_int),
            "chm_net_gradients": ([vp, i32, i32, i32, vp, vp, vp, vp, C.c_float, vp, P(d)],
                                  C.c_int),
            "chm_net_adam": ([vp, vp, C.c_float], C.c_int),
            "chm_net_guess": ([vp, i32, i32, vp, vp, vp], C.c_int),
            "chm_net_guess_noalloc": ([vp, i32, i32, vp, vp, vp], C.c_int),
            "chm_net_train_step": ([vp, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, C.c_float,
                                    C.c_float, P(d)], C.c_int),
            "chm_set_guess": ([vp, i32, vp, i32, i32], C.c_int),
            "chm_get_state": ([vp, i32, vp], C.c_int),
            "chm_create_batch": ([P(chm_mesh_t), P(chm_params_t), i32, vp, vp, P(vp)], C.c_int),
            "chm_batch_size": ([vp], C.c_int),
            "chm_set_fields_run": ([vp, i32, vp, vp, vp, vp, i32], C.c_int),
            "chm_get_fields_run": ([vp, i32, vp, vp, vp, vp, vp, i32], C.c_int),
            "chm_boundary": ([vp, vp], C.c_int),
            "chm_get_history": ([vp, i32, vp, vp, P(i32), P(i64), i32], C.c_int),
            "chm_step_many": ([vp, i32, i32, vp, vp], C.c_int),
            "chm_schur_info": ([vp, P(i32), P(d)], C.c_int),
            "chm_set_history": ([vp, i32, vp, vp, i32, i64, i32], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def params_from_dict(p: dict) -> chm_params_t:
    s = chm_params_t()
    s.tau = p["tau"]
    eps = p["eps"] if isinstance(p["eps"], (list, tuple)) else (p["eps"], p["eps"])
    mob = p["mobility"] if isinstance(p["mobility"], (list, tuple)) else (p["mobility"],) * 2
    s.eps[0], s.eps[1] = eps
    s.mobility[0], s.mobility[1] = mob
    s.potential = POTENTIALS[p["potential"]]
    for k in ("Np", "Nn", "Ns", "chi_pn", "chi_ps", "chi_ns", "log_floor", "rtol",
              "cheb_ratio", "cheb_ratio_mass"):
        setattr(s, k, float(p[k]))
    s.evap_ds = float(p.get("evap_ds", 0.0))
    s.evap_steps = int(p.get("evap_steps", p.get("steps", 0))) if s.evap_ds > 0 else 0
    for k in ("restart", "max_iters", "amg_cycles", "schur_pcg", "cheb_degree",
              "cheb_degree_mass", "coarse_max", "max_levels"):
        setattr(s, k, int(p[k]))
    s.smoother = SMOOTHERS[p["smoother"]]
    s.use_graphs = int(p.get("use_graphs", 1))
    s.precision = {"fp64": 0, "fp32": 1}[p.get("precision", "fp64")]
    s.boundary = int(p.get("boundary", 0))
    s.bc_k = float(p.get("bc_k", 0.0))
    s.bc_g[0], s.bc_g[1] = p.get("bc_g", (0.0, 0.0))
    s.bc_h[0], s.bc_h[1] = p.get("bc_h", (0.0, 0.0))
    s.bc_pattern = int(p.get("bc_pattern", 0))
    s.krylov = {"fgmres": 0, "minres": 1}[p.get("krylov", "fgmres")]
    s.amg_tol = float(p.get("amg_tol", 0.0))
    s.mass_solver = {"amg": 0, "chebyshev": 1}[p.get("mass_solver", "amg")]
    s.wide_index = int(p.get("wide_index", 0))
    s.runs_per_lane = int(p.get("runs_per_lane", 0))
    s.cheb_degree_coarse = int(p.get("cheb_degree_coarse", 0))
    s.range_check = int(p.get("range_check", 0))
    s.ortho = {"dcgs2": 0, "cgs2": 1}[p.get("ortho", "dcgs2")]
    s.values_direct = int(p.get("values_direct", 0))
    return s


def _check(h, rc: int, what: str):
    if rc != CHM_OK:
        msg = library().chm_last_error(h)
        raise ChmError(rc, f"{what}: {msg.decode() if msg else ''}")


def _dev_ptr(t):
    return C.c_void_p(t.data_ptr())


def chm_quadrature(dim: int):
    bary = np.zeros(64 * 4)
    w = np.zeros(64)
    n = C.c_int32()
    rc = library().chm_quadrature(dim, C.byref(n), bary.ctypes.data_as(C.c_void_p),
                                  w.ctypes.data_as(C.c_void_p))
    if rc:
        raise ChmError(rc, "chm_quadrature")
    k = n.value
    return bary[: k * (dim + 1)].reshape(k, dim + 1).copy(), w[:k].copy()


def run_from_dict(p: dict) -> chm_run_t:
    """The per-run values of a parameter dict (chi's, solvent removal)."""
    r = chm_run_t()
    r.chi_pn, r.chi_ps, r.chi_ns = float(p["chi_pn"]), float(p["chi_ps"]), float(p["chi_ns"])
    r.evap_ds = float(p.get("evap_ds", 0.0))
    r.evap_steps = int(p.get("evap_steps", p.get("steps", 0))) if r.evap_ds > 0 else 0
    return r


class Solver:
    """One chm_solver_t on the current torch device and stream.  runs: None
    for one run, or a list of parameter dicts (one per run of a batch; only
    their chi's and solvent removal may differ from params)."""

    def __init__(self, coords: np.ndarray, cells: np.ndarray, params: dict, stream=None,
                 runs=None):
        import torch
        self.torch = torch
        self.lib = library()
        self.coords = np.ascontiguousarray(coords, dtype=np.float64)
        self.cells = np.ascontiguousarray(cells, dtype=np.int32)
        self.dim = self.coords.shape[1]
        self.nv = self.coords.shape[0]
        self.params = dict(params)
        mesh = chm_mesh_t(self.dim, self.nv, self.coords.ctypes.data_as(C.c_void_p),
                          self.cells.shape[0], self.cells.ctypes.data_as(C.c_void_p))
        self._prm = params_from_dict(params)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = C.c_void_p()
        self.nb = 1 if runs is None else len(runs)
        if runs is None:
            rc = self.lib.chm_create(C.byref(mesh), C.byref(self._prm), C.c_void_p(stream),
                                     C.byref(h))
        else:
            rp = (chm_run_t * self.nb)(*[run_from_dict(dict(params, **r)) for r in runs])
            rc = self.lib.chm_create_batch(C.byref(mesh), C.byref(self._prm), self.nb, rp,
                                           C.c_void_p(stream), C.byref(h))
        if rc != CHM_OK:
            msg = self.lib.chm_last_error(None)
            raise ChmError(rc, f"chm_create: {msg.decode() if msg else ''}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.chm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- state
    def set_fields(self, phi_p, phi_n, mu_p=None, mu_n=None, run: int = 0):
        torch = self.torch
        ts = [None if a is None else torch.as_tensor(np.asarray(a, dtype=np.float64)).cuda()
              for a in (phi_p, phi_n, mu_p, mu_n)]
        ptrs = [None if t is None else _dev_ptr(t) for t in ts]
        rc = self.lib.chm_set_fields_run(self.h, run, *ptrs, 1)
        _check(self.h, rc, "chm_set_fields")

    def get_fields(self, run: int = 0) -> dict:
        torch = self.torch
        out = {k: torch.empty(self.nv, dtype=torch.float64, device="cuda")
               for k in ("phi_p", "phi_n", "phi_s", "mu_p", "mu_n")}
        rc = self.lib.chm_get_fields_run(self.h, run, *(_dev_ptr(out[k]) for k in
                                                        ("phi_p", "phi_n", "phi_s", "mu_p",
                                                         "mu_n")), 1)
        _check(self.h, rc, "chm_get_fields")
        return {k: v.cpu().numpy() for k, v in out.items()}

    def step(self, nsteps: int = 1):
        """Per step: a stats dict (one run) or a list of them (one per run)."""
        nb = self.nb
        st = (chm_stats_t * max(1, nsteps * nb))()
        rc = self.lib.chm_step(self.h, nsteps, st)
        flat = [dict(iters=(s.iters[0], s.iters[1]), relres=(s.relres[0], s.relres[1]),
                     status=s.status, clamped=s.clamped, t_step_ms=s.t_step_ms,
                     guess_used=(s.guess_used[0], s.guess_used[1]),
                     res0=(s.res0[0], s.res0[1]), outside=s.outside)
                for s in st[:nsteps * nb]]
        stats = flat if nb == 1 else [flat[k * nb:(k + 1) * nb] for k in range(nsteps)]
        if rc != CHM_OK:
            msg = self.lib.chm_last_error(self.h)
            err = ChmError(rc, f"chm_step: {msg.decode() if msg else ''}")
            err.stats = stats
            raise err
        return stats

    def schur_info(self):
        """(CG steps per As solve in use, measured V-cycle contraction or 0)."""
        k, rho = C.c_int32(), C.c_double()
        _check(self.h, self.lib.chm_schur_info(self.h, C.byref(k), C.byref(rho)),
               "chm_schur_info")
        return k.value, rho.value

    def get_history(self, run: int = 0) -> dict:
        """Checkpoint data beyond the fields: the last two solutions of the
        solve (CUDA tensors, state-vector layout; None past `valid`), how
        many are valid, and the run's completed steps."""
        torch = self.torch
        y1 = torch.empty(4 * self.nv, dtype=torch.float64, device="cuda")
        y2 = torch.empty_like(y1)
        valid, steps = C.c_int32(), C.c_int64()
        rc = self.lib.chm_get_history(self.h, run, _dev_ptr(y1), _dev_ptr(y2), C.byref(valid),
                                      C.byref(steps), 1)
        _check(self.h, rc, "chm_get_history")
        return dict(y1=y1 if valid.value >= 1 else None, y2=y2 if valid.value >= 2 else None,
                    valid=valid.value, steps=steps.value)

    def set_history(self, hist: dict, run: int = 0):
        """Restore what get_history returned (after set_fields)."""
        ptr = lambda t: None if t is None else _dev_ptr(t)
        rc = self.lib.chm_set_history(self.h, run, ptr(hist["y1"]), ptr(hist["y2"]),
                                      int(hist["valid"]), int(hist["steps"]), 1)
        _check(self.h, rc, "chm_set_history")

    def set_guess(self, mode: str, net=None, H: int = 0, W: int = 0):
        rc = self.lib.chm_set_guess(self.h, GUESS_MODES[mode], net.h if net is not None else None,
                                    H, W)
        _check(self.h, rc, "chm_set_guess")

    def boundary(self):
        """The boundary vectors (G_p, G_n) of the current state (run 0)."""
        g = self.torch.empty(2 * self.nv, dtype=self.torch.float64, device="cuda")
        _check(self.h, self.lib.chm_boundary(self.h, _dev_ptr(g)), "chm_boundary")
        g = g.cpu().numpy()
        return g[0::2].copy(), g[1::2].copy()

    def get_state(self, solution: bool = False):
        """The state vector (4 n doubles, solver block layout) as a CUDA tensor;
        solution=True: the last solution of the solve (before solvent removal)."""
        out = self.torch.empty(4 * self.nv, dtype=self.torch.float64, device="cuda")
        _check(self.h, self.lib.chm_get_state(self.h, int(solution), _dev_ptr(out)),
               "chm_get_state")
        return out

    # ---- inspection
    def nnz(self) -> int:
        return self.lib.chm_nnz(self.h)

    def matrix(self, which: str):
        idx = {"M": 0, "K": 1, "As": 2}[which]
        nnz = self.nnz()
        rp = np.zeros(self.nv + 1, np.int32)
        ci = np.zeros(nnz, np.int32)
        v = np.zeros(nnz)
        rc = self.lib.chm_get_matrix(self.h, idx, rp.ctypes.data_as(C.c_void_p),
                                     ci.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p))
        _check(self.h, rc, "chm_get_matrix")
        return rp, ci, v

    def num_levels(self, hier: int) -> int:
        return self.lib.chm_num_levels(self.h, hier)

    def layout(self, hier: int, lev: int = 0) -> tuple:
        """(lanes per row, bytes per column index) of a level's A as the solve
        kernels read it; hier = -1 for the solver's M, K, As."""
        lanes, ib = C.c_int32(), C.c_int32()
        rc = self.lib.chm_level_layout(self.h, hier, lev, C.byref(lanes), C.byref(ib))
        _check(self.h, rc, "chm_level_layout")
        return lanes.value, ib.value

    def value_table(self, hier: int, lev: int = 0) -> int:
        """Distinct values in the value table of a level's A (hier 0 or 1), or
        of M (hier -1, lev 0) / K (hier -1, lev 1); 0 = no table."""
        m = C.c_int32()
        rc = self.lib.chm_value_table(self.h, hier, lev, C.byref(m))
        _check(self.h, rc, "chm_value_table")
        return m.value

    def level(self, hier: int, lev: int) -> dict:
        n, na, npp = C.c_int64(), C.c_int64(), C.c_int64()
        rho = C.c_double()
        rc = self.lib.chm_level_info(self.h, hier, lev, C.byref(n), C.byref(na), C.byref(npp),
                                     C.byref(rho))
        _check(self.h, rc, "chm_level_info")
        n, na, npp = n.value, na.value, npp.value
        arr = dict(Arp=np.zeros(n + 1, np.int32), Aci=np.zeros(na, np.int32), Av=np.zeros(na),
                   agg=np.full(n, -1, np.int32), Prp=np.zeros(n + 1, np.int32),
                   Pci=np.zeros(npp, np.int32), Pv=np.zeros(npp))
        rc = self.lib.chm_level_get(self.h, hier, lev,
                                    *(arr[k].ctypes.data_as(C.c_void_p) for k in
                                      ("Arp", "Aci", "Av", "agg", "Prp", "Pci", "Pv")))
        _check(self.h, rc, "chm_level_get")
        out = dict(n=n, rho=rho.value, A=(arr["Arp"], arr["Aci"], arr["Av"]))
        if npp:
            out.update(agg=arr["agg"], P=(arr["Prp"], arr["Pci"], arr["Pv"]),
                       nc=int(arr["agg"].max()) + 1)
        return out

    def _pairs(self, a, b=None):
        """[n] x 2 pair layout from one or two host arrays."""
        torch = self.torch
        a = np.asarray(a, dtype=np.float64)
        if b is None:
            b = a
        t = torch.tensor(np.stack([a, np.asarray(b, dtype=np.float64)], axis=1), device="cuda")
        return t.contiguous()

    def vcycle(self, hier: int, b0, b1=None):
        """One V-cycle from zero on two right-hand sides; returns (x0, x1)."""
        torch = self.torch
        b = self._pairs(b0, b1)
        x = torch.zeros_like(b)
        rc = self.lib.chm_vcycle(self.h, hier, _dev_ptr(b), _dev_ptr(x))
        _check(self.h, rc, "chm_vcycle")
        x = x.cpu().numpy()
        return x[:, 0].copy(), x[:, 1].copy()

    def schur_solve(self, b0, b1=None):
        torch = self.torch
        b = self._pairs(b0, b1)
        x = torch.zeros_like(b)
        rc = self.lib.chm_schur_solve(self.h, _dev_ptr(b), _dev_ptr(x))
        _check(self.h, rc, "chm_schur_solve")
        x = x.cpu().numpy()
        return x[:, 0].copy(), x[:, 1].copy()

    def _block(self, v0, v1):
        """Block-vector layout from two species' vectors of length 2n."""
        v0 = np.asarray(v0, dtype=np.float64)
        v1 = np.asarray(v1, dtype=np.float64)
        return self.torch.tensor(np.stack([v0, v1], axis=1), device="cuda").contiguous()

    def _unblock(self, t):
        a = t.cpu().numpy()
        return a[:, 0].copy(), a[:, 1].copy()

    def apply_saddle(self, x0, x1):
        x = self._block(x0, x1)
        y = self.torch.zeros_like(x)
        rc = self.lib.chm_apply_saddle(self.h, _dev_ptr(x), _dev_ptr(y))
        _check(self.h, rc, "chm_apply_saddle")
        return self._unblock(y)

    def apply_prec(self, v0, v1):
        v = self._block(v0, v1)
        w = self.torch.zeros_like(v)
        rc = self.lib.chm_apply_prec(self.h, _dev_ptr(v), _dev_ptr(w))
        _check(self.h, rc, "chm_apply_prec")
        return self._unblock(w)

    def rhs(self):
        b = self.torch.zeros((2 * self.nv, 2), dtype=self.torch.float64, device="cuda")
        rc = self.lib.chm_rhs(self.h, _dev_ptr(b))
        _check(self.h, rc, "chm_rhs")
        return self._unblock(b)

    def timer_enable(self, kind: int = 0, enable: bool = True):
        _check(self.h, self.lib.chm_timer_enable(self.h, kind, int(enable)), "chm_timer_enable")

    def timer_read(self):
        n, ms, by = C.c_int64(), C.c_double(), C.c_int64()
        _check(self.h, self.lib.chm_timer_read(self.h, C.byref(n), C.byref(ms), C.byref(by)),
               "chm_timer_read")
        return n.value, ms.value, by.value

    def setup_info(self):
        ms, lm, la = C.c_double(), C.c_int64(), C.c_int64()
        self.lib.chm_setup_info(self.h, C.byref(ms), C.byref(lm), C.byref(la))
        return dict(setup_ms=ms.value, levels_mass=lm.value, levels_as=la.value)


# ---------------------------------------------------------------- learned guess
def flatten_params(params) -> np.ndarray:
    """[(w [3, 3, ci, co], b [co]), ...] -> the flat FP32 parameter layout."""
    out = []
    for (w, b), (ci, co) in zip(params, NET_LAYERS):
        w = np.asarray(w, dtype=np.float32)
        b = np.asarray(b, dtype=np.float32)
        assert w.shape == (3, 3, ci, co) and b.shape == (co,)
        out += [w.ravel(), b.ravel()]
    flat = np.concatenate(out)
    assert flat.size == NET_NPARAMS
    return np.ascontiguousarray(flat)


def unflatten_params(flat) -> list:
    flat = np.asarray(flat, dtype=np.float32)
    out, k = [], 0
    for ci, co in NET_LAYERS:
        w = flat[k:k + 9 * ci * co].reshape(3, 3, ci, co).copy()
        k += 9 * ci * co
        b = flat[k:k + co].copy()
        k += co
        out.append((w, b))
    return out


def step_many(solvers, nsteps: int = 1):
    """chm_step_many: advance the solvers concurrently (one host thread each;
    give each its own stream so their launches overlap).  Returns per solver
    what Solver.step returns."""
    count = len(solvers)
    handles = (C.c_void_p * count)(*[s.h for s in solvers])
    bufs = [(chm_stats_t * max(1, nsteps * s.nb))() for s in solvers]
    ptrs = (C.c_void_p * count)(*[C.cast(b, C.c_void_p) for b in bufs])
    codes = (C.c_int32 * count)()
    rc = library().chm_step_many(handles, count, nsteps, ptrs, codes)
    out = []
    for s, b in zip(solvers, bufs):
        flat = [dict(iters=(x.iters[0], x.iters[1]), relres=(x.relres[0], x.relres[1]),
                     status=x.status, clamped=x.clamped, t_step_ms=x.t_step_ms,
                     guess_used=(x.guess_used[0], x.guess_used[1]), res0=(x.res0[0], x.res0[1]),
                     outside=x.outside)
                for x in b[:nsteps * s.nb]]
        out.append(flat if s.nb == 1 else [flat[k * s.nb:(k + 1) * s.nb] for k in range(nsteps)])
    if rc != CHM_OK:
        bad = next(i for i in range(count) if codes[i] != CHM_OK)
        _check(solvers[bad].h, codes[bad], f"chm_step_many (solver {bad})")
    return out


class Net:
    """One chm_net_t (the guess network) on the current torch stream.
    Tensors passed in are torch CUDA tensors; marshalling only."""

    def __init__(self, max_pixels: int, stream=None):
        import torch
        self.torch = torch
        self.lib = library()
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        h = C.c_void_p()
        rc = self.lib.chm_net_create(int(max_pixels), C.c_void_p(stream), C.byref(h))
        if rc != CHM_OK:
            msg = self.lib.chm_net_last_error(None)
            raise ChmError(rc, f"chm_net_create: {msg.decode() if msg else ''}")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.chm_net_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def _check(self, rc, what):
        if rc != CHM_OK:
            msg = self.lib.chm_net_last_error(self.h)
            raise ChmError(rc, f"{what}: {msg.decode() if msg else ''}")

    def set_params(self, params):
        flat = params if isinstance(params, np.ndarray) else flatten_params(params)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(self.lib.chm_net_set_params(self.h, flat.ctypes.data_as(C.c_void_p)),
                    "chm_net_set_params")

    def get_params(self, flat: bool = False):
        out = np.zeros(NET_NPARAMS, np.float32)
        self._check(self.lib.chm_net_get_params(self.h, out.ctypes.data_as(C.c_void_p)),
                    "chm_net_get_params")
        return out if flat else unflatten_params(out)

    def features(self, H: int, W: int, x2, x1):
        torch = self.torch
        feats = torch.empty((H, W, 8), dtype=torch.float32, device="cuda")
        sigma = np.zeros(4)
        self._check(self.lib.chm_net_features(self.h, H, W, _dev_ptr(x2), _dev_ptr(x1),
                                              _dev_ptr(feats), sigma.ctypes.data_as(C.c_void_p)),
                    "chm_net_features")
        return feats, sigma

    def forward(self, feats):
        torch = self.torch
        feats = feats.contiguous()
        B, h, w, _ = feats.shape
        y = torch.empty((B, h, w, 4), dtype=torch.float32, device="cuda")
        self._check(self.lib.chm_net_forward(self.h, B, h, w, _dev_ptr(feats), _dev_ptr(y)),
                    "chm_net_forward")
        return y

    def gradients(self, feats, target, mask, weights=None, smooth: float = 0.0):
        feats, target = feats.contiguous(), target.contiguous()
        mask = mask.to(self.torch.uint8).contiguous()
        B, h, w, _ = feats.shape
        g = np.zeros(NET_NPARAMS, np.float32)
        loss = C.c_double()
        wts = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
        self._check(self.lib.chm_net_gradients(
            self.h, B, h, w, _dev_ptr(feats), _dev_ptr(target), _dev_ptr(mask),
            None if wts is None else wts.ctypes.data_as(C.c_void_p), float(smooth),
            g.ctypes.data_as(C.c_void_p), C.byref(loss)), "chm_net_gradients")
        return unflatten_params(g), loss.value

    def adam(self, grads, lr: float):
        flat = grads if isinstance(grads, np.ndarray) else flatten_params(grads)
        flat = np.ascontiguousarray(flat, dtype=np.float32)
        self._check(self.lib.chm_net_adam(self.h, flat.ctypes.data_as(C.c_void_p), float(lr)),
                    "chm_net_adam")

    def guess(self, H: int, W: int, x2, x1):
        out = self.torch.empty_like(x1)
        self._check(self.lib.chm_net_guess(self.h, H, W, _dev_ptr(x2), _dev_ptr(x1), _dev_ptr(out)),
                    "chm_net_guess")
        return out

    def guess_noalloc(self, H: int, W: int, x2, x1, out):
        """chm_net_guess_noalloc into the caller's tensor `out`; enqueued on
        the network's stream (the caller synchronises)."""
        self._check(self.lib.chm_net_guess_noalloc(self.h, H, W, _dev_ptr(x2), _dev_ptr(x1),
                                                   _dev_ptr(out)), "chm_net_guess_noalloc")
        return out

    def train_step(self, H: int, W: int, crop_h: int, crop_w: int, x2s, x1s, x0s, oy, ox,
                   lr: float, smooth: float = 0.0) -> float:
        B = len(x2s)
        arr = lambda ts: (C.c_void_p * B)(*[t.data_ptr() for t in ts])
        oy = np.ascontiguousarray(oy, dtype=np.int32)
        ox = np.ascontiguousarray(ox, dtype=np.int32)
        loss = C.c_double()
        self._check(self.lib.chm_net_train_step(self.h, B, H, W, crop_h, crop_w, arr(x2s), arr(x1s),
                                                arr(x0s), oy.ctypes.data_as(C.c_void_p),
                                                ox.ctypes.data_as(C.c_void_p), float(lr),
                                                float(smooth), C.byref(loss)), "chm_net_train_step")
        return loss.value

