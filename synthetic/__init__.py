"""Seeded synthetic inputs for the ternary Cahn-Hilliard solve.

This module is shared by the CPU oracle tests, the GPU parity tests and the
benchmark.  It produces inputs only: meshes (vertex coordinates and simplex
connectivity), initial volume fractions with seeded uniform noise, and plain
parameter presets.  It holds none of the method's arithmetic (no matrices, no
potentials, no solver steps).

Mesh conventions
----------------
* 2D: an ``nx x ny`` grid of squares on ``[0, Lx] x [0, Ly]``, vertices
  numbered lexicographically with x fastest, ``v(i, j) = j*(nx+1) + i``.
  Each square with corners a=(i,j), b=(i+1,j), c=(i+1,j+1), d=(i,j+1) is cut
  along the a-c diagonal into the triangles (a,b,c) and (a,c,d).  The paper
  uses uniform P1 triangulations of rectangles (Section 4); the diagonal
  direction is not stated there.
* 3D: an ``nx x ny x nz`` grid of boxes, each cut into the six Kuhn
  tetrahedra that share the main diagonal (0,0,0)-(1,1,1) of the box.

Random numbers
--------------
Counter-based SplitMix64 (Steele, Lea and Flood, 2014): the k-th draw of
stream ``seed`` is ``mix(seed + (k+1)*0x9E3779B97F4A7C15)``; a double in
[0, 1) takes the top 53 bits.  The initial state follows Section 4 of the
paper: a mean volume fraction per component plus a uniform perturbation of
amplitude 0.01, then each node's three fractions are renormalised to sum to
one (the constraint of equation (eq:sumphis)).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "mesh_rect_2d", "mesh_box_3d", "splitmix64", "uniform01",
    "initial_fractions", "preset", "PRESETS", "BASE_SEED",
]

BASE_SEED = 20220407

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mesh_rect_2d(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0):
    """Uniform right-diagonal triangulation of ``[0,lx] x [0,ly]``.

    Returns ``(coords float64[(nx+1)*(ny+1), 2], cells int32[2*nx*ny, 3])``.
    """
    if nx < 1 or ny < 1:
        raise ValueError("need at least one cell per direction")
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")          # [ny+1, nx+1]
    coords = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    a = (j * (nx + 1) + i).ravel()
    b = a + 1
    c = a + (nx + 1) + 1
    d = a + (nx + 1)
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    cells = np.empty((2 * nx * ny, 3), dtype=np.int32)
    cells[0::2] = t1
    cells[1::2] = t2
    return coords, cells


def mesh_box_3d(nx: int, ny: int, nz: int, lx: float = 1.0, ly: float = 1.0,
                lz: float = 1.0):
    """Kuhn (six-tetrahedra) triangulation of ``[0,lx] x [0,ly] x [0,lz]``.

    Returns ``(coords float64[(nx+1)(ny+1)(nz+1), 3], cells int32[6*nx*ny*nz, 4])``;
    vertex ``(i,j,k)`` has index ``(k*(ny+1) + j)*(nx+1) + i``.
    """
    if min(nx, ny, nz) < 1:
        raise ValueError("need at least one cell per direction")
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = ((k * (ny + 1) + j) * (nx + 1) + i).ravel()
    step = (1, nx + 1, (nx + 1) * (ny + 1))   # vertex offset of a +1 move in x, y, z
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    cells = np.empty((6 * base.size, 4), dtype=np.int32)
    for t, p in enumerate(perms):
        v0 = base
        v1 = v0 + step[p[0]]
        v2 = v1 + step[p[1]]
        v3 = v2 + step[p[2]]
        cells[t::6] = np.stack([v0, v1, v2, v3], axis=1)
    return coords, cells


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output for the given draw counters of stream ``seed``."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed % (1 << 64)) + (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, n: int) -> np.ndarray:
    """``n`` doubles in [0, 1) from SplitMix64 stream ``seed``."""
    z = splitmix64(seed, np.arange(n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def initial_fractions(n_vertices: int, mean_p: float, mean_n: float,
                      amplitude: float = 0.01, seed: int = BASE_SEED):
    """Seeded initial volume fractions ``(phi_p, phi_n, phi_s)``.

    Each of the three components gets ``mean + U(-amplitude, amplitude)`` per
    vertex (draw ``3*v + c`` of the stream), then the three are divided by
    their sum so that they add up to one at every vertex.
    """
    mean_s = 1.0 - mean_p - mean_n
    u = uniform01(seed, 3 * n_vertices).reshape(n_vertices, 3)
    means = np.array([mean_p, mean_n, mean_s])
    raw = means[None, :] + amplitude * (2.0 * u - 1.0)
    raw = raw / raw.sum(axis=1, keepdims=True)
    return (np.ascontiguousarray(raw[:, 0]), np.ascontiguousarray(raw[:, 1]),
            np.ascontiguousarray(raw[:, 2]))


NET_LAYERS = ((8, 32), (32, 32), (32, 32), (32, 4))   # (c_in, c_out) of the 3x3 layers


def net_init(seed: int = BASE_SEED + 7, zero_last: bool = True, bias_scale: float = 0.0):
    """Seeded FP32 parameters [(w [3, 3, c_in, c_out], b [c_out]), ...] of the
    guess network: w uniform in +-sqrt(6 / (9 c_in)) (He-uniform), biases
    uniform in +-bias_scale; the last layer zero when ``zero_last``."""
    params = []
    for k, (ci, co) in enumerate(NET_LAYERS):
        u = uniform01(seed + 1000 * k, 9 * ci * co + co)
        a = np.sqrt(6.0 / (9 * ci))
        w = ((2.0 * u[:9 * ci * co] - 1.0) * a).reshape(3, 3, ci, co).astype(np.float32)
        b = ((2.0 * u[9 * ci * co:] - 1.0) * bias_scale).astype(np.float32)
        if zero_last and k == len(NET_LAYERS) - 1:
            w[:] = 0.0
            b[:] = 0.0
        params.append((w, b))
    return params


# Parameter presets.  Values the paper states (Section 4): chi_pn=1,
# chi_ps=chi_ns=0.3, N_p=N_n=20, N_s=1, eps=1e-3, tau between 1e-7 and 1e-4.
_COMMON = dict(
    tau=1e-4, eps=1e-3, mobility=1.0,
    potential="flory_huggins", Np=20.0, Nn=20.0, Ns=1.0,
    chi_pn=1.0, chi_ps=0.3, chi_ns=0.3, log_floor=1e-12,
    rtol=1e-8, restart=30, max_iters=300,
    amg_cycles=1, schur_pcg=3, smoother="chebyshev", cheb_degree=4, cheb_ratio=30.0,
    cheb_degree_mass=2, cheb_ratio_mass=4.0, coarse_max=256,
    max_levels=10,
)

PRESETS = {
    # 2D unit square, 32x32 squares, 5 steps, no evaporation.
    "square32": dict(_COMMON, dim=2, n=(32, 32), extent=(1.0, 1.0),
                     mean_p=0.1, mean_n=0.1, steps=5, evap_ds=0.0, evap_stop=0.0),
    # 2D unit square, 512x512 squares, 200 steps, solvent lowered linearly
    # from 0.8 to 0.3 (0.0025 per step).  Preconditioner settings measured
    # fastest per time step on this mesh: the mass block of Algorithm 1 is a
    # degree-5 Chebyshev semi-iteration (as accurate as the mass V-cycle here,
    # with no coarse levels); each As solve is 2 CG steps with V-cycles whose
    # degree-7 Chebyshev smoother covers [rho/5, rho] (degree 4 below the
    # finest level).
    "square512": dict(_COMMON, dim=2, n=(512, 512), extent=(1.0, 1.0), coarse_max=2048,
                      mean_p=0.1, mean_n=0.1, steps=200, evap_ds=0.0025, evap_stop=0.3,
                      mass_solver="chebyshev", cheb_degree_mass=5,
                      cheb_degree=7, cheb_ratio=5.0, schur_pcg=2, cheb_degree_coarse=4),
    # The paper's 2D experiment (Section 4): a 10 x 2.5 film (y is the height),
    # polynomial potential, phi_p = phi_n = 0.35 +- 0.01, solvent evaporation
    # through the top (k = 5e-3) and a patterned substrate at the bottom
    # (g_p = g_n = 0.01, h = 0, alternating sixths).
    "paper2d": dict(_COMMON, dim=2, n=(96, 24), extent=(10.0, 2.5), potential="polynomial",
                    mean_p=0.35, mean_n=0.35, steps=5, evap_ds=0.0, evap_stop=0.0,
                    boundary=1, bc_k=5e-3, bc_g=(0.01, 0.01), bc_h=(0.0, 0.0), bc_pattern=1),
    # 3D box of 96x96x48 cubes, Kuhn tetrahedra, 50 steps.  Measured fastest
    # per time step in a sweep of these settings: the mass block a degree-3
    # Chebyshev semi-iteration (the 3D mass matrix is well conditioned); each
    # As solve one CG step (a V-cycle with the optimal scaling) whose
    # smoother has degree 5 over [rho/20, rho] on the finest level and a
    # single step below it (the outer iteration count hardly depends on the
    # coarse levels' accuracy here).
    "box96": dict(_COMMON, dim=3, n=(96, 96, 48), extent=(1.0, 1.0, 0.5), coarse_max=2048,
                  mean_p=0.1, mean_n=0.1, steps=50, evap_ds=0.0, evap_stop=0.0,
                  mass_solver="chebyshev", cheb_degree_mass=3, schur_pcg=1,
                  cheb_degree=5, cheb_ratio=20.0, cheb_degree_coarse=1),
}


def preset(name: str, **overrides):
    """A copy of a preset with ``overrides`` applied."""
    p = dict(PRESETS[name])
    p.update(overrides)
    return p


def make_mesh(p: dict):
    """Mesh of a preset dict."""
    if p["dim"] == 2:
        return mesh_rect_2d(p["n"][0], p["n"][1], *p["extent"])
    return mesh_box_3d(p["n"][0], p["n"][1], p["n"][2], *p["extent"])
