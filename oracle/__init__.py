"""FP64 CPU oracle for the Hermite wave-equation methods — TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (built from
``hermite_oracle.c`` by :func:`build`) with numpy arrays and shares nothing with the
GPU library.

Array conventions: node-major arrays of shape ``(n_nodes, M**d)`` with the node
index ``i0 + n0*(i1 + n1*i2)`` and the coefficient index ``l0 + M*(l1 + M*l2)``;
``M = m+1`` for u and ``m`` for v.  Values are scaled Taylor coefficients
``h^l/l! d^l f`` (Sec. 2.2 of the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

PERIODIC, DIRICHLET, NEUMANN = 0, 1, 2
DISS_FULL, DISS_SIMPLE, CONSERVATIVE = 0, 1, 2
PRIMAL, DUAL = 0, 1


def build() -> str:
    """Compile liboracle.so with gcc (FP64, OpenMP)."""
    src = os.path.join(_HERE, "hermite_oracle.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-o", tmp, src, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("m", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("xl", ctypes.c_double * 3), ("xr", ctypes.c_double * 3),
                ("c", ctypes.c_double), ("dt", ctypes.c_double), ("bc", ctypes.c_int * 3),
                ("method", ctypes.c_int), ("taylor_stages", ctypes.c_int)]


def make_problem(d, m, n, xl, xr, c, dt, bc, method, taylor_stages=0) -> Problem:
    def three(v, fill):
        v = list(v) if isinstance(v, (list, tuple)) else [v] * d
        return v + [fill] * (3 - len(v))
    p = Problem()
    p.d, p.m = d, m
    p.n[:] = [int(x) for x in three(n, 1)]
    p.xl[:] = [float(x) for x in three(xl, 0.0)]
    p.xr[:] = [float(x) for x in three(xr, 1.0)]
    p.c, p.dt = float(c), float(dt)
    p.bc[:] = [int(x) for x in three(bc, PERIODIC)]
    p.method = int(method)
    p.taylor_stages = int(taylor_stages)
    return p


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int64)
        pp = ctypes.POINTER(Problem)
        L.hwo_hermite_matrix.argtypes = [ctypes.c_int, dp]
        L.hwo_nodes.argtypes = [pp, ctypes.c_int]
        L.hwo_nodes.restype = ctypes.c_int64
        L.hwo_diss_half.argtypes = [pp, ctypes.c_int, dp, dp, dp, dp, ip, ctypes.c_int64, ctypes.c_int]
        L.hwo_diss_half_forced.argtypes = [pp, ctypes.c_int, dp, dp, dp, ctypes.c_int, dp, dp, ip,
                                           ctypes.c_int64, ctypes.c_int]
        L.hwo_cons_half.argtypes = [pp, ctypes.c_int, dp, dp, dp, ip, ctypes.c_int64, ctypes.c_int]
        L.hwo_diss_half_ext.argtypes = [pp, ctypes.c_int, dp, dp, dp, ctypes.c_int, dp, dp, dp, dp, ip,
                                        ctypes.c_int64, ctypes.c_int]
        L.hwo_cons_half_ext.argtypes = [pp, ctypes.c_int, dp, dp, dp, ctypes.c_int, dp, dp, ip,
                                        ctypes.c_int64, ctypes.c_int]
        L.hwo_cons_startup.argtypes = [pp, dp, dp, dp, ctypes.c_int]
        L.hwo_cons_energy.argtypes = [pp, ctypes.c_int, dp, dp, dp, ctypes.c_int]
        L.hwo_cons_energy.restype = ctypes.c_double
        L.hwo_seminorm.argtypes = [pp, ctypes.c_int, dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.hwo_seminorm.restype = ctypes.c_double
        L.hwo_diss_energy.argtypes = [pp, ctypes.c_int, dp, dp, ctypes.c_int]
        L.hwo_diss_energy.restype = ctypes.c_double
        _lib = L
    return _lib


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def hermite_matrix(m: int) -> np.ndarray:
    """H_m of Sec. 2.2: maps [left l=0..m, right l=0..m] to the 2m+2 monomial
    coefficients about the cell centre in z = (x - x_c)/h."""
    P = 2 * m + 2
    H = np.zeros((P, P))
    rc = lib().hwo_hermite_matrix(m, _dp(H))
    if rc:
        raise ValueError(f"hermite_matrix failed ({rc})")
    return H


def nodes(p: Problem, grid: int) -> int:
    return int(lib().hwo_nodes(ctypes.byref(p), grid))


def _sel(sel):
    if sel is None:
        return None, 0
    s = np.ascontiguousarray(sel, dtype=np.int64)
    return s, s.size


def wall_faces(p: Problem):
    """The faces of the wall records, in their order: (dim, side, tangential extents)
    for every non-periodic dimension (side -1 = low wall, +1 = high wall).  The
    tangential extents are those of the input (dual) grid of a half step onto the
    primal grid, with one ghost position added at each end of a non-periodic
    dimension (index 0 = beyond the low wall, n + 1 = beyond the high wall)."""
    faces = []
    for i in range(p.d):
        if p.bc[i] == PERIODIC:
            continue
        ext = [p.n[t] + (0 if p.bc[t] == PERIODIC else 2) for t in range(p.d) if t != i]
        faces.append((i, -1, ext))
        faces.append((i, 1, ext))
    return faces


def wall_points(p: Problem) -> int:
    return int(sum(int(np.prod(e)) if e else 1 for _, _, e in wall_faces(p)))


def _walls(p, walls, M):
    w = np.ascontiguousarray(walls, dtype=np.float64)
    if w.shape != (wall_points(p), M ** p.d):
        raise ValueError(f"wall records must have shape {(wall_points(p), M ** p.d)}, got {w.shape}")
    return w


def diss_half(p: Problem, to_grid: int, u, v, sel=None, nthreads=0, forcing=None, walls=None):
    """One dissipative half step onto `to_grid` (Sec. 3.1.2, Sec. 3.3).  With `sel`
    only those output nodes are computed (rows in the order given).  `forcing`, if
    given, has shape (nodes of to_grid, R, (2m)^d): the scaled space-time Taylor
    coefficients h^k/k! d^k d^r/dt^r f of the forcing at every output node and the
    start of the half step, r < R (Sec. 3.1.2 eq. (recursion_diss_1d_2)).  `walls`, if
    given, is (wall_u, wall_v): the inhomogeneous / time-dependent wall data of
    Sec. 3.1.3, records of shape (wall_points, (m+1)^d) and (wall_points, m^d) (layout in
    hermite_oracle.c), used when to_grid is the primal grid."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    s, ns = _sel(sel)
    cnt = ns if s is not None else nodes(p, to_grid)
    uo = np.zeros((cnt, (p.m + 1) ** p.d))
    vo = np.zeros((cnt, p.m ** p.d))
    selp = None if s is None else s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    f, nf = None, 0
    if forcing is not None:
        f = np.ascontiguousarray(forcing, dtype=np.float64)
        if f.ndim != 3 or f.shape[0] != nodes(p, to_grid) or f.shape[2] != (2 * p.m) ** p.d:
            raise ValueError(f"forcing must have shape (nodes, R, (2m)^d), got {f.shape}")
        nf = f.shape[1]
    wu = wv = None
    if walls is not None:
        wu, wv = _walls(p, walls[0], p.m + 1), _walls(p, walls[1], p.m)
    rc = lib().hwo_diss_half_ext(ctypes.byref(p), to_grid, _dp(u), _dp(v), _dp(f), nf, _dp(wu), _dp(wv),
                                 _dp(uo), _dp(vo), selp, ns, nthreads)
    if rc:
        raise ValueError(f"diss_half failed ({rc})")
    return uo, vo


def cons_half(p: Problem, to_grid: int, u_from, u_old, sel=None, nthreads=0, forcing=None, walls=None):
    """One conservative half step (Sec. 4.1 eq. (convUpdate), Sec. 4.3): new data on
    `to_grid` from the other grid's data at the middle time and the old data.
    `forcing`: shape (nodes of to_grid, R, (2m+2)^d), the scaled Taylor coefficients
    h^k/k! d^k d^q/dt^q f at every output node and the middle time (eq. (wavequ));
    `walls`: wall records of shape (wall_points, (m+1)^d) (Sec. 3.1.3), used when
    to_grid is the primal grid."""
    u_from = np.ascontiguousarray(u_from, dtype=np.float64)
    u_old = np.ascontiguousarray(u_old, dtype=np.float64)
    s, ns = _sel(sel)
    cnt = ns if s is not None else nodes(p, to_grid)
    un = np.zeros((cnt, (p.m + 1) ** p.d))
    f, nf = None, 0
    if forcing is not None:
        f = np.ascontiguousarray(forcing, dtype=np.float64)
        if f.ndim != 3 or f.shape[0] != nodes(p, to_grid) or f.shape[2] != (2 * p.m + 2) ** p.d:
            raise ValueError(f"forcing must have shape (nodes, R, (2m+2)^d), got {f.shape}")
        nf = f.shape[1]
    wu = _walls(p, walls, p.m + 1) if walls is not None else None
    selp = None if s is None else s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rc = lib().hwo_cons_half_ext(ctypes.byref(p), to_grid, _dp(u_from), _dp(u_old), _dp(f), nf, _dp(wu),
                                 _dp(un), selp, ns, nthreads)
    if rc:
        raise ValueError(f"cons_half failed ({rc})")
    return un


def cons_startup(p: Problem, u0, v0=None, nthreads=0):
    """Dual-grid data at t0 + dt/2 from primal u0, v0 (exact Taylor evolution of the
    degree-m cell interpolants)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    v0 = None if v0 is None else np.ascontiguousarray(v0, dtype=np.float64)
    out = np.zeros((nodes(p, DUAL), (p.m + 1) ** p.d))
    rc = lib().hwo_cons_startup(ctypes.byref(p), _dp(u0), _dp(v0), _dp(out), nthreads)
    if rc:
        raise ValueError(f"cons_startup failed ({rc})")
    return out


def cons_energy(p: Problem, grid_a: int, u_a, u_b_new, u_b_old, nthreads=0) -> float:
    """2(|p_A|^2 - <p_B^new, p_B^old>) in the |.|_{m+1} seminorm (equals
    |P+|^2 + |P-|^2 of Sec. 5.2 in 1-D)."""
    args = [np.ascontiguousarray(a, dtype=np.float64) for a in (u_a, u_b_new, u_b_old)]
    return float(lib().hwo_cons_energy(ctypes.byref(p), grid_a, *[_dp(a) for a in args], nthreads))


def seminorm(p: Problem, data_grid: int, f, g, mdata: int, q: int, nthreads=0) -> float:
    f = np.ascontiguousarray(f, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    return float(lib().hwo_seminorm(ctypes.byref(p), data_grid, _dp(f), _dp(g), mdata, q, nthreads))


def diss_energy(p: Problem, data_grid: int, u, v, nthreads=0) -> float:
    """c^2 |I_m u|^2_{m+1} + |I_{m-1} v|^2_m (1-D, Sec. 3.2 eq. (stable1))."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    return float(lib().hwo_diss_energy(ctypes.byref(p), data_grid, _dp(u), _dp(v), nthreads))


def diss_advance(p: Problem, u, v, n_full_steps: int, nthreads=0):
    """n full dissipative steps from primal data (two half steps each)."""
    for _ in range(n_full_steps):
        u, v = diss_half(p, DUAL, u, v, nthreads=nthreads)
        u, v = diss_half(p, PRIMAL, u, v, nthreads=nthreads)
    return u, v


def cons_advance(p: Problem, u_primal, u_dual, n_full_steps: int, nthreads=0):
    """n full conservative steps from primal at t and dual at t + dt/2: update the
    primal grid using the dual, then the dual grid using the new primal."""
    for _ in range(n_full_steps):
        u_primal = cons_half(p, PRIMAL, u_dual, u_primal, nthreads=nthreads)
        u_dual = cons_half(p, DUAL, u_primal, u_dual, nthreads=nthreads)
    return u_primal, u_dual
