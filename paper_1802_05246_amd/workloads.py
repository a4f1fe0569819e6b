"""Seeded synthetic inputs and exact solutions for the Hermite wave solvers.

This module holds none of the method's arithmetic.  It produces nodal data -- the
scaled Taylor coefficients ``h^l/l! d^l f`` of closed-form functions at the nodes
of the primal or dual grid (Sec. 2.1, Sec. 3.1.1 of the paper) -- and evaluates
exact solutions of ``u_tt = c^2 Lap u`` for error measurement.  Both the oracle
side and the GPU side are fed from here.

Layouts: node-major arrays ``(n_nodes, M**d)``, node index ``i0 + n0*(i1 + n1*i2)``,
coefficient index ``l0 + M*(l1 + M*l2)``.

Workload recipes (shapes, sizes and value distributions of the paper's runs; the
paper measures on no public dataset):
  * ``c1_1d``   -- 1-D periodic standing waves (dissipative, m=3, 64 cells)
  * ``c2_2d``   -- 2-D periodic Gaussian pulses (dissipative, m=3, 512^2)
  * ``c3_2d``   -- 2-D Dirichlet product of sine modes (conservative, m=4, 2048^2)
  * ``c4_3d``   -- 3-D periodic Gaussian pulses (dissipative, m=3, 256^3)
  * ``c5_batch``-- 256 independent 2-D problems of uneven N, m, c, method, walls
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np

PERIODIC, DIRICHLET, NEUMANN = 0, 1, 2
DISS_FULL, DISS_SIMPLE, CONSERVATIVE = 0, 1, 2
PRIMAL, DUAL = 0, 1


@dataclasses.dataclass
class Spec:
    """Problem statement (Sec. 2.1, Sec. 3): dimension, degree, grid, speed, step,
    walls, method."""
    d: int
    m: int
    n: Sequence[int]
    xl: Sequence[float]
    xr: Sequence[float]
    c: float
    dt: float
    bc: Sequence[int]
    method: int = DISS_FULL
    taylor_stages: int = 0

    def h(self, i: int) -> float:
        return (self.xr[i] - self.xl[i]) / self.n[i]

    def extent(self, grid: int, i: int) -> int:
        if self.bc[i] == PERIODIC:
            return int(self.n[i])
        return int(self.n[i]) + 1 if grid == PRIMAL else int(self.n[i])

    def nodes(self, grid: int) -> int:
        return int(np.prod([self.extent(grid, i) for i in range(self.d)]))

    def coords(self, grid: int, i: int) -> np.ndarray:
        off = 0.0 if grid == PRIMAL else 0.5
        return self.xl[i] + (np.arange(self.extent(grid, i)) + off) * self.h(i)

    def points(self, grid: int) -> np.ndarray:
        """(n_nodes, d) coordinates in node order (x fastest)."""
        axes = [self.coords(grid, i) for i in range(self.d)]
        mesh = np.meshgrid(*axes, indexing="ij")
        return np.stack([g.transpose(tuple(range(self.d))[::-1]).reshape(-1)
                         for g in mesh], axis=1)

    def lam(self) -> float:
        return self.c * self.dt / min(self.h(i) for i in range(self.d))


def make_spec(d, m, n, xl=0.0, xr=1.0, c=1.0, cfl=None, dt=None, bc=PERIODIC,
              method=DISS_FULL, taylor_stages=0) -> Spec:
    def vec(v):
        return list(v) if isinstance(v, (list, tuple, np.ndarray)) else [v] * d
    n_, xl_, xr_, bc_ = vec(n), vec(xl), vec(xr), vec(bc)
    hmin = min((xr_[i] - xl_[i]) / n_[i] for i in range(d))
    if dt is None:
        dt = cfl * hmin / c
    return Spec(d, m, [int(x) for x in n_], [float(x) for x in xl_], [float(x) for x in xr_],
                float(c), float(dt), [int(x) for x in bc_], method, taylor_stages)


# ----------------------------------------------------------------------------
# scaled derivatives of 1-D closed-form factors: table D[l, j] = h^l/l! f^(l)(x_j)
# ----------------------------------------------------------------------------
def _scale(L: int, h: float) -> np.ndarray:
    return np.array([h ** l / math.factorial(l) for l in range(L + 1)])


def sine_derivs(x, k, phase, L, h):
    """f = sin(k x + phase); f^(l) = k^l sin(k x + phase + l pi/2)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.stack([k ** l * np.sin(k * x + phase + l * np.pi / 2) for l in range(L + 1)])
    return out * _scale(L, h)[:, None]


def gaussian_derivs(x, x0, sigma, L, h, period=None):
    """f = exp(-(x-x0)^2/(2 sigma^2)), with the minimum-image displacement when a
    period is given.  With z = (x-x0)/(sigma sqrt 2): f^(l) = (-1)^l (sigma sqrt2)^-l
    Hphys_l(z) exp(-z^2) (physicists' Hermite polynomials)."""
    x = np.asarray(x, dtype=np.float64)
    dx = x - x0
    if period is not None:
        dx = dx - period * np.round(dx / period)
    s2 = sigma * math.sqrt(2.0)
    z = dx / s2
    e = np.exp(-z * z)
    Hm1, H0 = np.zeros_like(z), np.ones_like(z)
    out = []
    for l in range(L + 1):
        out.append((-1.0 / s2) ** l * H0 * e)
        Hm1, H0 = H0, 2.0 * z * H0 - 2.0 * l * Hm1
    return np.stack(out) * _scale(L, h)[:, None]


def poly_derivs(coeffs, x, L, h):
    """f = sum_j coeffs[j] x^j (numpy polynomial order)."""
    P = np.polynomial.Polynomial(coeffs)
    out = []
    for l in range(L + 1):
        out.append(P.deriv(l)(np.asarray(x, dtype=np.float64)) if l <= P.degree() + 1
                   else np.zeros_like(np.asarray(x, dtype=np.float64)))
    return np.stack(out) * _scale(L, h)[:, None]


def tensor_nodal(tables: Sequence[np.ndarray], M: int, device=None):
    """Combine per-dimension tables D_i[l_i, j_i] (l_i < M) into the node-major array
    prod_i D_i[l_i, j_i] with x fastest in both node and coefficient index.  With a
    torch `device` the product is formed there (returns a float64 tensor)."""
    d = len(tables)
    if device is not None:
        import torch
        T = [torch.as_tensor(np.asarray(t)[:M], dtype=torch.float64, device=device) for t in tables]
        ein = torch.einsum
    else:
        T = [np.asarray(t)[:M] for t in tables]
        ein = np.einsum
    if d == 1:
        return T[0].T.contiguous() if device is not None else T[0].T.copy()
    if d == 2:
        a = ein("aj,bk->kjba", T[0], T[1])  # (j1, j0, l1, l0)
    else:
        a = ein("aj,bk,cl->lkjcba", T[0], T[1], T[2])
    n_nodes = int(np.prod([t.shape[1] for t in T]))
    if device is not None:
        return a.reshape(n_nodes, M ** d).contiguous()
    return np.ascontiguousarray(a.reshape(n_nodes, M ** d))


def separable_nodal(spec: Spec, grid: int, M: int, factors: List[Callable], device=None):
    """sum over terms of prod_i f_i(x_i): `factors` is a list of terms, each a
    callable (dim, x, L, h) -> table."""
    total = None
    for term in factors:
        tabs = [term(i, spec.coords(grid, i), M - 1, spec.h(i)) for i in range(spec.d)]
        a = tensor_nodal(tabs, M, device)
        if total is None:
            total = a
        else:
            total += a
            del a
    return total


def plane_wave_nodal(spec: Spec, grid: int, M: int, kvec, phase, amp=1.0) -> np.ndarray:
    """f = amp sin(k.x + phase): d^l f = amp prod k_i^l_i sin(k.x + phase + |l| pi/2)."""
    pts = spec.points(grid)
    arg = pts @ np.asarray(kvec, dtype=np.float64) + phase
    d = spec.d
    out = np.zeros((pts.shape[0], M ** d))
    for cidx in range(M ** d):
        ls = [(cidx // M ** i) % M for i in range(d)]
        s = amp * np.sin(arg + sum(ls) * np.pi / 2)
        for i, l in enumerate(ls):
            s = s * (kvec[i] ** l) * spec.h(i) ** l / math.factorial(l)
        out[:, cidx] = s
    return out


def pulses_nodal(spec: Spec, grid: int, M: int, centres, amps, sigma, device=None):
    """Sum of Gaussian pulses A exp(-|x-x_p|^2/(2 sigma^2)) (minimum image per
    dimension on periodic domains)."""
    terms = []
    for x0, A in zip(centres, amps):
        def term(i, x, L, h, x0=x0, A=A):
            per = (spec.xr[i] - spec.xl[i]) if spec.bc[i] == PERIODIC else None
            t = gaussian_derivs(x, x0[i], sigma, L, h, per)
            return t * A if i == 0 else t
        terms.append(term)
    return separable_nodal(spec, grid, M, terms, device)


# ----------------------------------------------------------------------------
# exact solutions
# ----------------------------------------------------------------------------
def radial_pulses_exact(points, t, centres, amps, sigma, c, period=1.0, images=2, xp=np):
    """Exact solution in 3-D for Gaussian pulse data with zero velocity:
    u = sum_p sum_images A [phi(ct + r) - phi(ct - r)]/(2r), phi(s) = s g(s),
    g(s) = exp(-s^2/(2 sigma^2)); r -> 0 limit A g(ct)(1 - (ct)^2/sigma^2).
    `points` is (N, 3) in the namespace `xp` (numpy or torch)."""
    ct = c * t
    out = xp.zeros_like(points[:, 0])

    def g(s):
        return xp.exp(-s * s / (2.0 * sigma * sigma))

    rng = range(-images, images + 1)
    for x0, A in zip(centres, amps):
        for a in rng:
            for b in rng:
                for e in rng:
                    dx = points[:, 0] - (x0[0] + a * period)
                    dy = points[:, 1] - (x0[1] + b * period)
                    dz = points[:, 2] - (x0[2] + e * period)
                    r = xp.sqrt(dx * dx + dy * dy + dz * dz)
                    if float(r.min()) > ct + 12 * sigma:
                        continue
                    rs = xp.where(r > 1e-7, r, xp.ones_like(r))
                    val = ((ct + rs) * g(ct + rs) - (ct - rs) * g(ct - rs)) / (2 * rs)
                    lim = g(xp.zeros_like(r) + ct) * (1.0 - ct * ct / (sigma * sigma))
                    out = out + A * xp.where(r > 1e-7, val, lim)
    return out


def nodal_l2(spec: Spec, values, exact) -> float:
    """(prod_i h_i sum_nodes (u - u_exact)^2)^(1/2) on the value coefficient."""
    hprod = float(np.prod([spec.h(i) for i in range(spec.d)]))
    diff = np.asarray(values, dtype=np.float64) - np.asarray(exact, dtype=np.float64)
    return math.sqrt(hprod * float(np.sum(diff * diff)))


# ----------------------------------------------------------------------------
# workload recipes (seed 1802 + k)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    spec: Spec
    steps: int
    u0: np.ndarray                      # primal data at t0
    v0: Optional[np.ndarray]            # primal velocity data (dissipative) or None
    u_half: Optional[np.ndarray] = None # dual data at t0 + dt/2 (conservative)
    exact: Optional[Callable] = None    # exact(t, grid) -> value coefficient per node
    meta: dict = dataclasses.field(default_factory=dict)


def c1_1d(n=64, m=3, cfl=0.9, t_final=1.0, seed=1803) -> Workload:
    """1-D dissipative, periodic [0,1], u0 = sum_k a_k sin(2 pi k x), v0 = 0."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=3)
    spec = make_spec(1, m, n, 0.0, 1.0, 1.0, cfl=cfl, bc=PERIODIC, method=DISS_FULL)
    steps = int(round(t_final / spec.dt))
    terms = []
    for k in range(1, 4):
        terms.append(lambda i, x, L, h, k=k: a[k - 1] * sine_derivs(x, 2 * np.pi * k, 0.0, L, h))
    u0 = separable_nodal(spec, PRIMAL, m + 1, terms)
    v0 = np.zeros((spec.nodes(PRIMAL), m ** 1))

    def exact(t, grid=PRIMAL):
        x = spec.coords(grid, 0)
        return sum(a[k - 1] * np.sin(2 * np.pi * k * x) * np.cos(2 * np.pi * k * spec.c * t)
                   for k in range(1, 4))
    return Workload("c1_1d", spec, steps, u0, v0, exact=exact, meta={"a": a.tolist()})


def _pulse_draw(rng, count, d):
    centres, amps = [], []
    for _ in range(count):
        centres.append(rng.uniform(0.0, 1.0, size=d))
        amps.append(float(rng.uniform(0.5, 1.0)))
    return centres, amps


def c2_2d(n=512, m=3, cfl=0.9, steps=1000, seed=1804) -> Workload:
    """2-D dissipative, periodic unit square, 4 Gaussian pulses (sigma 0.05), v0 = 0."""
    rng = np.random.default_rng(seed)
    centres, amps = _pulse_draw(rng, 4, 2)
    spec = make_spec(2, m, n, 0.0, 1.0, 1.0, cfl=cfl, bc=PERIODIC, method=DISS_FULL)
    u0 = pulses_nodal(spec, PRIMAL, m + 1, centres, amps, 0.05)
    v0 = np.zeros((spec.nodes(PRIMAL), m ** 2))
    return Workload("c2_2d", spec, steps, u0, v0,
                    meta={"centres": [c.tolist() for c in centres], "amps": amps, "sigma": 0.05})


def c3_2d(n=2048, m=4, cfl=1.0, steps=2000, seed=1805) -> Workload:
    """2-D conservative, Dirichlet unit square, u = sin(pi k1 x) sin(pi k2 y)
    cos(c pi |k| t); both time levels from the exact solution."""
    rng = np.random.default_rng(seed)
    k1, k2 = (int(v) for v in rng.integers(1, 9, size=2))
    spec = make_spec(2, m, n, 0.0, 1.0, 1.0, cfl=cfl, bc=DIRICHLET, method=CONSERVATIVE)
    om = spec.c * np.pi * math.hypot(k1, k2)

    def level(grid, t):
        terms = [lambda i, x, L, h: (sine_derivs(x, np.pi * (k1 if i == 0 else k2), 0.0, L, h)
                                     * (math.cos(om * t) if i == 0 else 1.0))]
        return separable_nodal(spec, grid, m + 1, terms)
    u0 = level(PRIMAL, 0.0)
    uh = level(DUAL, 0.5 * spec.dt)

    def exact(t, grid=PRIMAL):
        pts = spec.points(grid)
        return np.sin(np.pi * k1 * pts[:, 0]) * np.sin(np.pi * k2 * pts[:, 1]) * math.cos(om * t)
    return Workload("c3_2d", spec, steps, u0, None, u_half=uh, exact=exact,
                    meta={"k1": k1, "k2": k2, "level": level})


def c4_3d(n=256, m=3, cfl=0.9, steps=200, seed=1806, sigma=0.05, device=None) -> Workload:
    """3-D dissipative, periodic unit cube, 8 Gaussian pulses (sigma 0.05), v0 = 0.
    With a torch `device` the nodal arrays are built there."""
    rng = np.random.default_rng(seed)
    centres, amps = _pulse_draw(rng, 8, 3)
    spec = make_spec(3, m, n, 0.0, 1.0, 1.0, cfl=cfl, bc=PERIODIC, method=DISS_FULL)
    u0 = pulses_nodal(spec, PRIMAL, m + 1, centres, amps, sigma, device)
    if device is not None:
        import torch
        v0 = torch.zeros((spec.nodes(PRIMAL), m ** 3), dtype=torch.float64, device=device)
    else:
        v0 = np.zeros((spec.nodes(PRIMAL), m ** 3))

    def exact(t, grid=PRIMAL, points=None, xp=np):
        pts = spec.points(grid) if points is None else points
        return radial_pulses_exact(pts, t, centres, amps, sigma, spec.c, xp=xp)
    return Workload("c4_3d", spec, steps, u0, v0, exact=exact,
                    meta={"centres": [c.tolist() for c in centres], "amps": amps, "sigma": sigma})


def c5_batch(count=256, steps=500, seed=1807, cfl=0.8, n_lo=64, n_hi=1024, device=None) -> List[Workload]:
    """Independent 2-D problems: per problem N ~ round(exp U(ln n_lo, ln n_hi)),
    m ~ U{2..6}, c ~ U(0.5, 2), method ~ {dissipative full, conservative},
    walls ~ {Dirichlet, Neumann, periodic}, 4 pulses (centre, amplitude); v0 = 0.
    The conservative second level comes from the start-up step (v0 = 0).  With a
    torch `device` the initial data is built there."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        N = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        m = int(rng.integers(2, 7))
        c = float(rng.uniform(0.5, 2.0))
        method = [DISS_FULL, CONSERVATIVE][int(rng.integers(0, 2))]
        bc = [DIRICHLET, NEUMANN, PERIODIC][int(rng.integers(0, 3))]
        centres, amps = _pulse_draw(rng, 4, 2)
        spec = make_spec(2, m, N, 0.0, 1.0, c, cfl=cfl, bc=bc, method=method)
        sigma = 0.05
        u0 = pulses_nodal(spec, PRIMAL, m + 1, centres, amps, sigma, device=device)
        if method == CONSERVATIVE:
            v0 = None
        elif device is not None:
            import torch
            v0 = torch.zeros((spec.nodes(PRIMAL), m ** 2), dtype=torch.float64, device=device)
        else:
            v0 = np.zeros((spec.nodes(PRIMAL), m ** 2))
        out.append(Workload(f"c5_{b}", spec, steps, u0, v0,
                            meta={"centres": [x.tolist() for x in centres], "amps": amps}))
    return out


def random_state(spec: Spec, seed: int, grid: int = PRIMAL, lo=-1.0, hi=1.0):
    """Random nodal coefficients (u, v) for stability and parity tests."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(lo, hi, size=(spec.nodes(grid), (spec.m + 1) ** spec.d))
    v = rng.uniform(lo, hi, size=(spec.nodes(grid), max(spec.m, 1) ** spec.d))
    return u, v
