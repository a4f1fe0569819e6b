"""Convergence orders and stability of the oracle (Sec. 3.4 eqs. (utrunc),(vtrunc),
Sec. 4.4 eq. (Ctrunc), Sec. 5.1, Sec. 5.3).

Errors are nodal L2 errors of the value coefficient against exact solutions; rates
are measured between the finest refinements of each run (asymptotic regime).
"""
import math

import numpy as np
import pytest

import oracle
from paper_1802_05246_amd import workloads as W
from helpers import oracle_growth_per_step


def _P(spec):
    return oracle.make_problem(spec.d, spec.m, spec.n, spec.xl, spec.xr, spec.c, spec.dt,
                               spec.bc, spec.method, spec.taylor_stages)


def _rate(ns, errs):
    return math.log(errs[-2] / errs[-1]) / math.log(ns[-1] / ns[-2])


def _gauss_box_exact(x, t):
    """e^{-20x^2} in the Dirichlet box [-3/2, 3/2] (Sec. 5.1): d'Alembert on the
    odd 6-periodic extension."""
    def f(s):
        s = (s + 1.5) % 6.0 - 1.5
        return np.where(s < 1.5, np.exp(-20 * s * s), -np.exp(-20 * (3.0 - s) ** 2))
    return 0.5 * (f(x + t) + f(x - t))


def _run_gauss_box(m, n, cfl, method, T=2.0):
    spec = W.make_spec(1, m, n, -1.5, 1.5, 1.0, cfl=cfl, bc=W.DIRICHLET, method=method)
    steps = int(round(T / spec.dt))
    g = [lambda i, x, L, h: W.gaussian_derivs(x, 0.0, 1 / math.sqrt(40), L, h)]
    u0 = W.separable_nodal(spec, W.PRIMAL, m + 1, g)
    p = _P(spec)
    if method == W.CONSERVATIVE:
        u, _ = oracle.cons_advance(p, u0, oracle.cons_startup(p, u0, None), steps)
    else:
        u, _ = oracle.diss_advance(p, u0, np.zeros((n + 1, m)), steps)
    return W.nodal_l2(spec, u[:, 0], _gauss_box_exact(spec.coords(W.PRIMAL, 0), steps * spec.dt))


@pytest.mark.parametrize("m,cfl,expect,ns", [
    (2, 0.8, 3.0, [29, 35, 42]), (2, 1.0, 4.0, [29, 35, 42]), (3, 1.0, 6.0, [29, 35, 42])])
def test_diss_gaussian_box_rates(m, cfl, expect, ns):
    """Sec. 5.1: dissipative rates 2m-1 (lambda = 0.8) and 2m (lambda = 1) with
    homogeneous Dirichlet walls through the odd ghost extension."""
    errs = [_run_gauss_box(m, n, cfl, W.DISS_FULL) for n in ns]
    assert abs(_rate(ns, errs) - expect) < 0.3, errs


def test_cons_gaussian_box_rate():
    """Sec. 5.1: conservative rate 2m at lambda = 0.8 (m = 1)."""
    ns = [56, 80, 112]
    errs = [_run_gauss_box(1, n, 0.8, W.CONSERVATIVE) for n in ns]
    assert abs(_rate(ns, errs) - 2.0) < 0.3, errs


def test_cons_gaussian_box_exact_at_cfl_one():
    """At c dt = h the 1-D conservative update is d'Alembert's formula, so the
    error is round-off (start-up and steps both exact)."""
    for m in (1, 2):
        assert _run_gauss_box(m, 24, 1.0, W.CONSERVATIVE) < 1e-13


def _run_plane_wave(m, n, cfl, method, T=0.5):
    """Sec. 5.3: u = sin(2 pi kappa (x + y + sqrt2 t)), kappa = m+1, periodic square."""
    kap = m + 1
    spec = W.make_spec(2, m, n, 0.0, 1.0, 1.0, cfl=cfl, bc=W.PERIODIC, method=method)
    steps = int(round(T / spec.dt))
    k = 2 * np.pi * kap
    om = k * math.sqrt(2)
    u0 = W.plane_wave_nodal(spec, W.PRIMAL, m + 1, [k, k], 0.0)
    p = _P(spec)
    if method == W.CONSERVATIVE:
        uh = W.plane_wave_nodal(spec, W.DUAL, m + 1, [k, k], om * 0.5 * spec.dt)
        u, _ = oracle.cons_advance(p, u0, uh, steps)
    else:
        v0 = W.plane_wave_nodal(spec, W.PRIMAL, m, [k, k], math.pi / 2, amp=om)
        u, _ = oracle.diss_advance(p, u0, v0, steps)
    pts = spec.points(W.PRIMAL)
    ex = np.sin(k * (pts[:, 0] + pts[:, 1]) + om * steps * spec.dt)
    return W.nodal_l2(spec, u[:, 0], ex)


@pytest.mark.parametrize("method,m,cfl,expect", [
    (W.DISS_FULL, 2, 1.0, 4.0), (W.DISS_FULL, 3, 1.0, 6.0),
    (W.CONSERVATIVE, 1, 1.0, 4.0), (W.CONSERVATIVE, 2, 1.0, 6.0)])
def test_plane_wave_rates_2d(method, m, cfl, expect):
    """Sec. 5.3: 2-D rates 2m (dissipative) and 2m+2 (conservative) at lambda = 1."""
    ns = [12, 16, 20]
    errs = [_run_plane_wave(m, n, cfl, method) for n in ns]
    assert abs(_rate(ns, errs) - expect) < 0.3, errs


def test_plane_wave_dissipative_lambda08_at_least_2m_minus_1():
    """Sec. 3.4 prediction i: order 2m-1 for lambda < 1 (pre-asymptotic runs show
    a higher slope; the rate never drops below 2m-1)."""
    ns = [12, 16, 20]
    errs = [_run_plane_wave(2, n, 0.8, W.DISS_FULL) for n in ns]
    assert _rate(ns, errs) > 3.0 - 0.3, errs


@pytest.mark.parametrize("m", [2, 3])
def test_standing_wave_1d_rate(m):
    """The 1-D periodic standing-wave workload (u0 = sum a_k sin 2 pi k x, v0 = 0):
    order 2m-1 at lambda = 0.8."""
    def err(n):
        w = W.c1_1d(n=n, m=m, cfl=0.8)
        p = _P(w.spec)
        u, _ = oracle.diss_advance(p, w.u0, w.v0, w.steps)
        return W.nodal_l2(w.spec, u[:, 0], w.exact(w.steps * w.spec.dt))
    ns = [48, 64, 96]
    errs = [err(n) for n in ns]
    assert abs(_rate(ns, errs) - (2 * m - 1)) < 0.3, errs


@pytest.mark.parametrize("method,m,d,cfl", [(W.DISS_FULL, 3, 2, 1.0), (W.DISS_SIMPLE, 3, 2, 1.0),
                                            (W.DISS_FULL, 2, 3, 1.0), (W.CONSERVATIVE, 3, 2, 1.0)])
def test_stable_at_cfl_one(method, m, d, cfl):
    """Sec. 1 / Sec. 3.3: stable for c dt <= h.  Random zero-velocity data on a
    small periodic grid: the coefficient amplitude reached after the first block of
    steps is not exceeded (beyond a factor 3) over the following blocks."""
    n = [6, 6, 4][:d]
    spec = W.make_spec(d, m, n, 0.0, 1.0, 1.0, cfl=cfl, bc=W.PERIODIC, method=method)
    p = _P(spec)
    u, v = W.random_state(spec, 3)
    block = 50 if d == 2 else 15
    amps = []
    if method == W.CONSERVATIVE:
        ud = oracle.cons_startup(p, u, None)
        for _ in range(4):
            u, ud = oracle.cons_advance(p, u, ud, block)
            amps.append(np.abs(u).max())
    else:
        v = np.zeros_like(v)
        for _ in range(4):
            u, v = oracle.diss_advance(p, u, v, block)
            amps.append(np.abs(u).max())
    assert np.isfinite(amps).all() and max(amps[1:]) < 3 * amps[0], amps


# ---- stability of the variants (Sec. 3.3, Sec. 6.1), measured on the oracle --------------
def test_full_exact_series_m5_unstable_at_cfl_one():
    """The modified-first-step variant with the exact series has a growing mode for
    m = 5 at c dt = h (while m <= 3 decays)."""
    assert oracle_growth_per_step(2, 5, 1.0, W.DISS_FULL) > 1.0 + 1e-3
    assert oracle_growth_per_step(2, 3, 1.0, W.DISS_FULL) < 1.0 + 1e-4


def test_simple_variant_truncated_series_unstable():
    """Cutting the Taylor series of the straightforward variant after stage 2m+1
    (2m+2 terms with s = 0) makes m = 3 unstable at lambda = 0.8; the exact series and
    the cut after stage 2m+2 stay stable."""
    assert oracle_growth_per_step(2, 3, 0.8, W.DISS_SIMPLE, taylor_stages=7, n=12) > 1.1
    assert oracle_growth_per_step(2, 3, 0.8, W.DISS_SIMPLE, taylor_stages=8, n=12) < 1.0 + 1e-4
    assert oracle_growth_per_step(2, 3, 0.8, W.DISS_SIMPLE, taylor_stages=0, n=12) < 1.0 + 1e-4
