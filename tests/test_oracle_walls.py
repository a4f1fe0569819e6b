"""Pins of the oracle's inhomogeneous / time-dependent wall data (Sec. 3.1.3) and of the
conservative method's forcing term (Sec. 4, eq. (wavequ) with f).

Wall data.  At a non-periodic wall the ghost polynomial is fixed by the interior data and
by the boundary condition: the prescribed-parity part W of the solution about the wall
(Dirichlet: the even normal part, whose constant term is the boundary value g and whose
higher even terms follow from g through the PDE; Neumann: the odd normal part) enters the
ghost as R(interior) + 2 W(ghost).  Pins: for any polynomial solution of the wave
equation (of the degrees a half step evolves exactly) a half step onto the primal grid
with the exact wall records reproduces the exact solution at every node, walls and
corners included, in d = 1..3 and both methods; without the records (homogeneous walls)
it does not; and with time-dependent records from a travelling wave that does not vanish
at the walls the dissipative method converges at its order 2m-1.
"""
import math

import numpy as np
import numpy.polynomial.polynomial as npoly
import pytest

import oracle
from paper_1802_05246_amd import workloads as W
from test_oracle_pins import _lap, _oracle_problem, _poly_nodal, _poly_solution, _rand_poly


def _eval_poly(cf, pts):
    d = cf.ndim
    if d == 1:
        return npoly.polyval(pts[:, 0], cf)
    if d == 2:
        return npoly.polyval2d(pts[:, 0], pts[:, 1], cf)
    return npoly.polyval3d(pts[:, 0], pts[:, 1], pts[:, 2], cf)


def _scaled_derivs_at(cf, pts, orders, h):
    """h^k/k! d^k of the tensor polynomial cf at the points, one multi-index k."""
    g = cf
    scale = 1.0
    for i, k in enumerate(orders):
        if k:
            g = npoly.polyder(g, k, axis=i) if g.shape[i] > k else np.zeros_like(g)
        scale *= h[i] ** k / math.factorial(k)
    return scale * _eval_poly(g, pts)


def wall_records(spec, cf, M):
    """Wall records (oracle.wall_faces order) of the tensor polynomial cf, Mrec = M: at
    every wall point (wall coordinate in the normal dimension, dual-grid positions with
    one ghost position at each end in the others) the scaled coefficients whose normal
    degree is 2j (Dirichlet) or 2j+1 (Neumann), j = 0..M-1."""
    p = _oracle_problem(spec)
    d = spec.d
    h = [spec.h(i) for i in range(d)]
    recs = []
    for i, side, ext in oracle.wall_faces(p):
        tang = [t for t in range(d) if t != i]
        grids = []
        for t, e in zip(tang, ext):
            if spec.bc[t] == W.PERIODIC:
                grids.append(spec.xl[t] + (np.arange(e) + 0.5) * h[t])
            else:
                grids.append(spec.xl[t] + (np.arange(e) - 0.5) * h[t])
        mesh = np.meshgrid(*grids, indexing="ij") if grids else []
        npts = int(np.prod(ext)) if ext else 1
        pts = np.zeros((npts, d))
        pts[:, i] = spec.xl[i] if side < 0 else spec.xr[i]
        for k, t in enumerate(tang):
            # x fastest among the tangential dimensions
            pts[:, t] = np.transpose(mesh[k]).reshape(-1) if d == 3 else mesh[k].reshape(-1)
        rec = np.zeros((npts, M ** d))
        for c in range(M ** d):
            ls = [(c // M ** t) % M for t in range(d)]
            k = list(ls)
            k[i] = 2 * ls[i] + (0 if spec.bc[i] == W.DIRICHLET else 1)
            rec[:, c] = _scaled_derivs_at(cf, pts, k, h)
        recs.append(rec)
    return np.concatenate(recs, axis=0)


BOXES = [
    (1, [W.DIRICHLET]), (1, [W.NEUMANN]),
    (2, [W.DIRICHLET, W.NEUMANN]), (2, [W.NEUMANN, W.NEUMANN]), (2, [W.DIRICHLET, W.DIRICHLET]),
    (3, [W.DIRICHLET, W.NEUMANN, W.DIRICHLET]),
]


@pytest.mark.parametrize("d,bc", BOXES)
@pytest.mark.parametrize("method", [W.DISS_SIMPLE, W.DISS_FULL])
def test_diss_walls_exact_for_polynomial_solutions(d, bc, method):
    m = {1: 3, 2: 2, 3: 1}[d]
    rng = np.random.default_rng(5 + 10 * d + method + sum(bc))
    spec = W.make_spec(d, m, [3, 4, 2][:d], xl=[0.1, -0.2, 0.3][:d], xr=[0.7, 0.5, 0.9][:d],
                       c=1.3, cfl=0.8, bc=bc, method=method)
    if method == W.DISS_SIMPLE or d == 1:
        u0, v0 = _rand_poly(rng, d, 2 * m + 1), np.pad(_rand_poly(rng, d, 2 * m - 1), [(0, 2)] * d)
    else:
        u0 = np.pad(_rand_poly(rng, d, 2 * m - 1), [(0, 2)] * d)
        v0 = np.pad(_rand_poly(rng, d, 2 * m - 2), [(0, 3)] * d)
    uT, vT = _poly_solution(u0, v0, spec.c, 0.5 * spec.dt, d)
    p = _oracle_problem(spec)
    ud, vd = _poly_nodal(u0, spec, W.DUAL, m + 1), _poly_nodal(v0, spec, W.DUAL, m)
    walls = (wall_records(spec, u0, m + 1), wall_records(spec, v0, m))
    uo, vo = oracle.diss_half(p, oracle.PRIMAL, ud, vd, walls=walls)
    ue, ve = _poly_nodal(uT, spec, W.PRIMAL, m + 1), _poly_nodal(vT, spec, W.PRIMAL, m)
    np.testing.assert_allclose(uo, ue, atol=1e-10 * np.abs(ue).max(), rtol=0)
    np.testing.assert_allclose(vo, ve, atol=1e-10 * np.abs(ve).max(), rtol=0)
    # homogeneous walls are wrong for this data (it does not vanish at the walls)
    uh, vh = oracle.diss_half(p, oracle.PRIMAL, ud, vd)
    assert np.abs(uh - ue).max() > 1e-3 * np.abs(ue).max()
    # the half step onto the dual grid needs no ghosts: the records are ignored
    upr, vpr = _poly_nodal(u0, spec, W.PRIMAL, m + 1), _poly_nodal(v0, spec, W.PRIMAL, m)
    ua, va = oracle.diss_half(p, oracle.DUAL, upr, vpr, walls=walls)
    ub, vb = oracle.diss_half(p, oracle.DUAL, upr, vpr)
    np.testing.assert_array_equal(ua, ub)


@pytest.mark.parametrize("d,bc", BOXES)
def test_cons_walls_exact_for_polynomial_solutions(d, bc):
    m = {1: 3, 2: 2, 3: 1}[d]
    rng = np.random.default_rng(77 + 10 * d + sum(bc))
    spec = W.make_spec(d, m, [3, 4, 2][:d], xl=[0.1, -0.2, 0.3][:d], xr=[0.7, 0.5, 0.9][:d],
                       c=0.9, cfl=1.0, bc=bc, method=W.CONSERVATIVE)
    u0, v0 = _rand_poly(rng, d, 2 * m + 1), _rand_poly(rng, d, 2 * m + 1)
    tau = 0.5 * spec.dt
    um, _ = _poly_solution(u0, v0, spec.c, -tau, d)
    up, _ = _poly_solution(u0, v0, spec.c, tau, d)
    p = _oracle_problem(spec)
    ud = _poly_nodal(u0, spec, W.DUAL, m + 1)
    old = _poly_nodal(um, spec, W.PRIMAL, m + 1)
    ue = _poly_nodal(up, spec, W.PRIMAL, m + 1)
    un = oracle.cons_half(p, oracle.PRIMAL, ud, old, walls=wall_records(spec, u0, m + 1))
    np.testing.assert_allclose(un, ue, atol=1e-10 * np.abs(ue).max(), rtol=0)
    uh = oracle.cons_half(p, oracle.PRIMAL, ud, old)
    assert np.abs(uh - ue).max() > 1e-3 * np.abs(ue).max()


def test_wall_records_of_odd_data_are_the_homogeneous_case():
    """Data that already has the wall's parity has W = 0 there: zero records give the
    homogeneous ghosts bit for bit."""
    spec = W.make_spec(2, 2, [4, 3], 0.0, 1.0, 1.0, cfl=0.9, bc=[W.DIRICHLET, W.NEUMANN])
    p = _oracle_problem(spec)
    u, v = W.random_state(spec, 3, grid=W.DUAL)
    n = oracle.wall_points(p)
    z = (np.zeros((n, 9)), np.zeros((n, 4)))
    a = oracle.diss_half(p, oracle.PRIMAL, u, v, walls=z)
    b = oracle.diss_half(p, oracle.PRIMAL, u, v)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def _travelling_wave_run(n, m, lam=0.8, t_final=0.5, kappa=2.0, use_walls=True):
    """1-D, [0, 1], Dirichlet walls with the time-dependent data of the travelling wave
    u = sin(2 pi kappa (x - c t) + 0.3), exact records at every half step; returns the
    nodal L2 error of the value coefficient at the final step."""
    c = 1.0
    spec = W.make_spec(1, m, n, 0.0, 1.0, c, cfl=lam, bc=W.DIRICHLET, method=W.DISS_FULL)
    p = _oracle_problem(spec)
    k = 2 * math.pi * kappa
    h = spec.h(0)

    def data(grid, t, M, deriv_t=0):
        x = spec.coords(grid, 0)
        # d^l/dx^l d^r/dt^r sin(k x - k c t + 0.3) = k^l (-k c)^r sin(. + (l + r) pi/2)
        out = np.stack([k ** l * (-k * c) ** deriv_t * np.sin(k * x - k * c * t + 0.3 + (l + deriv_t) * math.pi / 2)
                        * h ** l / math.factorial(l) for l in range(M)], axis=1)
        return out

    def records(t, M, deriv_t):
        rec = []
        for xw in (0.0, 1.0):
            r = np.zeros((1, M))
            for j in range(M):
                kk = 2 * j
                r[0, j] = (k ** kk * (-k * c) ** deriv_t * math.sin(k * xw - k * c * t + 0.3 + (kk + deriv_t) * math.pi / 2)
                           * h ** kk / math.factorial(kk))
            rec.append(r)
        return np.concatenate(rec)

    steps = round(t_final / spec.dt)
    u, v = data(W.PRIMAL, 0.0, m + 1), data(W.PRIMAL, 0.0, m, 1)
    t = 0.0
    for _ in range(steps):
        u, v = oracle.diss_half(p, oracle.DUAL, u, v)
        t += 0.5 * spec.dt
        w = (records(t, m + 1, 0), records(t, m, 1)) if use_walls else None
        u, v = oracle.diss_half(p, oracle.PRIMAL, u, v, walls=w)
        t += 0.5 * spec.dt
    ex = np.sin(k * spec.coords(W.PRIMAL, 0) - k * c * t + 0.3)
    return W.nodal_l2(spec, u[:, 0], ex)


@pytest.mark.parametrize("m", [2, 3])
def test_time_dependent_dirichlet_data_converges_at_design_order(m):
    errs = [_travelling_wave_run(n, m) for n in (40, 80)]
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - (2 * m - 1)) < 0.3, (errs, rate)
    # with homogeneous walls the run solves another problem: no convergence to this wave
    assert _travelling_wave_run(80, m, use_walls=False) > 1e3 * errs[1]


# ---------------------------------------------------------------------------
# conservative method with a forcing term: u_tt = c^2 Lap u + f
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,m", [(1, 2), (1, 3), (2, 1), (2, 2), (3, 1)])
@pytest.mark.parametrize("cfl", [0.7, 1.0])
def test_cons_forced_polynomial_solution_exact(d, m, cfl):
    """u(x, t) = sum_b t^b U_b(x) (U_b of degree 2m+1 per dimension, b <= 4) and its
    forcing f = u_tt - c^2 Lap u: a conservative half step from the exact levels at
    -dt/2 (old) and 0 (the other grid) with the forcing's time derivatives at t = 0
    reproduces the exact level at dt/2; without the forcing, or with its second time
    derivative left out, it does not."""
    rng = np.random.default_rng(31 + 10 * d + m)
    spec = W.make_spec(d, m, [3] * d, 0.0, 1.0, 1.0, cfl=cfl, bc=W.DIRICHLET, method=W.CONSERVATIVE)
    bdeg = 4
    U = [_rand_poly(rng, d, 2 * m + 1) for _ in range(bdeg + 1)]
    c2 = spec.c ** 2
    f = []
    for r in range(bdeg + 1):
        acc = -c2 * _lap(U[r], d)
        if r + 2 <= bdeg:
            acc = acc + (r + 2) * (r + 1) * U[r + 2]
        f.append(math.factorial(r) * acc)
    tau = 0.5 * spec.dt
    um = sum(((-tau) ** b) * U[b] for b in range(bdeg + 1))
    up = sum((tau ** b) * U[b] for b in range(bdeg + 1))
    p = _oracle_problem(spec)
    src = _poly_nodal(U[0], spec, W.PRIMAL, m + 1)
    old = _poly_nodal(um, spec, W.DUAL, m + 1)
    ue = _poly_nodal(up, spec, W.DUAL, m + 1)
    phi = np.stack([_poly_nodal(fr, spec, W.DUAL, 2 * m + 2) for fr in f], axis=1)
    un = oracle.cons_half(p, oracle.DUAL, src, old, forcing=phi)
    np.testing.assert_allclose(un, ue, atol=1e-10 * max(1.0, np.abs(ue).max()), rtol=0)
    u0 = oracle.cons_half(p, oracle.DUAL, src, old)
    assert np.abs(u0 - ue).max() > 1e-6
    u2 = oracle.cons_half(p, oracle.DUAL, src, old, forcing=phi[:, :2])
    assert np.abs(u2 - ue).max() > 1e-9
