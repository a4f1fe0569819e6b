"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances.  FP64 form: rel-L2 <= 1e-10 for u and for v separately, over every
coefficient of every node (expected 1e-13..1e-11; cond(H_6) ~ 1.4e5 sets the
ceiling).  FP32 form: the error is measured in the norm the paper measures errors
in, the L2 norm of the solution: the relative L2 norm over the cell of the local
Taylor polynomials of [u, tau*v] (tau = dt/2) at the nodes.  Each half step
perturbs the data by single-precision rounding (u32 = 2^-24); interpolation and the
time sums amplify it by a modest factor in this norm that grows with the size of the
Hermite operator's entries (largest |entry| of H_m: 1, 2, 6, 21, 90, 385, 1638 for
m = 0..6), and the perturbations add up over the checked half steps:
tol = 200 u32 n_half max(1, max|H_m| / max|H_3|).  (Coefficient by coefficient the
highest mixed derivatives of smooth data are tiny and are computed through products
of Hermite rows with entries up to 21 (m = 3); their relative rounding error is
large although they hardly contribute to the function.)
"""
import sys

import numpy as np
import pytest

from paper_1802_05246_amd import workloads as W

from helpers import oracle_reference_run, poly_rel_err, rel_l2, sampled_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


U32 = 2.0 ** -24


_HMAX = [1.0, 2.0, 6.0, 21.0, 90.0, 385.0, 1638.0]  # largest |entry| of H_m


def fp32_tol(m, n_half):
    return 200.0 * U32 * max(1, n_half) * max(1.0, _HMAX[m] / _HMAX[3])


def joint_err(spec, gu, gv, ou, ov):
    return poly_rel_err(spec, gu, ou, gv, ov)


def state_err(spec, gu, gv, ou, ov, prec, n_half):
    """(error, tolerance) of a GPU state against the oracle's, random data.
    FP64: plain relative L2 over every coefficient of every node, u and v separately,
    bar 1e-10.  FP32: the same per-field plain relative L2 and the polynomial L2 of the
    joint [u, tau v], all against fp32_tol(m, n_half)."""
    eu = rel_l2(gu, ou)
    ev = rel_l2(gv, ov) if gv is not None and ov is not None else 0.0
    if prec in ("fp64", 0):
        return max(eu, ev), 1e-10
    return max(eu, ev, joint_err(spec, gu, gv, ou, ov)), fp32_tol(spec.m, n_half)


def _B():
    from paper_1802_05246_amd import binding as B
    return B


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    _B().lib()  # fail loudly if the HIP library is missing
    yield


def _state(spec, seed):
    rng = np.random.default_rng(seed)
    M = spec.m + 1
    u = rng.uniform(-1, 1, (spec.nodes(W.PRIMAL), M ** spec.d))
    if spec.method == W.CONSERVATIVE:
        w = rng.uniform(-1, 1, (spec.nodes(W.DUAL), M ** spec.d))
    else:
        w = rng.uniform(-1, 1, (spec.nodes(W.PRIMAL), spec.m ** spec.d))
    return u, w


CASES = [
    # (d, m, n, bc, method, taylor_stages)
    (1, 1, [9], [W.PERIODIC], W.DISS_FULL, 0),
    (1, 3, [11], [W.DIRICHLET], W.DISS_FULL, 0),
    (1, 6, [7], [W.NEUMANN], W.DISS_FULL, 0),
    (2, 2, [7, 5], [W.PERIODIC, W.DIRICHLET], W.DISS_FULL, 0),
    (2, 3, [9, 6], [W.PERIODIC, W.PERIODIC], W.DISS_FULL, 0),
    (2, 3, [5, 7], [W.NEUMANN, W.DIRICHLET], W.DISS_SIMPLE, 0),
    (2, 5, [4, 5], [W.DIRICHLET, W.PERIODIC], W.DISS_FULL, 0),
    (2, 2, [6, 6], [W.PERIODIC, W.PERIODIC], W.DISS_FULL, 6),
    (3, 1, [5, 4, 3], [W.PERIODIC, W.DIRICHLET, W.NEUMANN], W.DISS_FULL, 0),
    (3, 3, [5, 4, 6], [W.PERIODIC, W.PERIODIC, W.PERIODIC], W.DISS_FULL, 0),
    (3, 3, [4, 3, 5], [W.DIRICHLET, W.NEUMANN, W.PERIODIC], W.DISS_FULL, 0),
    (3, 2, [4, 4, 3], [W.PERIODIC, W.PERIODIC, W.DIRICHLET], W.DISS_SIMPLE, 0),
    (3, 3, [5, 4, 3], [W.PERIODIC, W.PERIODIC, W.PERIODIC], W.DISS_SIMPLE, 0),
    (3, 3, [4, 3, 4], [W.DIRICHLET, W.PERIODIC, W.NEUMANN], W.DISS_SIMPLE, 0),
    (3, 3, [4, 5, 3], [W.PERIODIC, W.PERIODIC, W.PERIODIC], W.DISS_FULL, 7),
    (3, 3, [3, 4, 4], [W.PERIODIC, W.DIRICHLET, W.PERIODIC], W.DISS_FULL, 8),
    (2, 3, [6, 5], [W.PERIODIC, W.PERIODIC], W.DISS_SIMPLE, 7),
    (1, 0, [8], [W.PERIODIC], W.CONSERVATIVE, 0),
    (1, 4, [9], [W.DIRICHLET], W.CONSERVATIVE, 0),
    (2, 4, [7, 6], [W.DIRICHLET, W.DIRICHLET], W.CONSERVATIVE, 0),
    (2, 2, [5, 8], [W.NEUMANN, W.PERIODIC], W.CONSERVATIVE, 0),
    (3, 2, [4, 5, 3], [W.PERIODIC, W.NEUMANN, W.DIRICHLET], W.CONSERVATIVE, 0),
]


def _case_id(c):
    d, m, n, bc, meth, st = c
    return f"d{d}-m{m}-n{'x'.join(map(str, n))}-bc{''.join(map(str, bc))}-meth{meth}-st{st}"


@pytest.mark.parametrize("case", CASES, ids=[_case_id(c) for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_small_grids_match_oracle(case, prec):
    B = _B()
    d, m, n, bc, meth, stages = case
    _log(f"[parity] {_case_id(case)} {prec}")
    spec = W.make_spec(d, m, n, 0.0, [1.0, 0.9, 0.8][:d], 1.1, cfl=0.9, bc=bc, method=meth,
                       taylor_stages=stages)
    u, w = _state(spec, 17 + d + m)
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    s = B.Solver(spec, precision=precision, kernel=B.HW_KERNEL_GENERIC)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    n_half = 6
    s.half_steps(n_half)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    ou, ow = oracle_reference_run(spec, u_in, w_in, n_half)
    err, tol = state_err(spec, gu, gw, ou, ow, prec, n_half)
    _log(f"    rel-L2 = {err:.3e} (tol {tol:g})")
    assert err <= tol
    s.close()


def _dense_supported(d, m, meth):
    return d == 1 or (d == 2 and not (meth == W.CONSERVATIVE and m >= 6))


DENSE_CASES = [c for c in CASES if _dense_supported(c[0], c[1], c[4])] + [
    (2, 1, [5, 4], [W.DIRICHLET, W.NEUMANN], W.DISS_FULL, 0),
    (2, 3, [6, 7], [W.DIRICHLET, W.DIRICHLET], W.DISS_FULL, 0),
    (2, 2, [4, 6], [W.NEUMANN, W.NEUMANN], W.DISS_SIMPLE, 0),
    (2, 0, [6, 5], [W.PERIODIC, W.DIRICHLET], W.CONSERVATIVE, 0),
    (2, 3, [5, 6], [W.NEUMANN, W.NEUMANN], W.CONSERVATIVE, 0),
    (1, 2, [6], [W.NEUMANN], W.DISS_SIMPLE, 5),
    (2, 4, [5, 4], [W.PERIODIC, W.NEUMANN], W.DISS_FULL, 0),
    (2, 6, [4, 4], [W.DIRICHLET, W.PERIODIC], W.DISS_FULL, 0),
    (2, 6, [4, 5], [W.NEUMANN, W.DIRICHLET], W.DISS_SIMPLE, 0),
    (2, 5, [5, 4], [W.DIRICHLET, W.NEUMANN], W.CONSERVATIVE, 0),
]


@pytest.mark.parametrize("case", DENSE_CASES, ids=[_case_id(c) for c in DENSE_CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_kernel_matches_oracle(case, prec):
    """The per-lane dense kernel (d <= 2: each cell's half step as one matrix applied to
    its corners) against the oracle, same bars as the generic kernel."""
    B = _B()
    d, m, n, bc, meth, stages = case
    _log(f"[parity dense] {_case_id(case)} {prec}")
    spec = W.make_spec(d, m, n, 0.0, [1.0, 0.9, 0.8][:d], 1.1, cfl=0.9, bc=bc, method=meth,
                       taylor_stages=stages)
    u, w = _state(spec, 29 + d + m)
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    s = B.Solver(spec, precision=precision, kernel=B.HW_KERNEL_DENSE)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    n_half = 6
    s.half_steps(n_half)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    ou, ow = oracle_reference_run(spec, u_in, w_in, n_half)
    err, tol = state_err(spec, gu, gw, ou, ow, prec, n_half)
    _log(f"    rel-L2 = {err:.3e} (tol {tol:g})")
    assert err <= tol
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_advance_equals_plain_launches_bitwise(prec):
    B = _B()
    spec = W.make_spec(2, 3, [12, 10], 0.0, 1.0, 1.0, cfl=0.9, bc=[W.PERIODIC, W.DIRICHLET])
    u, w = _state(spec, 5)
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    a = B.Solver(spec, precision=precision)
    b = B.Solver(spec, precision=precision)
    a.set_state(u, w)
    b.set_state(u, w)
    a.advance(3)
    a.advance(2)
    b.half_steps(10)
    ua, wa = a.get_state()
    ub, wb = b.get_state()
    assert torch.equal(ua, ub) and torch.equal(wa, wb)
    # resume: get_state -> set_state on a fresh solver continues bitwise
    c = B.Solver(spec, precision=B.HW_FP64)
    d_ = B.Solver(spec, precision=B.HW_FP64)
    c.set_state(u, w)
    c.advance(4)
    d_.set_state(u, w)
    d_.advance(2)
    mid_u, mid_w = d_.get_state()
    e = B.Solver(spec, precision=B.HW_FP64)
    e.set_state(mid_u, mid_w)
    e.advance(2)
    assert torch.equal(c.get_state()[0], e.get_state()[0])
    for x in (a, b, c, d_, e):
        x.close()


@pytest.mark.parametrize("d,m,bc", [(2, 2, W.PERIODIC), (2, 3, W.DIRICHLET), (1, 4, W.NEUMANN),
                                    (3, 1, W.PERIODIC), (2, 4, W.DIRICHLET), (3, 3, W.NEUMANN),
                                    (3, 3, W.PERIODIC)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_energy_matches_oracle_and_is_conserved(d, m, bc, prec):
    """hw_energy (FP64 accumulation, in both state precisions) against the oracle's
    energy of the GPU's own last three levels (1e-12 relative: the same FP64 quantity
    summed in another order), and conserved over 8 half steps: to 1e-11 with the FP64
    state; with the FP32 state each half step's rounding moves it (bound 1e-4)."""
    import oracle
    from helpers import oracle_problem
    B = _B()
    spec = W.make_spec(d, m, [6, 5, 4][:d], 0.0, [1.0, 0.7, 0.6][:d], 1.0, cfl=1.0, bc=bc,
                       method=W.CONSERVATIVE)
    rng = np.random.default_rng(3)
    M = m + 1
    up = rng.uniform(0, 1, (spec.nodes(W.PRIMAL), M ** d))
    if bc != W.PERIODIC:
        from test_oracle_pins import _wall_compatible
        up = _wall_compatible(spec, up)
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    s = B.Solver(spec, precision=precision)
    s.cons_startup(up)
    energies = []
    for k in range(8):
        if k == 7:
            gp7, gd7 = (x.cpu().numpy() for x in s.get_state())
        s.half_steps(1)
        energies.append(s.energy())
    gp, gd = (x.cpu().numpy() for x in s.get_state())
    # after 8 half steps the dual grid was updated last: A = primal, B = dual
    p = oracle_problem(spec)
    e_or = oracle.cons_energy(p, oracle.PRIMAL, gp, gd, gd7)
    e = np.array(energies)
    drift = np.abs(e - e[0]).max() / abs(e[0])
    _log(f"[energy] d{d} m{m} bc{bc} {prec}: vs oracle {abs(energies[-1] - e_or) / abs(e_or):.2e}, "
         f"drift over 8 half steps {drift:.2e}")
    assert energies[-1] == pytest.approx(e_or, rel=1e-12)
    assert drift <= (1e-11 if prec == "fp64" else 1e-4)
    s.close()


def test_cons_startup_matches_oracle():
    import oracle
    from helpers import oracle_problem
    B = _B()
    for d, m, bc in [(2, 3, W.DIRICHLET), (3, 2, W.PERIODIC), (1, 5, W.NEUMANN)]:
        spec = W.make_spec(d, m, [6, 5, 4][:d], 0.0, 1.0, 1.3, cfl=0.8, bc=bc, method=W.CONSERVATIVE)
        rng = np.random.default_rng(d * m)
        u0 = rng.uniform(-1, 1, (spec.nodes(W.PRIMAL), (m + 1) ** d))
        v0 = rng.uniform(-1, 1, (spec.nodes(W.PRIMAL), (m + 1) ** d))
        for vv in (None, v0):
            s = B.Solver(spec, precision=B.HW_FP64)
            s.cons_startup(u0, vv)
            _, gd = s.get_state()
            od = oracle.cons_startup(oracle_problem(spec), u0, vv)
            assert rel_l2(gd.cpu().numpy(), od) < 1e-12
            s.close()


def test_batch_matches_oracle_per_problem():
    B = _B()
    specs, states = [], []
    mix = [(2, [9, 7], W.PERIODIC, W.DISS_FULL), (3, [6, 5], W.DIRICHLET, W.DISS_FULL),
           (4, [5, 5], W.NEUMANN, W.CONSERVATIVE), (2, [11, 4], W.DIRICHLET, W.CONSERVATIVE),
           (5, [4, 6], W.PERIODIC, W.DISS_FULL), (6, [3, 4], W.PERIODIC, W.CONSERVATIVE)]
    for k, (m, n, bc, meth) in enumerate(mix):
        spec = W.make_spec(2, m, n, 0.0, 1.0, 0.5 + 0.3 * k, cfl=0.8, bc=bc, method=meth)
        specs.append(spec)
        states.append(_state(spec, 100 + k))
    for prec in (B.HW_FP64, B.HW_FP32):
        s = B.Solver(problems=specs, precision=prec)
        ins = []
        for i, (u, w) in enumerate(states):
            s.set_state(u, w, i=i)
        for i in range(len(specs)):
            ins.append([x.cpu().numpy() for x in s.get_state(i)])
        s.advance(3)
        for i, spec in enumerate(specs):
            gu, gw = (x.cpu().numpy() for x in s.get_state(i))
            ou, ow = oracle_reference_run(spec, ins[i][0], ins[i][1], 6)
            err, tol = state_err(spec, gu, gw, ou, ow, "fp64" if prec == B.HW_FP64 else "fp32", 6)
            _log(f"[batch] problem {i} prec {prec} rel-L2 {err:.3e}")
            assert err <= tol
        s.close()


def _sampled_check(spec, precision, n_samples, seed, w_state=None, steps_half=1):
    """Run `steps_half` half steps (the last one checked) at full size and compare
    sampled output nodes with the oracle evaluated cell by cell."""
    B = _B()
    s = B.Solver(spec, precision=precision)
    u0, w0 = w_state
    s.set_state(u0, w0)
    del u0, w0
    if steps_half > 1:
        s.half_steps(steps_half - 1)
    xin_u, xin_w = s.get_state()
    to_grid = 1 - s.state_grid() if spec.method != W.CONSERVATIVE else (
        W.PRIMAL if (steps_half - 1) % 2 == 0 else W.DUAL)
    s.half_steps(1)
    yu, yw = s.get_state()
    rng = np.random.default_rng(seed)
    n_out = spec.nodes(to_grid)
    samples = list(rng.choice(n_out, size=n_samples, replace=False))
    # always include the first and last output node (wall / wrap-around cells)
    samples = [0, n_out - 1] + samples

    if spec.method == W.CONSERVATIVE:
        # xin: (primal, dual); the grid read is the other grid at the middle time
        src_u = xin_w if to_grid == W.PRIMAL else xin_u
        old = xin_u if to_grid == W.PRIMAL else xin_w
        new = yu if to_grid == W.PRIMAL else yw

        def u_in(ix):
            return src_u[torch.as_tensor(ix, device="cuda")].cpu().numpy()

        def u_old(ix):
            return old[torch.as_tensor(ix, device="cuda")].cpu().numpy()
        ou, _ = sampled_oracle(spec, to_grid, u_in, None, samples, u_old=u_old)
        gu = new[torch.as_tensor(samples, device="cuda")].cpu().numpy()
        gv = ov = None
    else:
        def u_in(ix):
            return xin_u[torch.as_tensor(ix, device="cuda")].cpu().numpy()

        def v_in(ix):
            return xin_w[torch.as_tensor(ix, device="cuda")].cpu().numpy()
        ou, ov = sampled_oracle(spec, to_grid, u_in, v_in, samples)
        sel = torch.as_tensor(samples, device="cuda")
        gu, gv = yu[sel].cpu().numpy(), yw[sel].cpu().numpy()
    s.close()
    B = _B()
    if precision == B.HW_FP64:
        err = max(rel_l2(gu, ou), rel_l2(gv, ov) if gv is not None else 0.0)
        tol = 1e-10
    else:
        # smooth data: the joint polynomial L2 of [u, tau v] and the value coefficient
        # (the high mixed coefficients and v after the first half step from v = 0 are
        # tiny, so their plain relative error measures FP32 rounding noise, not parity)
        err = max(joint_err(spec, gu, gv, ou, ov), rel_l2(gu[:, 0], ou[:, 0]))
        tol = fp32_tol(spec.m, 1)
    _log(f"    sampled rel-L2 = {err:.3e} (tol {tol:g})")
    assert err <= tol


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_3d_m3_sampled(prec):
    """256^3, m = 3, periodic, dissipative full: both half-step directions, sampled."""
    B = _B()
    _log(f"[full-size] c4 256^3 {prec}")
    w = W.c4_3d(device="cuda")
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    for steps_half in (1, 2):
        _sampled_check(w.spec, precision, 48, 7 + steps_half, (w.u0, w.v0), steps_half)
    del w
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_columns_3d_m3_sampled(prec):
    """128 x 128 x 512 cells, m = 3, periodic in x, Neumann in y, Dirichlet in z, random
    data: the 3-D kernel walks its columns in z-chunks, lengthened here to 256 cell layers
    (two chunks per column, each starting one node layer below itself); both half-step
    directions, sampled (the first and last output nodes sit at the walls)."""
    B = _B()
    _log(f"[long columns] 128 x 128 x 512 {prec}")
    spec = W.make_spec(3, 3, [128, 128, 512], 0.0, [1.0, 1.0, 4.0], 1.0, cfl=0.9,
                       bc=[W.PERIODIC, W.NEUMANN, W.DIRICHLET])
    g = torch.Generator(device="cuda")
    g.manual_seed(91)
    nodes = spec.nodes(W.PRIMAL)
    u0 = torch.rand(nodes, 64, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    v0 = torch.rand(nodes, 27, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    for steps_half in (1, 2):
        _sampled_check(spec, precision, 48, 11 + steps_half, (u0, v0), steps_half)
    del u0, v0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_3d_cons_m3_sampled(prec):
    """The conservative method in 3-D, m = 3, on the composed-map kernel: 256^3 periodic
    and 96 x 80 x 200 cells with Dirichlet / Neumann / periodic walls (z-chunks of the
    column walk), random data on both grids; both grids, sampled (wall nodes included)."""
    B = _B()
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    for n, bc, seed in (([256, 256, 256], [W.PERIODIC] * 3, 21),
                        ([96, 80, 200], [W.DIRICHLET, W.NEUMANN, W.PERIODIC], 22)):
        _log(f"[full-size] 3-D conservative m=3 n={n} bc={bc} {prec}")
        spec = W.make_spec(3, 3, n, 0.0, [1.0, 0.9, 1.1], 1.0, cfl=0.9, bc=bc, method=W.CONSERVATIVE)
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        up = torch.rand(spec.nodes(W.PRIMAL), 64, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        ud = torch.rand(spec.nodes(W.DUAL), 64, generator=g, device="cuda", dtype=torch.float64) * 2 - 1
        for steps_half in (1, 2):
            _sampled_check(spec, precision, 40, seed + steps_half, (up, ud), steps_half)
        del up, ud
        torch.cuda.empty_cache()


def test_full_size_2d_cons_m4_sampled():
    """2048^2, m = 4, Dirichlet, conservative: both grids, wall nodes included."""
    B = _B()
    _log("[full-size] c3 2048^2")
    w = W.c3_2d()
    for prec in (B.HW_FP64, B.HW_FP32):
        for steps_half in (1, 2):
            _sampled_check(w.spec, prec, 48, 11, (w.u0, w.u_half), steps_half)


def test_full_size_2d_diss_m3_sampled():
    B = _B()
    _log("[full-size] c2 512^2")
    w = W.c2_2d()
    for steps_half in (1, 2):
        _sampled_check(w.spec, B.HW_FP64, 64, 13, (w.u0, w.v0), steps_half)


TILED_CASES = [
    ([5, 4, 6], [W.PERIODIC, W.PERIODIC, W.PERIODIC]),
    ([9, 11, 3], [W.PERIODIC, W.PERIODIC, W.PERIODIC]),
    ([6, 5, 7], [W.DIRICHLET, W.NEUMANN, W.PERIODIC]),
    ([4, 9, 5], [W.NEUMANN, W.DIRICHLET, W.DIRICHLET]),
    ([7, 3, 4], [W.PERIODIC, W.DIRICHLET, W.NEUMANN]),
]


@pytest.mark.parametrize("n,bc", TILED_CASES, ids=[f"{'x'.join(map(str, n))}-bc{''.join(map(str, b))}" for n, b in TILED_CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiled_3d_m3_matches_oracle(n, bc, prec):
    """The LDS-tiled 3-D m = 3 kernel (ragged tiles, every wall type, both half-step
    directions, anisotropic h): FP64 to 1e-10 per coefficient, FP32 to the
    polynomial-L2 tolerance."""
    B = _B()
    _log(f"[tiled] n={n} bc={bc} {prec}")
    spec = W.make_spec(3, 3, n, 0.0, [1.0, 0.8, 0.9], 1.2, cfl=0.85, bc=bc, method=W.DISS_FULL)
    u, w = _state(spec, 31 + sum(n))
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    s = B.Solver(spec, precision=precision, kernel=B.HW_KERNEL_TILED)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    n_half = 4
    s.half_steps(n_half)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    ou, ow = oracle_reference_run(spec, u_in, w_in, n_half)
    err, tol = state_err(spec, gu, gw, ou, ow, prec, n_half)
    _log(f"    rel-L2 = {err:.3e} (tol {tol:g})")
    assert err <= tol
    s.close()


COMPOSED_CASES = [(n, bc, W.DISS_FULL, 0) for n, bc in TILED_CASES] + [
    ([5, 6, 4], [W.PERIODIC, W.DIRICHLET, W.PERIODIC], W.DISS_SIMPLE, 0),
    ([6, 4, 5], [W.NEUMANN, W.PERIODIC, W.DIRICHLET], W.DISS_SIMPLE, 0),
    ([5, 5, 4], [W.PERIODIC, W.PERIODIC, W.PERIODIC], W.DISS_FULL, 7),
    ([4, 5, 6], [W.DIRICHLET, W.PERIODIC, W.PERIODIC], W.DISS_FULL, 8),
    ([5, 4, 6], [W.PERIODIC, W.PERIODIC, W.PERIODIC], W.CONSERVATIVE, 0),
    ([6, 5, 7], [W.DIRICHLET, W.NEUMANN, W.PERIODIC], W.CONSERVATIVE, 0),
    ([4, 9, 5], [W.NEUMANN, W.DIRICHLET, W.DIRICHLET], W.CONSERVATIVE, 0),
    ([9, 3, 4], [W.PERIODIC, W.DIRICHLET, W.NEUMANN], W.CONSERVATIVE, 0),
]


@pytest.mark.parametrize("n,bc,meth,stages", COMPOSED_CASES,
                         ids=[f"{'x'.join(map(str, c[0]))}-bc{''.join(map(str, c[1]))}-meth{c[2]}-st{c[3]}"
                              for c in COMPOSED_CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_composed_3d_m3_matches_oracle(n, bc, meth, stages, prec):
    """The composed-map 3-D m = 3 kernel (ragged tiles, every wall type, both half-step
    directions, anisotropic h, both dissipative variants, truncated series, and the
    conservative method) against the oracle."""
    B = _B()
    _log(f"[composed] n={n} bc={bc} meth={meth} st={stages} {prec}")
    spec = W.make_spec(3, 3, n, 0.0, [1.0, 0.8, 0.9], 1.2, cfl=0.85, bc=bc, method=meth,
                       taylor_stages=stages)
    u, w = _state(spec, 37 + sum(n))
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    s = B.Solver(spec, precision=precision, kernel=B.HW_KERNEL_COMPOSED)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    n_half = 4
    s.half_steps(n_half)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    ou, ow = oracle_reference_run(spec, u_in, w_in, n_half)
    err, tol = state_err(spec, gu, gw, ou, ow, prec, n_half)
    _log(f"    rel-L2 = {err:.3e} (tol {tol:g})")
    assert err <= tol
    s.close()


@pytest.mark.parametrize("meth", [W.DISS_FULL, W.CONSERVATIVE])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_composed_3d_m3_wide_offsets_match_oracle(meth, prec, monkeypatch):
    """The composed-map kernel's 64-bit-offset form (taken on its own only for layers over
    4 GB) imposed on a small ragged grid with walls, against the oracle."""
    monkeypatch.setenv("HW_TUNE_FORCE", "cmap3d_offsets=64")
    test_composed_3d_m3_matches_oracle([6, 5, 7], [W.DIRICHLET, W.NEUMANN, W.PERIODIC], meth, 0, prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tiled_equals_generic(prec):
    """Same problem through both kernels: FP64 agree to round-off, FP32 to the
    FP32 tolerance (different summation orders)."""
    B = _B()
    spec = W.make_spec(3, 3, [10, 9, 8], 0.0, 1.0, 1.0, cfl=0.9, bc=W.PERIODIC)
    u, w = _state(spec, 77)
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    a = B.Solver(spec, precision=precision, kernel=B.HW_KERNEL_TILED)
    b = B.Solver(spec, precision=precision, kernel=B.HW_KERNEL_GENERIC)
    for s in (a, b):
        s.set_state(u, w)
        s.advance(3)
    ua, wa = (x.cpu().numpy() for x in a.get_state())
    ub, wb = (x.cpu().numpy() for x in b.get_state())
    if prec == "fp64":
        assert max(rel_l2(ua, ub), rel_l2(wa, wb)) < 1e-11
    else:
        assert joint_err(spec, ua, wa, ub, wb) < fp32_tol(3, 6)
    a.close()
    b.close()


SPLIT_CASES = [(1, 3, [9], [W.NEUMANN], W.DISS_FULL), (2, 3, [7, 6], [W.PERIODIC, W.DIRICHLET], W.DISS_FULL),
               (2, 4, [6, 5], [W.DIRICHLET, W.PERIODIC], W.DISS_SIMPLE),
               (3, 3, [5, 4, 3], [W.PERIODIC, W.NEUMANN, W.DIRICHLET], W.DISS_FULL),
               (3, 2, [4, 4, 4], [W.PERIODIC, W.PERIODIC, W.PERIODIC], W.DISS_SIMPLE)]


@pytest.mark.parametrize("case", SPLIT_CASES, ids=lambda c: f"d{c[0]}-m{c[1]}-meth{c[4]}")
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_kernel_form_equals_fused_bitwise(case, prec):
    """The two-kernel form (interpolants through memory in the state precision) against
    the oracle, to the bar of its precision, and against the fused generic kernel, which
    does the same arithmetic: identical results."""
    B = _B()
    d, m, n, bc, meth = case
    spec = W.make_spec(d, m, n, 0.0, 1.0, 1.3, cfl=0.9, bc=bc, method=meth)
    u, w = _state(spec, 31 + d + m)
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    out = []
    for kernel in (B.HW_KERNEL_GENERIC, B.HW_KERNEL_SPLIT):
        s = B.Solver(spec, precision=precision, kernel=kernel)
        s.set_state(u, w)
        if kernel == B.HW_KERNEL_SPLIT:
            u_in, w_in = (x.cpu().numpy() for x in s.get_state())
        s.advance(3)
        out.append(s.get_state())
        s.close()
    gu, gw = (x.cpu().numpy() for x in out[1])
    ou, ow = oracle_reference_run(spec, u_in, w_in, 6)
    err, tol = state_err(spec, gu, gw, ou, ow, prec, 6)
    _log(f"[split] {_case_id((d, m, n, bc, meth, 0))} {prec}: against the oracle {err:.3e} (tol {tol:.2e})")
    assert err <= tol
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])


BF16_U = 2.0 ** -9  # unit roundoff of a BF16 operand


@pytest.mark.parametrize("n,bc", TILED_CASES[:3], ids=[f"{'x'.join(map(str, n))}-bc{''.join(map(str, b))}" for n, b in TILED_CASES[:3]])
def test_tiled_bf16_operands_match_oracle(n, bc):
    """The BF16-operand form of the tiled kernel (FP32 storage and accumulation, BF16
    operands of the matrix-core stages) against the oracle, in the polynomial L2 norm
    of the joint [u, tau v]: the error is that of rounding the operands to 8-bit
    mantissas (reported, not a parity claim at FP32 level)."""
    B = _B()
    spec = W.make_spec(3, 3, n, 0.0, [1.0, 0.8, 0.9], 1.2, cfl=0.85, bc=bc, method=W.DISS_FULL)
    u, w = _state(spec, 31 + sum(n))
    s = B.Solver(spec, precision=B.HW_BF16, kernel=B.HW_KERNEL_TILED)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    n_half = 4
    s.half_steps(n_half)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    s.close()
    ou, ow = oracle_reference_run(spec, u_in, w_in, n_half)
    err = joint_err(spec, gu, gw, ou, ow)
    tol = 20.0 * BF16_U * n_half
    _log(f"[bf16] n={n} bc={bc} joint rel err {err:.3e} (tol {tol:.3g})")
    assert err <= tol


BATCH_KERNEL_CASES = [
    (m, meth, n, bc)
    for m, meth, n, bc in [
        (1, W.DISS_FULL, [9, 7], [W.PERIODIC, W.DIRICHLET]),
        (2, W.DISS_FULL, [6, 11], [W.NEUMANN, W.PERIODIC]),
        (3, W.DISS_SIMPLE, [13, 5], [W.DIRICHLET, W.NEUMANN]),
        (4, W.DISS_FULL, [7, 7], [W.PERIODIC, W.PERIODIC]),
        (5, W.DISS_FULL, [5, 6], [W.DIRICHLET, W.DIRICHLET]),
        (6, W.DISS_FULL, [4, 5], [W.NEUMANN, W.NEUMANN]),
        (0, W.CONSERVATIVE, [9, 8], [W.DIRICHLET, W.PERIODIC]),
        (2, W.CONSERVATIVE, [70, 3], [W.PERIODIC, W.NEUMANN]),
        (4, W.CONSERVATIVE, [6, 9], [W.DIRICHLET, W.DIRICHLET]),
        (6, W.CONSERVATIVE, [4, 4], [W.NEUMANN, W.PERIODIC]),
    ]
]


@pytest.mark.parametrize("case", BATCH_KERNEL_CASES, ids=lambda c: f"m{c[0]}-meth{c[1]}-n{c[2][0]}x{c[2][1]}")
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_kernel_single_problem_matches_oracle(case, prec):
    """The batched 2-D path (persistent dense launch over a tile work list) on one problem
    (ragged tiles, every wall type, both methods, m = 0..6): six half steps against the
    oracle."""
    B = _B()
    m, meth, n, bc = case
    spec = W.make_spec(2, m, n, 0.0, [1.0, 0.9], 1.1, cfl=0.9, bc=bc, method=meth)
    u, w = _state(spec, 300 + m + meth)
    s = B.Solver(spec, precision=B.HW_FP64 if prec == "fp64" else B.HW_FP32, kernel=B.HW_KERNEL_BATCH)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    s.half_steps(6)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    s.close()
    ou, ow = oracle_reference_run(spec, u_in, w_in, 6)
    err, tol = state_err(spec, gu, gw, ou, ow, prec, 6)
    _log(f"[batch kernel] m={m} meth={meth} n={n} {prec}: rel-L2 {err:.3e} (tol {tol:g})")
    assert err <= tol


def test_batch_kernel_graph_equals_plain_launches_and_reports_tuning():
    """A mixed batch through the batched path (one persistent launch per (m, method)
    class): the captured step loop equals plain launches bit for bit, and the
    autotuner's choices are reported."""
    B = _B()
    specs = [W.make_spec(2, m, [20 + 7 * m, 11 + 3 * m], 0.0, 1.0, 0.6 + 0.2 * m, cfl=0.8,
                         bc=[W.PERIODIC, W.DIRICHLET][m % 2], method=[W.DISS_FULL, W.CONSERVATIVE][m % 2])
             for m in range(2, 7)]
    states = [_state(sp, 500 + i) for i, sp in enumerate(specs)]
    a = B.Solver(problems=specs, precision=B.HW_FP32)
    b = B.Solver(problems=specs, precision=B.HW_FP32)
    for s in (a, b):
        for i, (u, w) in enumerate(states):
            s.set_state(u, w, i=i)
    a.advance(3)
    b.half_steps(6)
    for i in range(len(specs)):
        ga, gb = a.get_state(i), b.get_state(i)
        assert torch.equal(ga[0], gb[0]) and torch.equal(ga[1], gb[1])
    rep = B.hw_tuning_report()
    _log("[tuning]\n" + rep)
    assert "dense_list" in rep
    a.close()
    b.close()
