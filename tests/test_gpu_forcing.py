"""Forcing term of the dissipative method on the GPU (hw_half_step_forced), against the
oracle's stage recursion with the forcing of Sec. 3.1.2 eq. (recursion_diss_1d_2)
and against exact forced polynomial solutions."""
import numpy as np
import pytest

from helpers import oracle_problem, poly_rel_err, rel_l2
from paper_1802_05246_amd import workloads as W
from test_oracle_pins import _forced_polynomial_case

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

U32 = 2.0 ** -24


def _B():
    from paper_1802_05246_amd import binding as B
    B.lib()
    return B


@pytest.mark.parametrize("d,m,method", [(1, 3, W.DISS_FULL), (2, 2, W.DISS_FULL), (2, 3, W.DISS_SIMPLE),
                                        (3, 2, W.DISS_FULL), (3, 3, W.DISS_FULL)])
def test_forced_polynomial_solution_exact(d, m, method):
    """A half step from exact data with the exact forcing coefficients lands on the
    exact solution (degree 2m-1 in space, 4 in time)."""
    B = _B()
    spec, u0, v0, phi, uT, vT = _forced_polynomial_case(d, m, 0.9, method)
    s = B.Solver(spec, precision=B.HW_FP64, kernel=B.HW_KERNEL_GENERIC)
    s.set_state(u0, v0)
    s.half_step_forced(phi)
    gu, gv = (x.cpu().numpy() for x in s.get_state())
    s.close()
    np.testing.assert_allclose(gu, uT, atol=1e-11, rtol=0)
    np.testing.assert_allclose(gv, vT, atol=1e-10, rtol=0)


CASES = [
    # (d, m, n, bc, method, taylor_stages, orders)
    (1, 3, [9], [W.DIRICHLET], W.DISS_FULL, 0, 5),
    (2, 3, [6, 5], [W.PERIODIC, W.NEUMANN], W.DISS_FULL, 0, 4),
    (2, 2, [5, 5], [W.DIRICHLET, W.PERIODIC], W.DISS_SIMPLE, 0, 6),
    (2, 3, [5, 6], [W.PERIODIC, W.PERIODIC], W.DISS_FULL, 7, 4),
    (3, 2, [4, 3, 4], [W.PERIODIC, W.DIRICHLET, W.NEUMANN], W.DISS_FULL, 0, 3),
    (3, 3, [4, 4, 3], [W.PERIODIC, W.PERIODIC, W.PERIODIC], W.DISS_FULL, 0, 2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"d{c[0]}-m{c[1]}-meth{c[4]}-st{c[5]}-R{c[6]}")
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_forced_half_steps_match_oracle(case, prec):
    """Four forced half steps (alternating grids, walls mirrored) with random data and
    random forcing coefficients: GPU against the oracle."""
    B = _B()
    d, m, n, bc, meth, stages, R = case
    spec = W.make_spec(d, m, n, 0.0, 1.0, 1.2, cfl=0.9, bc=bc, method=meth, taylor_stages=stages)
    rng = np.random.default_rng(5 + d + m)
    u = rng.uniform(-1, 1, (spec.nodes(W.PRIMAL), (m + 1) ** d))
    v = rng.uniform(-1, 1, (spec.nodes(W.PRIMAL), m ** d))
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    s = B.Solver(spec, precision=precision, kernel=B.HW_KERNEL_GENERIC)
    s.set_state(u, v)
    ou, ov = (x.cpu().numpy() for x in s.get_state())  # the data in the state precision
    p = oracle_problem(spec)
    grid = W.PRIMAL
    for k in range(4):
        to = 1 - grid
        f = rng.uniform(-1, 1, (spec.nodes(to), R, (2 * m) ** d)) * 10.0
        s.half_step_forced(f)
        ou, ov = oracle.diss_half(p, to, ou, ov, forcing=f)
        grid = to
    gu, gv = (x.cpu().numpy() for x in s.get_state())
    s.close()
    if prec == "fp64":
        assert max(rel_l2(gu, ou), rel_l2(gv, ov)) <= 1e-10
    else:
        assert poly_rel_err(spec, gu, ou, gv, ov) <= 200.0 * U32 * 4


def test_forced_entry_point_errors():
    B = _B()
    spec = W.make_spec(2, 2, [4, 4], 0.0, 1.0, 1.0, cfl=0.9, method=W.DISS_FULL)
    s = B.Solver(spec, precision=B.HW_FP64)
    with pytest.raises(B.HwError) as e:
        s.half_step_forced(None)  # no state set yet
    assert e.value.status == B.HW_ESTATE
    u, v = W.random_state(spec, 1)
    s.set_state(u, v)
    f = torch.zeros((spec.nodes(W.DUAL), 17, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(B.HwError) as e:
        B.hw_half_step_forced(s.h, f, 17)
    assert e.value.status == B.HW_EINVAL
    with pytest.raises(B.HwError) as e:
        B.hw_half_step_forced(s.h, None, 2)
    assert e.value.status == B.HW_EINVAL
    s.half_step_forced(None)  # zero orders: a plain half step
    assert B.hw_state_grid(s.h) == B.HW_DUAL
    s.close()
    # the conservative method takes forcing (and u wall data) too, but no v wall data
    cons = W.make_spec(2, 2, [4, 4], 0.0, 1.0, 1.0, cfl=0.9, bc=W.DIRICHLET, method=W.CONSERVATIVE)
    sc = B.Solver(cons, precision=B.HW_FP64)
    with pytest.raises(B.HwError) as e:
        B.hw_half_step_forced(sc.h, None, 0)
    assert e.value.status == B.HW_ESTATE
    sc.cons_startup(W.random_state(cons, 2)[0])
    w = torch.zeros((40, 9), dtype=torch.float64, device="cuda")
    with pytest.raises(B.HwError) as e:
        B.hw_half_step_ext(sc.h, None, 0, w, w)
    assert e.value.status == B.HW_EINVAL
    sc.close()
    # batches take neither
    sb = B.Solver(problems=[spec, spec], precision=B.HW_FP64)
    with pytest.raises(B.HwError) as e:
        B.hw_half_step_ext(sb.h, None, 0, None, None)
    assert e.value.status == B.HW_EINVAL
    sb.close()
