"""Small 1-D problems: the step graph runs all its half steps in one single-workgroup launch
(problems of at most 512 cells), against the same solver stepped one launch per half step:
bitwise equal over repeated replays of one graph, with state reads between the replays; both
methods, every wall type, m = 1..6, sizes on both sides of the 512-cell limit and the
smallest grid (2 cells)."""
import numpy as np
import pytest

from paper_1802_05246_amd import workloads as W

from helpers import oracle_reference_run
from test_gpu_parity import _log, _state, state_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = [
    # m, method, n, wall
    (1, W.DISS_FULL, 64, W.PERIODIC),
    (3, W.DISS_FULL, 64, W.DIRICHLET),
    (3, W.DISS_SIMPLE, 7, W.NEUMANN),
    (6, W.DISS_FULL, 511, W.PERIODIC),
    (4, W.DISS_FULL, 700, W.DIRICHLET),
    (2, W.CONSERVATIVE, 64, W.PERIODIC),
    (5, W.CONSERVATIVE, 512, W.NEUMANN),
    (6, W.CONSERVATIVE, 33, W.DIRICHLET),
    (3, W.CONSERVATIVE, 640, W.PERIODIC),
    (3, W.DISS_FULL, 2, W.DIRICHLET),
]


def _id(c):
    return f"m{c[0]}-meth{c[1]}-n{c[2]}-bc{c[3]}"


@pytest.mark.parametrize("case", CASES, ids=[_id(c) for c in CASES])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_launch_graph_equals_plain_launches(case, prec):
    from paper_1802_05246_amd import binding as B
    m, meth, n, bc = case
    spec = W.make_spec(1, m, [n], 0.0, 1.0, 0.9, cfl=0.9, bc=[bc], method=meth)
    u, w = _state(spec, 1200 + m + n)
    s = B.Solver(spec, precision=B.HW_FP64 if prec == "fp64" else B.HW_FP32)
    runs = {}
    for mode in ("graph", "plain"):
        s.set_state(u, w)
        seq = []
        for _ in range(2):
            if mode == "graph":
                s.advance(3)        # the same captured graph both times
            else:
                s.half_steps(6)
            torch.cuda.synchronize()
            seq.append(tuple(x.cpu().numpy().copy() for x in s.get_state()))
        runs[mode] = seq
    s.close()
    for r in range(2):
        for a, b in zip(runs["graph"][r], runs["plain"][r]):
            assert np.array_equal(a, b), (prec, r)
    _log(f"[1-D graph] {_id(case)} {prec}: graph replays bitwise equal to plain launches")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_launch_graph_matches_oracle(prec):
    """The 1-D standing-wave workload's shape (64 cells, m = 3) through the one-launch graph
    against the oracle, to the parity tests' bars."""
    from paper_1802_05246_amd import binding as B
    spec = W.make_spec(1, 3, [64], 0.0, 1.0, 1.0, cfl=0.9, bc=[W.DIRICHLET], method=W.DISS_FULL)
    u, w = _state(spec, 1301)
    s = B.Solver(spec, precision=B.HW_FP64 if prec == "fp64" else B.HW_FP32)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    s.advance(5)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    s.close()
    ou, ow = oracle_reference_run(spec, u_in, w_in, 10)
    err, tol = state_err(spec, gu, gw, ou, ow, prec, 10)
    _log(f"[1-D graph vs oracle] {prec}: {err:.3e} (tol {tol:g})")
    assert err <= tol
