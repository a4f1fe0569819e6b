"""The batched 2-D solver's captured graph, in which each (m, method) class runs its chain of
launches as a branch of its own (forked from the capture stream and joined back into it),
against the same solver stepped launch by launch on one stream: bitwise equal, replay after
replay of the same graph, with the program's own work (state reads, synchronisations)
between the replays.  The batch holds every class, m = 2..6 with both methods, and every
wall type."""
import numpy as np
import pytest

from paper_1802_05246_amd import workloads as W

from test_gpu_parity import _log, _state

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MS = [2, 3, 4, 5, 6, 2, 3, 4, 5, 6, 4, 6]


def _specs():
    return [W.make_spec(2, m, [21 + 9 * i, 13 + 7 * i], 0.0, 1.0, 0.8 + 0.05 * i, cfl=0.85,
                        bc=[W.PERIODIC, W.DIRICHLET, W.NEUMANN][i % 3],
                        method=[W.DISS_FULL, W.CONSERVATIVE][(i // 5 + m) % 2])
            for i, m in enumerate(MS)]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_graph_branches_equal_plain_launches(prec):
    from paper_1802_05246_amd import binding as B
    specs = _specs()
    assert len({(sp.m, sp.method) for sp in specs}) == 10
    states = [_state(sp, 950 + i) for i, sp in enumerate(specs)]
    s = B.Solver(problems=specs, precision=B.HW_FP64 if prec == "fp64" else B.HW_FP32)

    def snapshot():
        torch.cuda.synchronize()
        return [tuple(x.cpu().numpy().copy() for x in s.get_state(i)) for i in range(len(specs))]

    runs = {}
    for mode in ("graph", "plain"):
        for i, (u, w) in enumerate(states):
            s.set_state(u, w, i=i)
        seq = []
        for _ in range(3):
            if mode == "graph":
                s.advance(2)        # the same captured graph each time
            else:
                s.half_steps(4)     # one launch per class and half step, in class order
            seq.append(snapshot())
        runs[mode] = seq
    s.close()
    for r in range(3):
        for i in range(len(specs)):
            for a, b in zip(runs["graph"][r][i], runs["plain"][r][i]):
                assert np.array_equal(a, b), (prec, r, i)
    _log(f"[batch graph] {prec}: 3 replays of 2 steps, {len(specs)} problems bitwise equal")
    # the replays advanced the state
    assert not np.array_equal(runs["graph"][0][0][0], runs["graph"][2][0][0])
