"""hw_energy_noalloc (the allocation-free energy call) against hw_energy, through the
C ABI: two calls in a row on two solvers, the second smaller, both state precisions.
The result is the same FP64 quantity summed in another order: relative 1e-13."""
import numpy as np
import pytest

from paper_1802_05246_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solver(B, d, m, n, bc, precision, seed):
    spec = W.make_spec(d, m, n, 0.0, 1.0, 1.0, cfl=1.0, bc=bc, method=W.CONSERVATIVE)
    rng = np.random.default_rng(seed)
    u0 = rng.uniform(0.0, 1.0, (spec.nodes(W.PRIMAL), (m + 1) ** d))
    s = B.Solver(spec, precision=precision)
    s.cons_startup(u0)
    s.half_steps(5)
    return s


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_energy_noalloc_matches_energy(prec):
    from paper_1802_05246_amd import binding as B
    B.lib()
    precision = B.HW_FP64 if prec == "fp64" else B.HW_FP32
    big = _solver(B, 2, 4, [96, 80], W.PERIODIC, precision, 1)   # 7680 cells: 2048 workgroups
    small = _solver(B, 2, 3, [7, 5], W.DIRICHLET, precision, 2)  # 48 / 35 cells
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for k, s in enumerate((big, small)):
        ref = s.energy()
        B.hw_energy_noalloc(s.h, out[k:])
        torch.cuda.synchronize()
        got = float(out[k])
        print(f"[noalloc] {prec} solver {k}: hw_energy {ref:.15e}, hw_energy_noalloc {got:.15e}", flush=True)
        assert got == pytest.approx(ref, rel=1e-13)
    # a call after the smaller one still serves the larger grid
    B.hw_energy_noalloc(big.h, out)
    torch.cuda.synchronize()
    assert float(out[0]) == pytest.approx(big.energy(), rel=1e-13)
    big.close()
    small.close()


def test_energy_noalloc_rejects_bad_calls():
    from paper_1802_05246_amd import binding as B
    B.lib()
    spec = W.make_spec(2, 2, [5, 5], 0.0, 1.0, 1.0, cfl=0.9, bc=W.PERIODIC, method=W.DISS_FULL)
    s = B.Solver(spec)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(B.HwError):
        B.hw_energy_noalloc(s.h, out)  # dissipative: no energy
    s.close()
