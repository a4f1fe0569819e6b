"""The 2-D dense kernels in every launch variant the autotuner may choose, against the
oracle: the per-lane gather form (tiles 16 and 128 cells wide), the LDS-staged form
(tiles 32 and 64 wide, corner nodes copied to LDS with coalesced loads, ghost nodes
mirrored there, outputs stored through LDS; codes -32, -64) and the row-chunked staged
form (one coefficient row of every node of the tile in LDS at a time, double-buffered;
codes -1032, -1064) and the composed-map form on the matrix cores (strips of 16 cells
walking their cell rows, corner sums formed in LDS, m = 3..6 only; code -2016).  The
variant is imposed with HW_TUNE_FORCE,
for the single-problem kernel ("dense") and the batched persistent kernel
("dense_list").  Grids span several tiles with ragged edges; every wall type, both
methods, m = 1..6; same bars as the other parity tests."""
import numpy as np
import pytest

from paper_1802_05246_amd import workloads as W

from helpers import oracle_reference_run
from test_gpu_parity import _log, _state, state_err

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CODES = [16, 128, -32, -64, -1032, -1064, -2016]

SINGLE = [
    # m, method, n, bc
    (1, W.DISS_FULL, [70, 9], [W.PERIODIC, W.DIRICHLET]),
    (3, W.DISS_FULL, [67, 10], [W.DIRICHLET, W.NEUMANN]),
    (3, W.DISS_SIMPLE, [33, 20], [W.NEUMANN, W.PERIODIC]),
    (4, W.CONSERVATIVE, [66, 9], [W.DIRICHLET, W.DIRICHLET]),
    (2, W.CONSERVATIVE, [40, 13], [W.PERIODIC, W.NEUMANN]),
    (5, W.CONSERVATIVE, [35, 6], [W.NEUMANN, W.DIRICHLET]),
    (6, W.DISS_FULL, [34, 5], [W.DIRICHLET, W.PERIODIC]),
]


def _id(c):
    m, meth, n, bc = c
    return f"m{m}-meth{meth}-n{n[0]}x{n[1]}-bc{bc[0]}{bc[1]}"


def _staged_fits(m, meth, prec, code):
    """Whether a staged form's LDS fits the 160 KB of a CU (whole records: node tile or
    output staging, odd strides; row chunks: two buffers of one odd-padded row per node);
    the library refuses the other choices.  The composed-map form serves m = 3..6."""
    if code == -2016:
        return 3 <= m <= 6
    tx = (-code) % 1000
    mu, mv = m + 1, (0 if meth == W.CONSERVATIVE else m)
    nodes = (tx + 1) * (256 // tx + 1)
    if -code >= 1000:
        words = 2 * nodes * (mu | 1)
    else:
        nip = (mu * mu + mv * mv) | 1
        words = max(nodes * nip, 256 * nip)
    return words * (8 if prec == "fp64" else 4) <= 160 * 1024


def _run(B, spec, kernel, seed, prec, n_half=4):
    u, w = _state(spec, seed)
    s = B.Solver(spec, precision=B.HW_FP64 if prec == "fp64" else B.HW_FP32, kernel=kernel)
    s.set_state(u, w)
    u_in, w_in = (x.cpu().numpy() for x in s.get_state())
    s.half_steps(n_half)
    gu, gw = (x.cpu().numpy() for x in s.get_state())
    s.close()
    ou, ow = oracle_reference_run(spec, u_in, w_in, n_half)
    return state_err(spec, gu, gw, ou, ow, prec, n_half)


@pytest.mark.parametrize("code", CODES)
@pytest.mark.parametrize("case", SINGLE, ids=[_id(c) for c in SINGLE])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dense_variant_matches_oracle(case, code, prec, monkeypatch):
    from paper_1802_05246_amd import binding as B
    m, meth, n, bc = case
    monkeypatch.setenv("HW_TUNE_FORCE", f"dense={code}")
    spec = W.make_spec(2, m, n, 0.0, [1.0, 0.9], 1.1, cfl=0.9, bc=bc, method=meth)
    _log(f"[dense variant {code}] {_id(case)} {prec}")
    if code < 0 and not _staged_fits(m, meth, prec, code):
        with pytest.raises(B.HwError):
            B.Solver(spec, precision=B.HW_FP64 if prec == "fp64" else B.HW_FP32, kernel=B.HW_KERNEL_DENSE)
        _log("    refused")
        return
    err, tol = _run(B, spec, B.HW_KERNEL_DENSE, 700 + m, prec)
    _log(f"    rel-L2 = {err:.3e} (tol {tol:g})")
    assert err <= tol


BATCH = SINGLE + [(6, W.CONSERVATIVE, [34, 7], [W.NEUMANN, W.PERIODIC])]


@pytest.mark.parametrize("code", CODES)
@pytest.mark.parametrize("case", BATCH, ids=[_id(c) for c in BATCH])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_batch_variant_matches_oracle(case, code, prec, monkeypatch):
    from paper_1802_05246_amd import binding as B
    m, meth, n, bc = case
    monkeypatch.setenv("HW_TUNE_FORCE", f"dense_list={code}")
    spec = W.make_spec(2, m, n, 0.0, [1.0, 0.9], 1.1, cfl=0.9, bc=bc, method=meth)
    _log(f"[batch variant {code}] {_id(case)} {prec}")
    if code < 0 and not _staged_fits(m, meth, prec, code):
        with pytest.raises(B.HwError):
            B.Solver(spec, precision=B.HW_FP64 if prec == "fp64" else B.HW_FP32, kernel=B.HW_KERNEL_BATCH)
        _log("    refused")
        return
    err, tol = _run(B, spec, B.HW_KERNEL_BATCH, 800 + m, prec)
    _log(f"    rel-L2 = {err:.3e} (tol {tol:g})")
    assert err <= tol


@pytest.mark.parametrize("code", [-32, -64, -1032, -1064, -2016])
def test_staged_batch_of_mixed_problems_matches_gather_form(code, monkeypatch):
    """A mixed batch (several problems per (m, method) class, ragged sizes, strips longer
    than one 64-row chunk) through the staged persistent kernels equals the gather form to
    FP64 rounding."""
    from paper_1802_05246_amd import binding as B
    ms = [3, 6, 3, 4, 5, 5, 4, 3] if code == -2016 else [2, 3, 3, 4, 2, 5, 4, 3]
    specs = [W.make_spec(2, m, [29 + 11 * i, 7 + 17 * i], 0.0, 1.0, 0.7 + 0.1 * i, cfl=0.8,
                         bc=[W.PERIODIC, W.DIRICHLET, W.NEUMANN][i % 3],
                         method=[W.DISS_FULL, W.CONSERVATIVE][(m + i) % 2])
             for i, m in enumerate(ms)]
    states = [_state(sp, 900 + i) for i, sp in enumerate(specs)]
    out = {}
    for c in (code, 64):
        monkeypatch.setenv("HW_TUNE_FORCE", f"dense_list={c}")
        s = B.Solver(problems=specs, precision=B.HW_FP64)
        for i, (u, w) in enumerate(states):
            s.set_state(u, w, i=i)
        s.advance(3)
        out[c] = [tuple(x.cpu().numpy() for x in s.get_state(i)) for i in range(len(specs))]
        s.close()
    for i in range(len(specs)):
        for a, b in zip(out[code][i], out[64][i]):
            err = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert err <= 1e-12, (i, err)
