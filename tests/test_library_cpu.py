"""Host-side checks of the C ABI that need no GPU: every declared entry point is
exported, argument validation precedes any device call, the binding fails loudly
when the library is missing."""
import os
import re

import pytest

from paper_1802_05246_amd import binding as B
from paper_1802_05246_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "hermite_wave.h")).read()
    return sorted(set(re.findall(r"\b(hw_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _declared() == sorted(B.ENTRY_POINTS)


def test_library_exports_every_declared_symbol():
    L = B.lib()
    for name in _declared():
        assert hasattr(L, name), name


def _err(p):
    with pytest.raises(B.HwError) as ei:
        B.hw_create(p)
    assert B.last_error()
    return ei.value.status


def test_validation_codes():
    good = W.make_spec(2, 3, [8, 8], cfl=0.9)
    p = B.make_problem(good)
    p.c = good.c
    p.dt = 1.01 * min(good.h(0), good.h(1)) / good.c
    assert _err(p) == B.HW_ECFL
    for field, val in [("d", 0), ("d", 4), ("m", 0), ("m", 7), ("method", 5), ("precision", 9),
                       ("kernel", 7), ("taylor_stages", -1)]:
        p = B.make_problem(good)
        setattr(p, field, val)
        assert _err(p) == B.HW_EINVAL, field
    p = B.make_problem(good)
    p.n[1] = 1
    assert _err(p) == B.HW_EINVAL
    # the two-kernel form serves single dissipative problems only
    p = B.make_problem(W.make_spec(2, 3, [8, 8], cfl=0.9, method=W.CONSERVATIVE), kernel=B.HW_KERNEL_SPLIT)
    assert _err(p) == B.HW_EUNSUPPORTED
    # the dense kernel serves single problems with d <= 2 only (and no BF16)
    p = B.make_problem(W.make_spec(3, 3, [4, 4, 4], cfl=0.9), kernel=B.HW_KERNEL_DENSE)
    assert _err(p) == B.HW_EUNSUPPORTED
    p = B.make_problem(W.make_spec(2, 3, [6, 6], cfl=0.9), precision=B.HW_BF16, kernel=B.HW_KERNEL_DENSE)
    assert _err(p) == B.HW_EUNSUPPORTED
    p = B.make_problem(W.make_spec(2, 6, [6, 6], cfl=0.9, method=W.CONSERVATIVE), kernel=B.HW_KERNEL_DENSE)
    assert _err(p) == B.HW_EUNSUPPORTED
    # the batched kernel serves 2-D problems in FP64 / FP32 only
    p = B.make_problem(W.make_spec(3, 2, [4, 4, 4], cfl=0.9), kernel=B.HW_KERNEL_BATCH)
    assert _err(p) == B.HW_EUNSUPPORTED
    p = B.make_problem(W.make_spec(2, 2, [6, 6], cfl=0.9), precision=B.HW_BF16, kernel=B.HW_KERNEL_BATCH)
    assert _err(p) == B.HW_EUNSUPPORTED
    p = B.make_problem(good)
    p.bc[0] = 7
    assert _err(p) == B.HW_EINVAL
    p = B.make_problem(good)
    p.xr[0] = p.xl[0]
    assert _err(p) == B.HW_EINVAL
    # the conservative method admits m = 0, the dissipative one does not
    p = B.make_problem(W.make_spec(1, 0, 8, cfl=0.9, method=W.DISS_FULL))
    assert _err(p) == B.HW_EINVAL
    # c dt == h exactly is allowed by validation (any failure is then allocation)
    p = B.make_problem(W.make_spec(2, 2, [8, 8], cfl=1.0))
    try:
        h = B.hw_create(p)
        B.hw_destroy(h)
    except B.HwError as e:
        assert e.status in (B.HW_ENOMEM, B.HW_EHIP)


def test_null_arguments():
    L = B.lib()
    assert L.hw_create(None, None) == B.HW_EINVAL
    assert L.hw_half_steps(None, 1, None) == B.HW_EINVAL
    assert L.hw_half_step_forced(None, None, 0, None) == B.HW_EINVAL
    assert L.hw_advance(None, 1, None) == B.HW_EINVAL
    assert L.hw_energy(None, None, None) == B.HW_EINVAL
    assert L.hw_state_grid(None) == -1
    L.hw_destroy(None)


def test_binding_raises_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(B.LibraryMissing):
        B.lib()
