"""Stability of the dissipative variants measured through the library (the study of
paper_1802_05246_amd.stability): growth per full step of the fluctuations of random
periodic data.  Sec. 3.3 (variants), Sec. 6.1 (the truncated series of the paper's
GPU kernels)."""
import pytest

from helpers import oracle_growth_per_step
from paper_1802_05246_amd import workloads as W

pytestmark = pytest.mark.gpu


def _g(*a, **k):
    from paper_1802_05246_amd.stability import growth_per_step
    return growth_per_step(*a, **k)


@pytest.mark.parametrize("d,m,lam", [(2, 1, 1.0), (2, 2, 1.0), (2, 3, 0.9), (2, 3, 1.0), (2, 4, 1.0),
                                     (3, 1, 1.0), (3, 2, 1.0), (3, 3, 0.9), (3, 3, 1.0)])
def test_full_exact_series_stable(d, m, lam):
    n = 8 if d == 2 else 6
    assert _g(d, m, lam, "full", "exact", n=n) <= 1.0 + 1e-4


@pytest.mark.parametrize("d,m", [(2, 1), (2, 3), (2, 5), (2, 6), (3, 1), (3, 2), (3, 3)])
def test_simple_exact_series_stable_at_cfl_one(d, m):
    n = 8 if d == 2 else 6
    assert _g(d, m, 1.0, "simple", "exact", n=n) <= 1.0 + 1e-4


def test_full_exact_series_m5_grows_at_cfl_one():
    assert _g(2, 5, 1.0, "full", "exact", n=8) > 1.0 + 1e-3


def test_simple_series_cut_after_stage_2m_plus_1_grows():
    assert _g(2, 3, 0.8, "simple", "2m+1", n=12) > 1.1
    assert _g(2, 3, 0.8, "simple", "2m+2", n=12) < 1.0


@pytest.mark.parametrize("d,m,lam,variant,stages,n", [(2, 5, 1.0, W.DISS_FULL, 0, 8),
                                                       (2, 3, 0.8, W.DISS_SIMPLE, 7, 12),
                                                       (3, 3, 1.0, W.DISS_FULL, 0, 4)])
def test_growth_matches_oracle(d, m, lam, variant, stages, n):
    """The same linear map on the same data: the measured growth agrees with the
    oracle's to round-off."""
    from paper_1802_05246_amd.stability import growth_per_step
    name = "full" if variant == W.DISS_FULL else "simple"
    series = {0: "exact", 2 * m + 1: "2m+1", 2 * m + 2: "2m+2"}[stages]
    g_gpu = growth_per_step(d, m, lam, name, series, n=n, steps=60)
    g_cpu = oracle_growth_per_step(d, m, lam, variant, taylor_stages=stages, n=n, steps=60)
    assert abs(g_gpu - g_cpu) <= 1e-9 * g_cpu, (g_gpu, g_cpu)
