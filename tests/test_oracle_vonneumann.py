"""Von Neumann stability of the dissipative method, from the oracle's own cell map.

The symbol G(theta) = sum_s T_s exp(i theta . (s - 1/2)) of one half step (the blocks
T_s read off the oracle on a one-cell box, `vonneumann.py`) has spectral radius at most
one for every theta iff the periodic scheme is stable.  Sec. 3.2 proves stability up to
c dt = h for all m in 1-D; Sec. 3.3 introduces the modified first step ("full" variant)
because the straightforward multi-dimensional extension ("simple") is reported unstable
at full CFL, and the GPU kernels of Sec. 6.1 cut the Taylor series after 2m+2 stages.

Measured here (60^2 theta grid in 2-D, 12^3 in 3-D, both holding the axis planes;
theta = 0 excluded), growth per half step:
* 1-D, both variants coincide: max|g| = 1 to round-off for m <= 6 at c dt / h = 1;
* full variant, exact series: stable for m <= 3 at every c dt <= h (2-D, and 3-D with
  the benchmark's m = 3), but not at high m near c dt = h: 2-D m = 4 at 1 grows by
  2.4e-6, m = 5 at 0.95 by 2.0e-3, m = 6 at 0.9 by 9.4e-4; 3-D m = 4 at 1 by 1.1e-3;
* simple variant, exact series: stable for every m <= 6 in 2-D at c dt = h;
* series cut after stage 2m+1 (2m+2 stages counting s = 0): unstable near c dt = h, the
  simple variant already at m = 1 (c dt / h = 0.9: +1.6e-3), and +0.16 (simple, m = 3,
  0.8) and +0.23 (full, m = 3, 0.9).
"""
import pytest

threadpoolctl = pytest.importorskip("threadpoolctl")

import vonneumann as vn  # noqa: E402


@pytest.fixture(autouse=True)
def _one_blas_thread():
    # many small eigenproblems: one thread each is fastest
    with threadpoolctl.threadpool_limits(1):
        yield


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
def test_1d_stable_at_cfl_one_every_order(m):
    assert vn.growth(1, m, 1.0) <= 1e-12


@pytest.mark.parametrize("m,lam", [(1, 1.0), (2, 1.0), (3, 0.8), (3, 1.0), (4, 0.95)])
def test_2d_full_exact_stable_low_order(m, lam):
    assert vn.growth(2, m, lam, "full", "exact") <= 1e-12


@pytest.mark.parametrize("lam", [0.9, 1.0])
def test_3d_full_exact_stable_at_benchmark_config(lam):
    """The 3-D benchmark method (m = 3, c dt / h = 0.9) and c dt = h."""
    assert vn.growth(3, 3, lam, "full", "exact") <= 1e-12


@pytest.mark.parametrize("m,lam,lo,hi", [(4, 1.0, 1.5e-6, 4.0e-6), (5, 0.95, 1.5e-3, 2.5e-3),
                                         (6, 0.9, 7.0e-4, 1.2e-3), (5, 1.0, 6.0e-3, 1.0e-2)])
def test_2d_full_exact_unstable_high_order_near_cfl_one(m, lam, lo, hi):
    """A weak unstable band at high m: the modified first step does not keep the method
    stable to c dt = h for every order in 2-D."""
    g = vn.growth(2, m, lam, "full", "exact")
    assert lo <= g <= hi, g


@pytest.mark.parametrize("m", [3, 6])
def test_2d_simple_exact_stable_at_cfl_one(m):
    assert vn.growth(2, m, 1.0, "simple", "exact") <= 1e-12


@pytest.mark.parametrize("variant,m,lam,lo,hi", [("simple", 1, 0.9, 1.2e-3, 2.0e-3),
                                                 ("simple", 3, 0.8, 0.12, 0.2),
                                                 ("full", 3, 0.9, 0.18, 0.28)])
def test_2d_truncated_series_unstable(variant, m, lam, lo, hi):
    g = vn.growth(2, m, lam, variant, "2m+1")
    assert lo <= g <= hi, g


def test_2d_truncated_series_one_stage_more_is_stable_there():
    """Keeping stage 2m+2 as well restores stability at those points."""
    assert vn.growth(2, 1, 0.9, "simple", "2m+2") <= 1e-12
    assert vn.growth(2, 3, 0.8, "simple", "2m+2") <= 1e-12
    assert vn.growth(2, 3, 0.9, "full", "2m+2") <= 1e-12


def test_symbol_of_exact_polynomial_step_is_translation():
    """Sanity of the symbol itself: in 1-D at c dt = h the dissipative method is exact
    for every wave moving at speed c, so the eigenvalues of G on the physical modes lie
    on the unit circle."""
    import numpy as np
    import itertools
    T = vn.cell_blocks(1, 2, 1.0)
    corners = np.array(list(itertools.product((0, 1), repeat=1)), dtype=float) - 0.5
    for th in (0.3, 1.1, 2.5):
        G = sum(T[k] * np.exp(1j * th * corners[k, 0]) for k in range(2))
        ev = np.abs(np.linalg.eigvals(G))
        assert np.isclose(ev.max(), 1.0, atol=1e-12)
