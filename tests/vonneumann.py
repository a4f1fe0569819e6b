"""Von Neumann analysis of the dissipative half step, built from the FP64 oracle.

A half step of the dissipative method (Sec. 3.1.2, Sec. 3.3) is linear and the same in
every cell: the data at an output node is a fixed linear map of the data at the 2^d
corners of its cell.  Writing T_s for the block that carries corner s (s in {0,1}^d,
corner position x_c + (s - 1/2) h) to the output node, a Fourier mode with data
exp(i theta . j) at node j leaves the half step as the same mode multiplied by the
symbol

    G(theta) = sum_s T_s exp(i theta . (s - 1/2)),

a matrix on one node's [u, v] coefficients.  On a periodic grid both half steps apply
the same map, so the scheme is stable iff the spectral radius of G(theta) is at most one
for every theta (Sec. 3.2 states the method is stable up to c dt = h for all orders).

The blocks T_s are read off the oracle: one oracle half step on a one-cell box (no walls
are involved in the primal-to-dual direction) per unit corner coefficient.  Nothing here
uses the GPU library.

Run ``python tests/vonneumann.py`` for the full table (variant, series, d, m, lambda).
"""
from __future__ import annotations

import itertools
import os
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

import oracle  # noqa: E402


def cell_blocks(d, m, lam, method=oracle.DISS_FULL, taylor_stages=0):
    """T[s] (2^d blocks, each n_state x n_state, s in the order of
    itertools.product((0, 1), repeat=d) with s[0] the x corner) of the half step with
    h = 1 in every dimension, c = 1 and dt = lam.  The state vector of a node is its
    (m+1)^d u coefficients followed by its m^d v coefficients."""
    Mu, Mv = (m + 1) ** d, m ** d
    ns = Mu + Mv
    p = oracle.make_problem(d, m, [1] * d, 0.0, 1.0, 1.0, lam, [oracle.DIRICHLET] * d, method,
                            taylor_stages=taylor_stages)
    n_in = oracle.nodes(p, oracle.PRIMAL)  # 2^d primal nodes of the one-cell box
    assert n_in == 2 ** d
    T = np.zeros((2 ** d, ns, ns))
    for corner in range(n_in):
        # primal node index corner = s0 + 2 (s1 + 2 s2): its position bits are s
        s = [(corner >> i) & 1 for i in range(d)]
        k = 0
        for i in range(d):
            k += s[i] << (d - 1 - i)  # index in itertools.product order (s[0] slowest)
        for j in range(ns):
            u = np.zeros((n_in, Mu))
            v = np.zeros((n_in, Mv))
            if j < Mu:
                u[corner, j] = 1.0
            else:
                v[corner, j - Mu] = 1.0
            uo, vo = oracle.diss_half(p, oracle.DUAL, u, v)
            T[k, :Mu, j] = uo[0]
            T[k, Mu:, j] = vo[0]
    return T


def theta_grid(d, npts):
    """npts points per dimension (npts even), theta_k = -pi + 2 pi k / npts: the grid holds
    theta_i = 0 and -pi in every dimension, so the lower-dimensional modes (theta_i = 0 for
    some i) are on it.  theta = 0 itself (the constant data, whose mean-velocity mode has
    a Jordan block at eigenvalue 1) is left out.  G(-theta) is the complex conjugate of
    G(theta) (the blocks are real), so of each pair (theta, -theta) only one is kept."""
    assert npts % 2 == 0
    ks = np.array(list(itertools.product(range(npts), repeat=d)))
    mirror = (npts - ks) % npts
    origin = npts // 2
    keep = [tuple(k) <= tuple(mk) and any(x != origin for x in k) for k, mk in zip(ks, mirror)]
    return -np.pi + 2.0 * np.pi * ks[np.array(keep)] / npts


def max_growth(T, d, npts, chunk=512):
    """max over the theta grid of the spectral radius of G(theta), minus one."""
    corners = np.array(list(itertools.product((0, 1), repeat=d)), dtype=np.float64) - 0.5
    thetas = theta_grid(d, npts)
    worst = -np.inf
    for a in range(0, len(thetas), chunk):
        th = thetas[a:a + chunk]
        ph = np.exp(1j * th @ corners.T)               # (n_theta, 2^d)
        G = np.einsum("ts,sij->tij", ph, T.astype(np.complex128))
        rho = np.abs(np.linalg.eigvals(G)).max(axis=1)
        worst = max(worst, float(rho.max()))
    return worst - 1.0


def growth(d, m, lam, variant="full", series="exact", npts=None):
    """max |g| - 1 for one (d, m, lambda, variant, series); series "exact" runs the Taylor
    series to its last non-zero stage, "2m+1" / "2m+2" keep stages 0..2m+1 / 0..2m+2."""
    method = oracle.DISS_FULL if variant == "full" else oracle.DISS_SIMPLE
    stages = {"exact": 0, "2m+1": 2 * m + 1, "2m+2": 2 * m + 2}[series]
    if npts is None:
        npts = {1: 120, 2: 60, 3: 12}[d]
    return max_growth(cell_blocks(d, m, lam, method, stages), d, npts)


def main(argv):
    """argv: optional d and variant to restrict the table (e.g. ``2 full``)."""
    lams = (0.5, 0.8, 0.9, 0.95, 1.0)
    dims = [int(argv[0])] if argv else [2, 3]
    variants = [argv[1]] if len(argv) > 1 else ["full", "simple"]
    print(f"{'d':>2} {'variant':>7} {'series':>6} {'m':>2} " + " ".join(f"lam={x:<6}" for x in lams))
    for d, mmax in ((2, 6), (3, 4)):
        if d not in dims:
            continue
        for variant in variants:
            for series in ("exact", "2m+1", "2m+2"):
                for m in range(1, mmax + 1):
                    row = [growth(d, m, lam, variant, series) for lam in lams]
                    print(f"{d:>2} {variant:>7} {series:>6} {m:>2} " + " ".join(f"{g:+.1e}  " for g in row),
                          flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
