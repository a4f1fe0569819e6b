"""The dense kernel's cell matrix (host code, cellmap.cpp) checked on the CPU: applied
to the corner data of a single cell it must reproduce the oracle's half step, and it
must have the reflection symmetry the kernel relies on (the rows of corner (s_0, s_1)
equal corner 0's rows times (-1)^(sum_i s_i (a_i + l_i)), exactly)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1802_05246_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1802_05246_amd", "csrc")


@pytest.fixture(scope="module")
def dump(tmp_path_factory):
    gxx = shutil.which("g++")
    hip_inc = "/opt/rocm/include"
    if gxx is None or not os.path.isdir(hip_inc):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("cellmap") / "cellmap_dump")
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I", CSRC, "-I", hip_inc,
                           os.path.join(ROOT, "tests", "cellmap_dump.cpp"), os.path.join(CSRC, "cellmap.cpp"),
                           "-o", exe])

    def run(d, m, method, c, dt, h, stages):
        args = [exe, str(d), str(m), str(method), repr(c), repr(dt), repr(h[0]),
                repr(h[1] if len(h) > 1 else 1.0), str(stages)]
        out = subprocess.check_output(args, text=True).split()
        n_in, n_out = int(out[0]), int(out[1])
        return np.array(out[2:], dtype=np.float64).reshape(n_in, n_out)
    return run


CASES = [(1, 1, W.DISS_FULL, 0), (1, 4, W.DISS_FULL, 0), (1, 6, W.DISS_SIMPLE, 0), (1, 3, W.DISS_FULL, 5),
         (1, 0, W.CONSERVATIVE, 0), (1, 5, W.CONSERVATIVE, 0),
         (2, 1, W.DISS_FULL, 0), (2, 3, W.DISS_FULL, 0), (2, 3, W.DISS_SIMPLE, 0), (2, 5, W.DISS_FULL, 0),
         (2, 2, W.DISS_FULL, 6), (2, 6, W.DISS_SIMPLE, 0),
         (2, 0, W.CONSERVATIVE, 0), (2, 4, W.CONSERVATIVE, 0), (2, 5, W.CONSERVATIVE, 0)]


@pytest.mark.parametrize("d,m,method,stages", CASES)
def test_cell_matrix_reproduces_the_oracle_half_step(dump, d, m, method, stages):
    # one periodic cell of two nodes per dimension: the output node 0 of the dual grid has
    # the primal nodes (s_0, s_1) as its corners, node index s_0 + 2 s_1 = corner index
    spec = W.make_spec(d, m, [2] * d, 0.0, [1.0, 0.8][:d], 1.3, cfl=0.85, bc=W.PERIODIC, method=method,
                       taylor_stages=stages)
    p = oracle.make_problem(spec.d, spec.m, spec.n, spec.xl, spec.xr, spec.c, spec.dt, spec.bc, spec.method,
                            spec.taylor_stages)
    G = dump(d, m, method, spec.c, spec.dt, [spec.h(i) for i in range(d)], stages)
    rng = np.random.default_rng(11 + 7 * d + m)
    nu = (m + 1) ** d
    u = rng.uniform(-1, 1, (2 ** d, nu))
    if method == W.CONSERVATIVE:
        x = u.reshape(-1)
        old = np.zeros((2 ** d, nu))
        out = oracle.cons_half(p, W.DUAL, u, old, sel=[0])[0]
        ref = 0.5 * out  # u_new = 2 S - u_old with u_old = 0
    else:
        v = rng.uniform(-1, 1, (2 ** d, m ** d))
        x = np.concatenate([np.concatenate([u[c], v[c]]) for c in range(2 ** d)])
        ou, ov = oracle.diss_half(p, W.DUAL, u, v, sel=[0])
        ref = np.concatenate([ou[0], ov[0]])
    got = G.T @ x
    assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)) * np.max(np.abs(G)))


@pytest.mark.parametrize("d,m,method,stages", CASES)
def test_cell_matrix_reflection_symmetry(dump, d, m, method, stages):
    G = dump(d, m, method, 1.0, 0.74, [0.74 / 0.9, 0.74 / 0.77], stages)
    M = m + 1
    nu, nv = M ** d, (0 if method == W.CONSERVATIVE else m ** d)
    ni = nu + nv
    n_out = G.shape[1]
    a_par = np.zeros((d, n_out), dtype=int)
    for o in range(n_out):
        mo, oo = (M, o) if o < nu else (m, o - nu)
        a_par[0, o] = oo % mo
        if d > 1:
            a_par[1, o] = oo // mo
    for c in range(1, 2 ** d):
        for l in range(ni):
            md, ll = (M, l) if l < nu else (m, l - nu)
            lidx = [ll % md, ll // md]
            e = np.zeros(n_out, dtype=int)
            for i in range(d):
                e += ((c >> i) & 1) * (a_par[i] + lidx[i])
            assert np.array_equal(G[c * ni + l], np.where(e % 2 == 1, -G[l], G[l]))


@pytest.mark.parametrize("n_tiles", [1, 5, 8, 9, 63, 1000, 4097])
@pytest.mark.parametrize("grid", [1, 3, 8, 13, 2048])
def test_batch_kernel_walk_covers_every_tile_once(n_tiles, grid):
    """The persistent batched dense kernel's XCD-aware walk (workgroup b takes the chunk of
    XCD b mod 8, stepping by the number of workgroups on that chunk; the index arithmetic
    of k_dense_list) visits every tile exactly once."""
    seen = np.zeros(n_tiles, dtype=np.int64)
    nx = min(grid, 8)
    chunk = (n_tiles + nx - 1) // nx
    for b in range(grid):
        xcd, slot = b % nx, b // nx
        per = (grid + nx - 1 - xcd) // nx
        t0, t1 = xcd * chunk, min(n_tiles, xcd * chunk + chunk)
        for t in range(t0 + slot, t1, per):
            seen[t] += 1
    assert (seen == 1).all()
