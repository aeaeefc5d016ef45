"""GPU checks at the benchmark's full size: 3D 7-point grid 128^3 with
weights 10^U(-3,3), MSP mu = 0.8, in the launch configuration bench.py
times.  Every step is checked on its own (hierarchy outputs bit for bit,
L x and M r element by element), and the whole solve against the
oracle's own full solve, stored by tests/golden/make_grid3d_golden.py
(about 3.5 hours of one host core): the iteration count within the band
of the oracle's FP64 variants (test_gpu_grid3d_family.py says why a band),
the converged solution at a sample of 4096 vertices within 1e-7, and the
FP64 residual recomputed on the host with the oracle's L."""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def full():
    from oracle import Graph, Hierarchy
    n, u, v, w = W.config_graph("grid3d_128")
    b = W.gaussian_rhs(n, W.MASTER_SEED + 3)
    say("fullsize: oracle graph + hierarchy", n, len(u))
    g = Graph(n, u, v, w)
    h = Hierarchy(g)
    say("fullsize: gpu setup")
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=200000)
    yield dict(n=n, u=u, v=v, w=w, b=b, g=g, h=h, G=G)
    G.close()


def test_fullsize_hierarchy_bit_exact(oracle_lib, full):
    import paper_2207_07847_amd as lap
    G, h = full["G"], full["h"]
    assert G.info["sizes"] == h.sizes
    for k in range(h.nlev - 1):
        a, m = lap.lap_export_level(G.h, k, h.sizes[k])
        a2, m2 = h.agg(k)
        assert np.array_equal(a, a2) and np.array_equal(m, m2), k


def test_fullsize_spmv(oracle_lib, full):
    say("fullsize: spmv")
    n, u, v, w, g, G = (full[k] for k in ("n", "u", "v", "w", "g", "G"))
    x = np.random.default_rng(5).standard_normal(n)
    y = G.apply_laplacian(x)
    y0 = g.apply(x)
    ax = np.abs(x)
    scale = (np.bincount(u, w * (ax[u] + ax[v]), minlength=n)
             + np.bincount(v, w * (ax[u] + ax[v]), minlength=n))
    assert np.all(np.abs(y - y0) <= 1e-15 * 16 * scale + 1e-300)


def test_fullsize_precond(oracle_lib, full):
    from oracle import MSP
    say("fullsize: oracle MSP factor")
    n, h, G = full["n"], full["h"], full["G"]
    r = np.random.default_rng(6).standard_normal(n)
    r -= r.mean()
    z0 = MSP(h, 0.8).apply(r)
    say("fullsize: gpu precond")
    z = G.apply_precond(r)
    err = np.linalg.norm(z - z0) / np.linalg.norm(z0)
    tol = 1e-10 + 1e3 * np.finfo(float).eps * 0.8 ** (-2.0 * (h.nlev - 1))
    say("  rel err", err, "tol", tol)
    assert err <= tol
    np.testing.assert_allclose(z, z0, rtol=0, atol=10 * tol * np.abs(z0).max())


def test_fullsize_solve(oracle_lib, full):
    from test_gpu_grid3d_family import check_solve
    say("fullsize: gpu solve")
    b, g, G = full["b"], full["g"], full["G"]
    st, x, info = G.solve(b, 1e-8)
    say("  ", info)
    assert st == 0 and info["relres_true"] <= 1e-8
    check_solve(128, st, x, info)
    bh = b - b.mean()
    rel = np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)
    say("  host relres", rel)
    assert rel <= 1.01e-8
    assert abs(x.mean()) <= 1e-12 * np.abs(x).max()
