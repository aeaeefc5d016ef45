"""GPU parity on power-law structure and for mixed precision.

Power-law graphs exercise the parts of the path that grids never reach:
rows too heavy for the sliced ELL (a wavefront per row, or a whole block
above 4096 neighbours), aggregates with more children than one block
stages in LDS, and hubs inside the one-block coarse tail.

Mixed precision (iterative refinement with an FP32 inner PCG) is checked
by what it promises: the FP64 true residual <= tol, recomputed on the host
with the oracle's L; and, on graphs small enough for a dense spectrum, the
distance to the oracle's solution at 1e-12 within the bound that any
iterate with that residual satisfies, kappa(L) * tol (on range(L):
||x - x*|| <= ||L^+|| ||r|| and ||x*|| >= ||b^|| / ||L||).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


def _hub():
    n, u, v = W.hub_graph(20000, 6000, 3000, 7)
    return n, u, v, W.uniform01_weights(len(u), 71)


def _chunglu():
    n, u, v = W.chung_lu(40000, 16.0, 2.1, 21)
    return n, u, v, W.uniform01_weights(len(u), 22)


def _oracle(n, u, v, w):
    from oracle import Graph, Hierarchy
    g = Graph(n, u, v, w)
    return g, Hierarchy(g)


def _spmv_bound(n, u, v, w, x):
    ax = np.abs(x)
    t = w * (ax[u] + ax[v])
    return 1e-15 * 16 * (np.bincount(u, t, minlength=n) + np.bincount(v, t, minlength=n))


@pytest.mark.parametrize("make", [_hub, _chunglu])
def test_spmv_heavy_rows(oracle_lib, make):
    n, u, v, w = make()
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    say("spmv heavy", n, "max degree", deg.max(), "rows > 128:", int((deg > 128).sum()))
    g, _ = _oracle(n, u, v, w)
    G = GpuLap(n, u, v, w)
    try:
        x = np.random.default_rng(3).standard_normal(n)
        y = G.apply_laplacian(x)
    finally:
        G.close()
    assert np.all(np.abs(y - g.apply(x)) <= _spmv_bound(n, u, v, w, x) + 1e-300)


@pytest.mark.parametrize("make", [_hub, _chunglu])
def test_precond_big_aggregates(oracle_lib, make):
    from oracle import MSP
    n, u, v, w = make()
    g, h = _oracle(n, u, v, w)
    G = GpuLap(n, u, v, w, mu=0.8)
    try:
        r = np.random.default_rng(4).standard_normal(n)
        r -= r.mean()
        z = G.apply_precond(r)
    finally:
        G.close()
    z0 = MSP(h, 0.8).apply(r)
    err = np.linalg.norm(z - z0) / np.linalg.norm(z0)
    tol = 1e-10 + 1e3 * np.finfo(float).eps * 0.8 ** (-2.0 * (h.nlev - 1))
    say("precond", n, "levels", h.nlev, "rel err", err, "tol", tol)
    assert err <= tol


def test_solve_hub_fp64(oracle_lib):
    from oracle import MSP, pcg
    n, u, v, w = _hub()
    g, h = _oracle(n, u, v, w)
    b = W.gaussian_rhs(n, 72)
    ref = pcg(g, b, 1e-8, 5000, MSP(h, 0.8))
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=5000)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    it, k = info["iterations"], ref.iterations
    say("hub fp64: gpu", it, "oracle", k, info)
    assert st == 0 and int(np.floor(0.70 * k)) - 1 <= it <= k + 1 + int(np.ceil(0.06 * k))
    bh = b - b.mean()
    assert np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh) <= 1.01e-8


MIXED_CASES = {
    "grid3d_16": lambda: (*W.config_graph("grid3d_128", 16 / 128), 0.8),
    "chunglu_40000": lambda: (*_chunglu(), 0.8),
    "hub_21267": lambda: (*_hub(), 0.8),
    "grid2d_64_plain": lambda: (*W.config_graph("grid2d_64"), None),
}


@pytest.mark.parametrize("name", list(MIXED_CASES))
def test_mixed_residual(oracle_lib, name):
    """FP64 true residual <= tol, on the GPU and recomputed on the host."""
    import paper_2207_07847_amd as lap
    from oracle import Graph
    n, u, v, w, mu = MIXED_CASES[name]()
    kw = dict(precision=lap.LAP_MIXED_FP32_FP64, max_iter=20000)
    if mu is None:
        kw["precond"] = lap.LAP_PREC_NONE
    else:
        kw["mu"] = mu
    b = W.gaussian_rhs(n, 81)
    G = GpuLap(n, u, v, w, **kw)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    g = Graph(n, u, v, w)
    bh = b - b.mean()
    host = np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)
    say("mixed", name, n, info, "host relres", host)
    assert st == 0 and info["relres_true"] <= 1e-8 and host <= 1.01e-8
    assert info["refinements"] >= 1
    assert abs(x.mean()) <= 1e-12 * np.abs(x).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_mixed_solution_within_kappa_bound(oracle_lib, seed):
    import paper_2207_07847_amd as lap
    from oracle import MSP, Graph, Hierarchy, pcg
    from oracle.dense import laplacian
    n, u, v = W.chung_lu(1500, 8.0, 2.1, 90 + seed)
    w = W.loguniform_weights(len(u), 91 + seed, -2.0, 2.0)
    b = W.gaussian_rhs(n, 92 + seed)
    g = Graph(n, u, v, w)
    ref = pcg(g, b, 1e-13, 20000, MSP(Hierarchy(g), 0.8))
    ev = np.linalg.eigvalsh(laplacian(n, u, v, w))
    kappa = ev[-1] / ev[1]
    G = GpuLap(n, u, v, w, mu=0.8, precision=lap.LAP_MIXED_FP32_FP64, max_iter=20000)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    diff = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    say("mixed vs oracle 1e-13:", info, "diff", diff, "kappa*tol", kappa * 1e-8)
    assert st == 0 and diff <= kappa * 1.01e-8


def test_mixed_precond_fp32(oracle_lib):
    """The FP32 preconditioner against the FP64 oracle: rounding of FP32
    coefficients and arithmetic only (relative 2-norm)."""
    import paper_2207_07847_amd as lap
    from oracle import MSP
    n, u, v, w, _ = MIXED_CASES["chunglu_40000"]()
    g, h = _oracle(n, u, v, w)
    G = GpuLap(n, u, v, w, mu=0.8, precision=lap.LAP_MIXED_FP32_FP64)
    try:
        r = np.random.default_rng(5).standard_normal(n)
        r -= r.mean()
        z = G.apply_precond(r)
    finally:
        G.close()
    z0 = MSP(h, 0.8).apply(r)
    err = np.linalg.norm(z - z0) / np.linalg.norm(z0)
    tol = 1e3 * np.finfo(np.float32).eps * 0.8 ** (-2.0 * (h.nlev - 1))
    say("fp32 precond: levels", h.nlev, "rel err", err, "tol", tol)
    assert err <= tol
