"""GPU checks at the full sizes of the two power-law workloads, in the
launch configurations bench.py times:

  * Chung-Lu, 4M ids, mean degree 16, exponent 2.1, weights U(0,1], largest
    component (3.9M vertices, 31.6M edges), MSP mu = 0.8, level = max, one
    Gaussian right-hand side, FP64 and mixed FP32/FP64 (Sec. 3.3, Sec. 4);
  * R-MAT scale 20, (0.57, 0.19, 0.19, 0.05), largest component (646K
    vertices, 15.7M edges), 64 right-hand sides e_i - e_j, the block solve
    in mixed precision.

The oracle's hierarchy and solve take minutes to hours at these sizes, so
each step is checked where an independent answer is cheap: L x element by
element against the oracle's L; the preconditioner through properties the
MSP has at any size (Sec. 3.1: M is symmetric and positive definite on
mean-free vectors, and its output is mean-free); every solve through the
FP64 residual of the original system recomputed on the host with the
oracle's L (the stop rule of Sec. 4), and a mean-free x.  The same steps
are compared with the oracle value by value at sizes it finishes in
seconds (test_gpu_parity.py, test_gpu_powerlaw_mixed.py, test_gpu_block.py).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def chunglu():
    from oracle import Graph
    n, u, v, w = W.config_graph("chunglu_4m")
    b = W.gaussian_rhs(n, W.MASTER_SEED + 3)
    say("fullsize chunglu_4m: oracle graph", n, len(u))
    g = Graph(n, u, v, w)
    say("fullsize chunglu_4m: gpu setup")
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=20000)
    yield dict(n=n, u=u, v=v, w=w, b=b, g=g, G=G)
    G.close()


def _spmv_scale_and_factor(n, u, v, w, x):
    """Per row: S = sum_j w_ij (|x_i| + |x_j|) and the factor f with the bar
    |delta| <= f eps S.  A d-term sum of terms that carry two roundings each
    errs by at most about (d + 2) u S (u = eps / 2) in any order; two such
    sums differ by twice that, and f = 2 (d + 4) leaves a margin of 2.  f is
    never below 72 (16e-15 / eps), the fixed bar of the smaller SpMV tests,
    which assumes short rows; hub rows here hold up to 1e5 terms."""
    ax = np.abs(x)
    s = w * (ax[u] + ax[v])
    S = np.bincount(u, s, minlength=n) + np.bincount(v, s, minlength=n)
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    f = np.maximum(2.0 * (deg + 4), 16e-15 / np.finfo(float).eps)
    return S, f, deg


def _host_relres(g, b, x):
    bh = b - b.mean()
    return np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)


def test_chunglu_spmv(oracle_lib, chunglu):
    n, u, v, w, g, G = (chunglu[k] for k in ("n", "u", "v", "w", "g", "G"))
    x = np.random.default_rng(5).standard_normal(n)
    say("fullsize chunglu_4m: spmv")
    y = G.apply_laplacian(x)
    S, f, deg = _spmv_scale_and_factor(n, u, v, w, x)
    ratio = np.abs(y - g.apply(x)) / (np.finfo(float).eps * S + 1e-300)
    worst = int(np.argmax(ratio / f))
    msg = (f"worst row {worst}: degree {deg[worst]}, |delta| = {ratio[worst]:.1f} eps S "
           f"(bar {f[worst]:.0f}); max degree {deg.max()}, largest |delta| / (eps S) "
           f"{ratio.max():.1f}")
    say("  ", msg)
    assert np.all(ratio <= f), msg


def test_chunglu_precond_properties(oracle_lib, chunglu):
    n, G = chunglu["n"], chunglu["G"]
    rng = np.random.default_rng(6)
    r1, r2 = rng.standard_normal(n), rng.standard_normal(n)
    r1 -= r1.mean()
    r2 -= r2.mean()
    say("fullsize chunglu_4m: precond")
    z1, z2 = G.apply_precond(r1), G.apply_precond(r2)
    # mean-free output
    for z in (z1, z2):
        assert abs(z.sum()) <= 1e-10 * np.abs(z).sum()
    # symmetric: r1.(M r2) = r2.(M r1), with the rounding of two n-term sums
    a, c = r1 @ z2, r2 @ z1
    scale = np.abs(r1) @ np.abs(z2) + np.abs(r2) @ np.abs(z1)
    say("  r1.Mr2", a, "r2.Mr1", c, "scale", scale)
    assert abs(a - c) <= 1e-10 * scale
    # positive on mean-free vectors
    assert r1 @ z1 > 0 and r2 @ z2 > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_chunglu_solve(oracle_lib, chunglu, precision):
    import paper_2207_07847_amd as lap
    n, u, v, w, b, g = (chunglu[k] for k in ("n", "u", "v", "w", "b", "g"))
    if precision == "fp64":
        G, own = chunglu["G"], False
    else:
        say("fullsize chunglu_4m: gpu setup (mixed)")
        G = GpuLap(n, u, v, w, mu=0.8, precision=lap.LAP_MIXED_FP32_FP64, max_iter=20000)
        own = True
    try:
        say(f"fullsize chunglu_4m: {precision} solve")
        st, x, info = G.solve(b, 1e-8)
    finally:
        if own:
            G.close()
    rel = _host_relres(g, b, x)
    msg = f"chunglu_4m {precision}: status {st}, {info}, host relres {rel:.3e}"
    say("  ", msg)
    assert st == 0 and info["relres_true"] <= 1e-8, msg
    assert rel <= 1.01e-8, msg
    assert abs(x.mean()) <= 1e-12 * np.abs(x).max(), msg


def test_rmat_block_solve(oracle_lib):
    import paper_2207_07847_amd as lap
    from oracle import Graph
    n, u, v, w = W.config_graph("rmat_20")
    B = W.pair_rhs(n, 64, W.MASTER_SEED + 6)
    say("fullsize rmat_20: oracle graph", n, len(u))
    g = Graph(n, u, v, w)
    say("fullsize rmat_20: gpu setup (block, mixed)")
    G = GpuLap(n, u, v, w, mu=0.8, precision=lap.LAP_MIXED_FP32_FP64, max_iter=20000,
               flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        say("fullsize rmat_20: block solve, 64 columns")
        st, X, info = G.solve_many(B, 1e-8)
    finally:
        G.close()
    rel = np.array([_host_relres(g, b, x) for b, x in zip(B, X)])
    its = [i["iterations"] for i in info]
    msg = (f"rmat_20 block: status {st}, iterations {min(its)}-{max(its)}, "
           f"worst relres true {max(i['relres_true'] for i in info):.3e}, host {rel.max():.3e}")
    say("  ", msg)
    assert st == 0 and all(i["status"] == 0 and i["relres_true"] <= 1e-8 for i in info), msg
    assert rel.max() <= 1.01e-8, msg
    assert np.all(np.abs(X.mean(axis=1)) <= 1e-12 * np.abs(X).max(axis=1)), msg
