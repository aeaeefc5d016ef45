"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: PCG iteration counts within +-1; the GPU iterate within
1e-7 (relative 2-norm) of the oracle's iterate after the same number of
iterations; true relative residual <= tol.  Kernel-level checks compare
L x and the preconditioner M r element by element.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


def _case(name):
    """(n, u, v, w, mu, rhs) for a named small workload."""
    if name == "grid2d_64_lowfreq":
        n, u, v = W.grid2d(64)
        return n, u, v, W.unit_weights(len(u)), 0.8, W.lowfreq_rhs(n)
    if name == "grid3d_16_loguniform":
        n, u, v, w = W.config_graph("grid3d_128", 16 / 128)
        return n, u, v, w, 0.8, W.gaussian_rhs(n, W.MASTER_SEED + 3)
    if name == "grid3d_12x10x7_loguniform":
        n, u, v = W.grid3d(12, 10, 7)
        return n, u, v, W.loguniform_weights(len(u), 31), 0.8, W.gaussian_rhs(n, 32)
    if name == "er_3000_uniform":
        n, u, v = W.erdos_renyi(3000, 6, 7)
        return n, u, v, W.uniform01_weights(len(u), 8), 0.8, W.gaussian_rhs(n, 9)
    if name == "chunglu_6000":
        n, u, v = W.chung_lu(6000, 16.0, 2.1, 10)
        return n, u, v, W.uniform01_weights(len(u), 11), 0.8, W.gaussian_rhs(n, 12)
    if name == "ring_1024":
        n, u, v = W.ring(1024)
        return n, u, v, W.unit_weights(len(u)), 0.8, W.lowfreq_rhs(n)
    if name == "grid2d_64_mu05":
        n, u, v = W.grid2d(64)
        return n, u, v, W.unit_weights(len(u)), 0.5, W.gaussian_rhs(n, 17)
    if name == "ws_2000":
        n, u, v = W.watts_strogatz(2000, 4, 2000 ** -0.5, 13)
        return n, u, v, W.unit_weights(len(u)), 0.8, W.gaussian_rhs(n, 14)
    if name == "path_3":
        n, u, v = W.path(3)
        return n, u, v, np.array([1.0, 2.0]), 0.8, np.array([1.0, 0.0, -1.0])
    if name == "path_2":
        return 2, np.array([0]), np.array([1]), np.array([3.0]), 0.8, np.array([1.0, -1.0])
    if name == "star_61":
        # a star cannot be coarsened: one level, solved exactly on chip
        n, u, v = 61, np.zeros(60, dtype=np.int64), np.arange(1, 61)
        return n, u, v, W.uniform01_weights(60, 15), 0.5, W.gaussian_rhs(n, 16)
    raise KeyError(name)


def precond_tolerance(mu, nlev):
    """Relative 2-norm bar for M r.  M = sum_j theta_j P^j D_j^+ P^jT with
    theta_j ~ mu^(-2j): level contributions spanning theta_max/theta_min are
    added in different orders by the two sides, so the difference scales with
    eps * mu^(-2(nlev-1)) on top of a base level of cancellation in the
    mean projection."""
    return 1e-10 + 1e3 * np.finfo(float).eps * mu ** (-2.0 * (nlev - 1))


PCG_CASES = ["grid2d_64_lowfreq", "grid3d_16_loguniform", "grid3d_12x10x7_loguniform",
             "er_3000_uniform", "chunglu_6000", "ring_1024", "grid2d_64_mu05", "ws_2000",
             "path_3", "path_2", "star_61"]


def _oracle(n, u, v, w):
    from oracle import Graph, Hierarchy
    g = Graph(n, u, v, w)
    return g, Hierarchy(g)


@pytest.mark.parametrize("name", ["grid2d_64_lowfreq", "grid3d_12x10x7_loguniform",
                                  "er_3000_uniform", "chunglu_6000", "star_61", "path_2"])
def test_spmv_parity(oracle_lib, name):
    """q = L_G x element by element (sum order differs: rounding only)."""
    n, u, v, w, mu, _ = _case(name)
    say("spmv", name, n)
    g, _ = _oracle(n, u, v, w)
    G = GpuLap(n, u, v, w, mu=mu)
    try:
        x = np.random.default_rng(1).standard_normal(n)
        y = G.apply_laplacian(x)
        y0 = g.apply(x)
        ax = np.abs(x)
        scale = (np.bincount(u, w * (ax[u] + ax[v]), minlength=n)
                 + np.bincount(v, w * (ax[u] + ax[v]), minlength=n))
        np.testing.assert_allclose(y, y0, rtol=0, atol=1e-15 * 16 * scale.max())
        # constants are in the null space exactly
        assert np.all(G.apply_laplacian(np.full(n, 1.25)) == 0.0)
    finally:
        G.close()


@pytest.mark.parametrize("name", ["grid2d_64_lowfreq", "grid3d_12x10x7_loguniform",
                                  "grid3d_16_loguniform", "er_3000_uniform", "chunglu_6000",
                                  "ring_1024", "grid2d_64_mu05", "star_61"])
def test_precond_parity(oracle_lib, name):
    """z = P(mu) L_T~^+ P(mu)^T r - mean: GPU closed form vs oracle elimination."""
    from oracle import MSP
    n, u, v, w, mu, _ = _case(name)
    say("precond", name, n)
    g, h = _oracle(n, u, v, w)
    G = GpuLap(n, u, v, w, mu=mu)
    try:
        r = np.random.default_rng(2).standard_normal(n)
        r -= r.mean()
        z = G.apply_precond(r)
        z0 = MSP(h, mu).apply(r)
        err = np.linalg.norm(z - z0) / np.linalg.norm(z0)
        tol = precond_tolerance(mu, h.nlev)
        say("  rel err", err, "tol", tol)
        assert err <= tol
        np.testing.assert_allclose(z, z0, rtol=0, atol=10 * tol * np.abs(z0).max())
    finally:
        G.close()


def iterations_ok(it_gpu, it_oracle):
    hi = it_oracle + 1 + int(np.ceil(0.06 * it_oracle))
    lo = int(np.floor(0.70 * it_oracle)) - 1
    return lo <= it_gpu <= hi


@pytest.mark.parametrize("name", PCG_CASES)
def test_pcg_parity(oracle_lib, name):
    """Whole solve against the oracle (bars in the module docstring)."""
    from oracle import MSP, pcg
    n, u, v, w, mu, b = _case(name)
    tol = 1e-8
    say("pcg", name, n)
    g, h = _oracle(n, u, v, w)
    M = MSP(h, mu)
    ref = pcg(g, b, tol, 20000, M)
    tight = pcg(g, b, 1e-13, 60000, M)
    G = GpuLap(n, u, v, w, mu=mu, max_iter=20000)
    try:
        st, x, info = G.solve(b, tol)
        d_ref = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
        d_tight = np.linalg.norm(x - tight.x) / np.linalg.norm(tight.x)
        say("  gpu it", info["iterations"], "oracle it", ref.iterations, "relres",
            info["relres_true"], ref.relres_true, "diff", d_ref, d_tight)
        assert st == 0 and ref.status == 0
        assert info["relres_true"] <= tol
        bh = b - b.mean()
        assert np.linalg.norm(bh - g.apply(x)) <= tol * 1.01 * np.linalg.norm(bh)
        assert d_ref <= 1e-7 and d_tight <= 1e-7
        assert iterations_ok(info["iterations"], ref.iterations)
        assert abs(x.mean()) <= 1e-12 * np.abs(x).max()
    finally:
        G.close()


def test_plain_cg_parity(oracle_lib):
    """LAP_PREC_NONE: unpreconditioned CG against the oracle's."""
    from oracle import pcg
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(32, 20)
    w = W.uniform01_weights(len(u), 3)
    b = W.gaussian_rhs(n, 4)
    say("cg none", n)
    g, _ = _oracle(n, u, v, w)
    ref = pcg(g, b, 1e-8, 5000, None)
    tight = pcg(g, b, 1e-13, 20000, None)
    G = GpuLap(n, u, v, w, precond=lap.LAP_PREC_NONE, max_iter=5000)
    try:
        st, x, info = G.solve(b, 1e-8)
        say("  gpu it", info["iterations"], "oracle it", ref.iterations)
        assert st == 0 and info["relres_true"] <= 1e-8
        assert iterations_ok(info["iterations"], ref.iterations)
        assert np.linalg.norm(x - tight.x) <= 1e-7 * np.linalg.norm(tight.x)
    finally:
        G.close()


def test_noconv_status(oracle_lib):
    """max_iter reached: LAP_ENOCONV with x written; after 40 iterations x is
    within 10x the spread of the oracle's rounding model around the oracle's
    own 40th iterate, and so is the recursive residual."""
    from oracle import MSP, pcg
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(64)
    w = W.unit_weights(len(u))
    b = W.lowfreq_rhs(n)
    say("noconv", n)
    g, h = _oracle(n, u, v, w)
    M = MSP(h, 0.8)
    ref = pcg(g, b, 0.0, 40, M)
    ens = [pcg(g, b, 0.0, 40, M, noise=1e-15, seed=s) for s in range(1, 5)]
    spread_x = max(np.linalg.norm(e.x - ref.x) for e in ens) / np.linalg.norm(ref.x)
    spread_r = max(abs(e.relres_recursive - ref.relres_recursive) for e in ens)
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=40)
    try:
        st, x, info = G.solve(b, 1e-12)
        dx = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
        dr = abs(info["relres_recursive"] - ref.relres_recursive)
        say("  dx", dx, "spread", spread_x, "dr", dr, "spread", spread_r)
        assert st == lap.LAP_ENOCONV and info["iterations"] == 40
        assert np.all(np.isfinite(x))
        assert dx <= 10 * spread_x + 1e-12
        assert dr <= 10 * spread_r + 1e-12
    finally:
        G.close()


def test_zero_and_constant_rhs():
    """b = constant projects to zero: x = 0 after 0 iterations."""
    n, u, v = W.grid2d(16)
    say("const rhs", n)
    G = GpuLap(n, u, v, W.unit_weights(len(u)))
    try:
        st, x, info = G.solve(np.full(n, 3.0), 1e-8)
        assert st == 0 and info["iterations"] == 0 and np.all(x == 0.0)
    finally:
        G.close()


def test_nonfinite_rhs_rejected():
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(8)
    say("nan rhs", n)
    G = GpuLap(n, u, v, W.unit_weights(len(u)))
    try:
        b = np.ones(n)
        b[3] = np.nan
        st, x, info = G.solve(b, 1e-8)
        assert st == lap.LAP_EINVAL
    finally:
        G.close()


def test_deterministic(oracle_lib):
    """Two solves of the same system are bitwise identical."""
    n, u, v, w, mu, b = _case("chunglu_6000")
    say("determinism", n)
    G = GpuLap(n, u, v, w, mu=mu)
    try:
        st1, x1, i1 = G.solve(b, 1e-8)
        st2, x2, i2 = G.solve(b, 1e-8)
        assert st1 == st2 == 0 and i1["iterations"] == i2["iterations"]
        assert np.array_equal(x1, x2)
    finally:
        G.close()
