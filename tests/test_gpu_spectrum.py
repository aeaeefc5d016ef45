"""GPU spectrum estimate (lap_estimate_spectrum) and choice of mu
(lap_select_mu) against the oracle's (oracle/lanczos.py).

Both run PCG from x = 0 on the same b and build the Lanczos tridiagonal
from its coefficients, and both stop at the relative residual 1e-10 (within
one step of each other).  Their PCG coefficients agree to rounding.  Ritz
values that have converged then agree closely; one that has not (lambda_min
after 40 steps at kappa ~ 1e3) moves with the rounding of every step, by
more than 1e-5 relative under noise at the preconditioner's own parity level.
So parity is checked on runs to the 1e-10 stop, where both extremes have
converged; a short run is checked to lie inside the converged interval
(Ritz values approach the extremes from inside), and against the dense
pencil spectrum the GPU finds the isolated extremes.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


def _oracle_estimate(n, u, v, w, b, precond, mu, steps):
    from oracle import MSP, Graph, Hierarchy
    from oracle.lanczos import spectrum_estimate
    from oracle.pegp import PEGP
    g = Graph(n, u, v, w)
    h = Hierarchy(g)
    M = MSP(h, mu) if precond == "msp" else PEGP(n, u, v, w, h.aggs(), mu)
    return spectrum_estimate(g.apply, M.apply, b, steps)


CASES = {
    "grid2d_32_log_msp0.8": lambda: (*W.grid2d(32), "log", "msp", 0.8),
    "grid2d_32_msp0.95": lambda: (*W.grid2d(32), None, "msp", 0.95),
    "grid3d_16_log_msp0.8": lambda: (*W.grid3d(16), "log", "msp", 0.8),
    "chung_lu_2000_msp0.8": lambda: (*W.chung_lu(2000, 8.0, 2.1, 41), "log", "msp", 0.8),
    "grid2d_32_pegp": lambda: (*W.grid2d(32), None, "pegp", 1 / 32),
}


@pytest.mark.parametrize("name", list(CASES))
def test_spectrum_parity(oracle_lib, name):
    import paper_2207_07847_amd as lap
    n, u, v, wk, precond, mu = CASES[name]()
    w = np.ones(len(u)) if wk is None else W.loguniform_weights(len(u), 43, -2.0, 2.0)
    b = W.gaussian_rhs(n, 44)
    lo0, hi0, k0 = _oracle_estimate(n, u, v, w, b, precond, mu, 1000)
    pc = lap.LAP_PREC_MSP if precond == "msp" else lap.LAP_PREC_PEGP
    G = GpuLap(n, u, v, w, mu=mu, precond=pc)
    try:
        st, lo, hi, k = G.estimate_spectrum(b, 1000)
        st40, lo40, hi40, k40 = G.estimate_spectrum(b, 40)
    finally:
        G.close()
    say(name, "gpu", lo, hi, k, "oracle", lo0, hi0, k0, "40 steps", lo40, hi40, k40)
    assert st == 0 and abs(k - k0) <= 1
    assert abs(lo - lo0) <= 1e-6 * lo0 and abs(hi - hi0) <= 1e-6 * hi0
    assert st40 == 0 and k40 == min(40, k)
    assert lo * (1 - 1e-9) <= lo40 <= hi40 <= hi * (1 + 1e-9)


def test_spectrum_inside_dense(oracle_lib):
    """Weighted 8x8 grid, MSP mu = 0.8: the GPU's estimate finds the dense
    pencil's extreme eigenvalues (both isolated)."""
    from oracle import Graph, Hierarchy, dense
    n, u, v = W.grid2d(8)
    w = W.loguniform_weights(len(u), 21, -1.0, 1.0)
    g = Graph(n, u, v, w)
    h = Hierarchy(g)
    L = dense.laplacian(n, u, v, w)
    Gt = dense.expanded(L, dense.p_mu(h.aggs(), n, 0.8))
    H = dense.positive_subgraph(Gt)
    T = dense.msp_from_h(H, h.aggs(), dense.level_sizes(h.aggs(), n))
    ev = np.sort(np.abs(dense.pencil_eigs(Gt, T)))
    ev = ev[ev > 1e-9 * ev.max()]
    G = GpuLap(n, u, v, w, mu=0.8)
    try:
        st, lo, hi, k = G.estimate_spectrum(W.gaussian_rhs(n, 22), 400)
    finally:
        G.close()
    assert st == 0
    assert abs(lo - ev[0]) <= 1e-8 * ev[0] and abs(hi - ev[-1]) <= 1e-8 * ev[-1], (lo, hi, ev[0], ev[-1])


def test_select_mu_parity(oracle_lib):
    """Weighted 32x32 grid, MSP, mu in {0.3, ..., 0.95}: the same choice as
    the oracle, and the same estimates."""
    import paper_2207_07847_amd as lap
    from oracle.lanczos import select_mu
    torch = pytest.importorskip("torch")
    n, u, v = W.grid2d(32)
    w = W.loguniform_weights(len(u), 31, -1.0, 1.0)
    b = W.gaussian_rhs(n, 32)
    mus = [0.3, 0.5, 0.7, 0.8, 0.9, 0.95]
    best0, k0 = select_mu(n, u, v, w, mus, b, 40)
    bd = torch.tensor(b, dtype=torch.float64, device="cuda")
    st, best, kap = lap.lap_select_mu(n, u, v, w, mus, bd.data_ptr(), 40,
                                      stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    say("select mu: gpu", mus[best], list(kap), "oracle", mus[best0], k0)
    assert st == 0 and best == best0
    # 40 steps leave lambda_min unconverged at kappa >~ 1e3, where rounding
    # moves the estimate by up to 1 % (measured: 0.7 % at mu = 0.5); the
    # candidates' estimates differ from each other by 13 % or more
    assert np.allclose(kap, k0, rtol=2e-2)


def test_spectrum_errors(oracle_lib):
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(8)
    w = np.ones(len(u))
    b = W.gaussian_rhs(n, 1)
    G = GpuLap(n, u, v, w, precond=lap.LAP_PREC_NONE)
    try:
        assert G.estimate_spectrum(b, 10)[0] == lap.LAP_EUNSUPPORTED
    finally:
        G.close()
    G = GpuLap(n, u, v, w)
    try:
        assert G.estimate_spectrum(b, 0)[0] == lap.LAP_EINVAL
        assert G.estimate_spectrum(np.full(n, np.nan), 10)[0] == lap.LAP_EINVAL
    finally:
        G.close()
