"""GPU FGMRES on the expanded system (LAP_FLAG_FGMRES) against the oracle's.

The GPU runs FGMRES in the original space with expanded inner products
(every basis vector lies in the range of P(mu)^T); the oracle runs it on
expanded vectors with the grounded expanded solve.  Both minimise the same
residual over the same Krylov spaces, so the step counts must agree up to
rounding (one step), both solutions must meet the residual they stop on,
and the GPU's solution must equal the oracle's FGMRES iterate after the
same number of steps within 1e-7 relative (the solution bar of the PCG
parity tests; what is left is rounding).
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


def _oracle_fgmres(n, u, v, w, b, precond, mu, max_levels=0, same_steps=None):
    """The oracle's FGMRES to tol 1e-8, and (same_steps) its iterate after
    exactly that many steps (tol 0)."""
    from oracle import MSP, Graph, Hierarchy
    from oracle.fgmres import fgmres_expanded
    from oracle.pegp import PEGP
    h = Hierarchy(Graph(n, u, v, w), max_levels=max_levels)
    M = MSP(h, mu) if precond == "msp" else PEGP(n, u, v, w, h.aggs(), mu)
    if same_steps is not None:
        return fgmres_expanded(n, u, v, w, h.aggs(), mu, b, M.solve_expanded, tol=0.0,
                               maxit=same_steps)
    return fgmres_expanded(n, u, v, w, h.aggs(), mu, b, M.solve_expanded)


def _host_relres(n, u, v, w, b, x):
    from oracle import Graph
    bh = b - b.mean()
    return np.linalg.norm(bh - Graph(n, u, v, w).apply(x)) / np.linalg.norm(bh)


CASES = []
for a in (16, 32, 64):
    n = a * a
    CASES += [(a, "msp", 0.8, 0), (a, "pegp", 1 / np.sqrt(n), 0), (a, "pegp", n ** -0.25, 2)]


@pytest.mark.parametrize("a,precond,mu,ml", CASES)
def test_fgmres_table3_grids(oracle_lib, a, precond, mu, ml):
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(a)
    w = np.ones(len(u))
    b = W.lowfreq_rhs(n)
    ref = _oracle_fgmres(n, u, v, w, b, precond, mu, ml)
    pc = lap.LAP_PREC_MSP if precond == "msp" else lap.LAP_PREC_PEGP
    G = GpuLap(n, u, v, w, mu=mu, precond=pc, max_levels=ml, max_iter=1000,
               flags=lap.LAP_FLAG_FGMRES)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    same = _oracle_fgmres(n, u, v, w, b, precond, mu, ml, same_steps=info["iterations"])
    d_same = np.linalg.norm(x - same.x) / np.linalg.norm(same.x)
    msg = (f"fgmres {n} {precond} mu {mu:.4g} level {ml or 'max'}: gpu {info['iterations']} "
           f"oracle {ref.iterations} steps; est {info['relres_recursive']:.3e} true "
           f"{info['relres_true']:.3e}; x vs oracle at the same step count {d_same:.2e}")
    say(msg)
    assert st == 0 and abs(info["iterations"] - ref.iterations) <= 1, msg
    assert info["relres_recursive"] <= 1e-8, msg
    # the original residual is the expanded one's image: same order
    assert _host_relres(n, u, v, w, b, x) <= 3e-8, msg
    assert d_same <= 1e-7, msg


def test_fgmres_weighted_powerlaw(oracle_lib):
    import paper_2207_07847_amd as lap
    n, u, v = W.chung_lu(4000, 8.0, 2.1, 97)
    w = W.loguniform_weights(len(u), 98, -2.0, 2.0)
    b = W.gaussian_rhs(n, 99)
    ref = _oracle_fgmres(n, u, v, w, b, "msp", 0.8)
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=1000, flags=lap.LAP_FLAG_FGMRES)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    say("fgmres chung-lu: gpu", info["iterations"], "oracle", ref.iterations, info)
    assert st == 0 and abs(info["iterations"] - ref.iterations) <= 1
    assert _host_relres(n, u, v, w, b, x) <= 1e-7


def test_fgmres_restarted(oracle_lib, monkeypatch):
    """A basis of 12 vectors: restarts from the true residual, more steps,
    the same bar on the expanded residual."""
    import paper_2207_07847_amd as lap
    monkeypatch.setenv("LAPGPU_FGMRES_RESTART", "12")
    n, u, v = W.grid2d(32)
    w = np.ones(len(u))
    b = W.lowfreq_rhs(n)
    full = _oracle_fgmres(n, u, v, w, b, "msp", 0.8).iterations
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=1000, flags=lap.LAP_FLAG_FGMRES)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    say("fgmres(12):", info["iterations"], "without restart", full)
    assert st == 0 and info["iterations"] > full
    assert _host_relres(n, u, v, w, b, x) <= 3e-8


def test_fgmres_unsupported():
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(16)
    w = np.ones(len(u))
    b = W.lowfreq_rhs(n)
    for kw in (dict(precond=lap.LAP_PREC_NONE), dict(precision=lap.LAP_MIXED_FP32_FP64)):
        G = GpuLap(n, u, v, w, mu=0.8, flags=lap.LAP_FLAG_FGMRES, **kw)
        try:
            st, _, _ = G.solve(b, 1e-8)
        finally:
            G.close()
        assert st == lap.LAP_EUNSUPPORTED, kw
