"""Pins of the oracle's FGMRES on the expanded system (Sec. 4's solver).

The oracle solves by PCG on the original system (reading A11); FGMRES on
the expanded system L_G~ x~ = P(mu)^T b is kept beside it to test that
reading against the step counts of Table 3.  These tests pin FGMRES itself
against definitions it must satisfy, then compare both solvers with the
table.
"""
import numpy as np
import pytest

import workloads as W


def _grid(a):
    n, u, v = W.grid2d(a)
    return n, u, v, np.ones(len(u))


def _krylov_residuals(A, b, kmax):
    """min_y ||b - A K_k y|| for k = 1..kmax by explicit least squares on an
    orthonormal basis of K_k = span{b, A b, ..., A^(k-1) b} (GMRES by
    definition, no Arnoldi recurrence)."""
    out = []
    K = [b / np.linalg.norm(b)]
    for k in range(1, kmax + 1):
        Q, _ = np.linalg.qr(np.array(K).T)
        AQ = A @ Q
        y, *_ = np.linalg.lstsq(AQ, b, rcond=None)
        out.append(np.linalg.norm(b - AQ @ y) / np.linalg.norm(b))
        nxt = A @ K[-1]
        K.append(nxt / np.linalg.norm(nxt))
    return np.array(out)


def test_fgmres_identity_preconditioner_is_gmres(oracle_lib):
    """With M = I the residual history equals GMRES's minimum residuals over
    the Krylov spaces of L_G~ and b~, computed by brute-force least squares."""
    from oracle import Graph, Hierarchy
    from oracle.dense import laplacian, p_mu
    from oracle.fgmres import fgmres_expanded
    n, u, v, w = _grid(6)
    h = Hierarchy(Graph(n, u, v, w))
    aggs = h.aggs()
    mu = 0.8
    res = fgmres_expanded(n, u, v, w, aggs, mu, W.lowfreq_rhs(n), lambda t: t.copy(),
                          tol=1e-10, maxit=25)
    Pm = p_mu(aggs, n, mu)
    A = Pm.T @ laplacian(n, u, v, w) @ Pm
    bt = Pm.T @ W.lowfreq_rhs(n)
    k = min(res.iterations, 12)
    ref = _krylov_residuals(A, bt, k)
    assert np.allclose(res.hist[1:k + 1], ref, rtol=1e-6, atol=1e-12), (res.hist[1:k + 1], ref)


def test_fgmres_exact_preconditioner_one_step(oracle_lib):
    """M~ = pinv(L_G~): the preconditioned operator is a projector on the
    range, so one step solves the system."""
    from oracle import Graph, Hierarchy
    from oracle.dense import laplacian, p_mu
    from oracle.fgmres import fgmres_expanded
    n, u, v, w = _grid(4)
    h = Hierarchy(Graph(n, u, v, w))
    Pm = p_mu(h.aggs(), n, 0.8)
    pinv = np.linalg.pinv(Pm.T @ laplacian(n, u, v, w) @ Pm)
    res = fgmres_expanded(n, u, v, w, h.aggs(), 0.8, W.lowfreq_rhs(n), lambda t: pinv @ t,
                          tol=1e-10)
    assert res.iterations == 1 and res.status == 0
    assert res.relres_expanded <= 1e-10


@pytest.mark.parametrize("precond", ["msp", "pegp"])
def test_fgmres_solution(oracle_lib, precond):
    """x = P(mu) x~ solves L_G x = b (the theorem of Sec. 2.2): against the
    dense pseudo-inverse, within the bound kappa(L) * tol; the least-squares
    estimate is the recomputed expanded residual; the history never rises."""
    from oracle import MSP, Graph, Hierarchy
    from oracle.dense import laplacian
    from oracle.fgmres import fgmres_expanded
    from oracle.pegp import PEGP
    n, u, v, w = _grid(12)
    w = W.loguniform_weights(len(u), 5, -1.0, 1.0)
    b = W.gaussian_rhs(n, 6)
    h = Hierarchy(Graph(n, u, v, w))
    M = MSP(h, 0.8) if precond == "msp" else PEGP(n, u, v, w, h.aggs(), 1 / 12)
    mu = 0.8 if precond == "msp" else 1 / 12
    res = fgmres_expanded(n, u, v, w, h.aggs(), mu, b, M.solve_expanded, tol=1e-10)
    L = laplacian(n, u, v, w)
    ev = np.linalg.eigvalsh(L)
    x0 = np.linalg.pinv(L) @ (b - b.mean())
    assert res.status == 0
    assert np.linalg.norm(res.x - x0) / np.linalg.norm(x0) <= ev[-1] / ev[1] * 1e-10 * 1.01
    assert abs(res.relres_expanded - res.relres_est) <= 1e-6 * max(res.relres_est, 1e-12) + 1e-13
    assert np.all(np.diff(res.hist) <= 1e-14)


def test_table3_fgmres_against_pcg(oracle_lib):
    """Table 3 (tol 1e-8, b = [1,...,1,1-n]) with both solvers.  PEGP:
    FGMRES on the expanded system stays within one step of the table, PCG
    matches it.  MSP (mu = 0.8): FGMRES needs markedly fewer steps than the
    table and PCG is the closer of the two, which is why the solve here is
    PCG (reading A11)."""
    from oracle import MSP, Graph, Hierarchy, pcg
    from oracle.fgmres import fgmres_expanded
    from oracle.pegp import PEGP
    from test_oracle_pins import TABLES
    for a in (16, 32, 64):
        n, u, v, w = _grid(a)
        b = W.lowfreq_rhs(n)
        g = Graph(n, u, v, w)
        h = Hierarchy(g)
        M = MSP(h, 0.8)
        f = fgmres_expanded(n, u, v, w, h.aggs(), 0.8, b, M.solve_expanded).iterations
        p = pcg(g, b, 1e-8, 1000, M).iterations
        t = TABLES[("table3", "grid", n, "msp_levelmax_steps")]
        assert abs(p - t) < abs(f - t) and f < t, (n, f, p, t)
        for ml, mu, col in [(0, 1 / np.sqrt(n), "pegp_levelmax_steps"),
                            (2, n ** -0.25, "pegp_level2_steps")]:
            h2 = Hierarchy(g, max_levels=ml)
            Pg = PEGP(n, u, v, w, h2.aggs(), mu)
            f2 = fgmres_expanded(n, u, v, w, h2.aggs(), mu, b, Pg.solve_expanded).iterations
            assert abs(f2 - TABLES[("table3", "grid", n, col)]) <= 1, (n, col, f2)
