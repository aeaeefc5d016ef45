"""FGMRES on the expanded system (test infrastructure only).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may use this module; it shares no
code with the GPU library.

The paper's experiments (Sec. 4) solve the expanded system
L_G~ x~ = b~ (Sec. 2.2), with L_G~ = P(mu)^T L_G P(mu) and b~ = P(mu)^T b,
(b projected to mean zero first), by flexible GMRES [Saad]
right-preconditioned by the grounded inverse of
L_H~ (PEGP) or of L_T~ (MSP), to a relative residual ||b~ - L_G~ x~|| /
||b~|| <= tol, at most 1000 steps.  The solution of the original system
is x = P(mu) x~ (the theorem of Sec. 2.2), reported mean-free.

This is flexible GMRES without restarts, written from its definition:
Arnoldi on the preconditioned directions z_j = M v_j with modified
Gram-Schmidt, Givens rotations keeping the Hessenberg matrix triangular,
the least-squares residual |g_{j+1}| as the stop test, and x~ = Z y from the
triangular solve at the end.  A step is one product with L_G~.
"""
from __future__ import annotations

import numpy as np

from .pegp import laplacian_sparse, p_mu_sparse


class FgmresResult:
    def __init__(self, x, xt, iterations, status, relres_est, relres_expanded, relres_true, hist):
        self.x = x                          # mean-free solution of L_G x = b
        self.xt = xt                        # expanded iterate x~
        self.iterations = iterations        # products with L_G~
        self.status = status                # 0 converged, 5 max steps
        self.relres_est = relres_est        # |g_{k+1}| / ||b~|| of the least squares
        self.relres_expanded = relres_expanded  # ||b~ - L_G~ x~|| / ||b~||, recomputed
        self.relres_true = relres_true      # ||b^ - L_G x|| / ||b^||, b^ = b - mean(b)
        self.hist = hist                    # |g_{j+1}| / ||b~|| per step


def fgmres_expanded(n, u, v, w, aggs, mu, b, solve_expanded, tol=1e-8, maxit=1000):
    """solve_expanded(bt) -> y~: the preconditioner on expanded vectors
    (MSP.solve_expanded or PEGP.solve_expanded built on the same aggs)."""
    L = laplacian_sparse(n, np.asarray(u), np.asarray(v), np.asarray(w, dtype=np.float64))
    P = p_mu_sparse(aggs, n, mu).tocsr()
    PT = P.T.tocsr()

    def A(z):
        return PT @ (L @ (P @ z))

    # b is projected first (b^ = b - mean(b), the solver's convention): the
    # expanded system is consistent only for b in range(L_G)
    b = np.asarray(b, dtype=np.float64)
    bt = PT @ (b - b.mean())
    beta = float(np.linalg.norm(bt))
    nt = bt.shape[0]
    if beta == 0.0:
        x = np.zeros(n)
        return FgmresResult(x, np.zeros(nt), 0, 0, 0.0, 0.0, 0.0, np.zeros(1))
    V = np.zeros((maxit + 1, nt))
    Z = np.zeros((maxit, nt))
    H = np.zeros((maxit + 1, maxit))
    cs = np.zeros(maxit)
    sn = np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    V[0] = bt / beta
    hist = [1.0]
    k = 0
    status = 5
    for j in range(maxit):
        Z[j] = solve_expanded(V[j])
        wv = A(Z[j])
        for i in range(j + 1):
            H[i, j] = float(np.dot(wv, V[i]))
            wv = wv - H[i, j] * V[i]
        H[j + 1, j] = float(np.linalg.norm(wv))
        # previous rotations on the new column, then the one zeroing H[j+1, j]
        for i in range(j):
            hi, hi1 = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * hi + sn[i] * hi1
            H[i + 1, j] = -sn[i] * hi + cs[i] * hi1
        den = float(np.hypot(H[j, j], H[j + 1, j]))
        cs[j], sn[j] = (1.0, 0.0) if den == 0.0 else (H[j, j] / den, H[j + 1, j] / den)
        H[j, j] = den
        H[j + 1, j] = 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]) / beta)
        if abs(g[j + 1]) <= tol * beta:
            status = 0
            break
        if den == 0.0 or np.linalg.norm(wv) == 0.0:
            break
        V[j + 1] = wv / np.linalg.norm(wv)
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - np.dot(H[i, i + 1:k], y[i + 1:k])) / H[i, i]
    xt = Z[:k].T @ y
    x = P @ xt
    x -= x.mean()
    rel_exp = float(np.linalg.norm(bt - A(xt))) / beta
    bh = b - b.mean()
    nb = float(np.linalg.norm(bh))
    rel_true = float(np.linalg.norm(bh - L @ x)) / nb if nb > 0 else 0.0
    return FgmresResult(x, xt, k, status, abs(g[k]) / beta, rel_exp, rel_true, np.array(hist))
