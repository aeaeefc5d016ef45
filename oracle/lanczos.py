"""Spectrum estimates of the preconditioned operator, and a choice of mu.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may use this module; it shares no
code with the GPU library.

How fast PCG converges with the MSP or PEGP preconditioner is governed by
kappa(M L_G) on range(L_G), which the theorem of Sec. 3.2 bounds by
1/(1 - rho) for mu small enough; how to pick mu for a given graph is left
open there (the remark after the theorem, and Sec. 5).  The estimate here is
the standard one from PCG's own coefficients (Saad, Iterative Methods for
Sparse Linear Systems, 2nd ed., Sec. 6.7.3): the k PCG steps with step
lengths alpha_j and direction updates beta_j are k steps of Lanczos on M L,
whose tridiagonal matrix T_k has

    T_jj     = 1/alpha_j + beta_j / alpha_{j-1}      (beta_0 = 0)
    T_j,j+1  = T_j+1,j = sqrt(beta_{j+1}) / alpha_j,

and the extreme eigenvalues of T_k (Ritz values) approach the extreme
eigenvalues of M L on range(L) from inside.  Here beta_{j+1} is the beta that
forms direction j+1 from z_{j+1}: p_{j+1} = z_{j+1} + beta_{j+1} p_j.

The choice of mu: for each candidate, the hierarchy (independent of mu) and
the preconditioner at that mu, the estimate from `steps` PCG steps on the
same right-hand side, and the candidate with the smallest estimated kappa
(PCG's step count grows as sqrt(kappa); an MSP application costs the same
at every mu).
"""
from __future__ import annotations

import numpy as np


class PcgCoefficients:
    def __init__(self, alpha, beta, relres):
        self.alpha = np.asarray(alpha, dtype=np.float64)   # alpha_0 .. alpha_{k-1}
        self.beta = np.asarray(beta, dtype=np.float64)     # beta_1 .. beta_{k-1}
        self.relres = relres                               # ||r_k|| / ||b^|| at the end

    @property
    def steps(self):
        return len(self.alpha)


def pcg_coefficients(apply_l, apply_m, b, steps, stop=1e-10):
    """PCG from its definition on L x = b^ (b^ = b - mean(b), x_0 = 0),
    z = apply_m(r) made mean-free, recording alpha_j and beta_{j+1}.  Stops
    after `steps` steps, or earlier when ||r|| <= stop ||b^|| or r^T z <= 0
    (breakdown).  The extreme Ritz values have converged long before the
    residual reaches 1e-10; closer to rounding level, the preconditioner's
    own rounding, now large next to r, corrupts the last coefficients and
    can put a Ritz value outside the spectrum."""
    b = np.asarray(b, dtype=np.float64)
    r = b - b.mean()
    bn = float(np.linalg.norm(r))
    z = np.asarray(apply_m(r), dtype=np.float64)
    z = z - z.mean()
    rz = float(r @ z)
    p = z.copy()
    alpha, beta = [], []
    relres = 1.0
    for _ in range(steps):
        if not rz > 0.0:
            break
        q = np.asarray(apply_l(p), dtype=np.float64)
        pq = float(p @ q)
        if not pq > 0.0:
            break
        a = rz / pq
        alpha.append(a)
        r = r - a * q
        relres = float(np.linalg.norm(r)) / bn
        if relres <= stop or len(alpha) == steps:
            break
        z = np.asarray(apply_m(r), dtype=np.float64)
        z = z - z.mean()
        rz_new = float(r @ z)
        bt = rz_new / rz
        beta.append(bt)
        p = z + bt * p
        rz = rz_new
    return PcgCoefficients(alpha, beta, relres)


def lanczos_matrix(alpha, beta):
    """T_k from alpha_0..alpha_{k-1} and beta_1..beta_{k-1} (dense)."""
    k = len(alpha)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alpha[j] + (beta[j - 1] / alpha[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(beta[j]) / alpha[j]
    return T


def spectrum_estimate(apply_l, apply_m, b, steps, stop=1e-10):
    """(lambda_min, lambda_max, steps taken) of M L on range(L)."""
    c = pcg_coefficients(apply_l, apply_m, b, steps, stop)
    ev = np.linalg.eigvalsh(lanczos_matrix(c.alpha, c.beta))
    return float(ev[0]), float(ev[-1]), c.steps


def select_mu(n, u, v, w, mus, b, steps, precond="msp", max_levels=0):
    """The candidate with the smallest estimated kappa, and every estimate."""
    from . import MSP, Graph, Hierarchy
    from .pegp import PEGP
    g = Graph(n, u, v, w)
    h = Hierarchy(g, max_levels=max_levels)
    kappas = []
    for mu in mus:
        M = MSP(h, mu) if precond == "msp" else PEGP(n, u, v, w, h.aggs(), mu)
        lo, hi, _ = spectrum_estimate(g.apply, M.apply, b, steps)
        kappas.append(hi / lo if lo > 0.0 else np.inf)
    return int(np.argmin(kappas)), kappas
