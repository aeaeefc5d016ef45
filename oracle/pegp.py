"""PEGP preconditioner with a sparse direct solve (oracle).

TEST INFRASTRUCTURE ONLY.  The positively weighted expanded graph
preconditioner (Sec. 3.2) applied to the original system through the
lifting of Sec. 3.1:  z = P(mu) L_H~^+ P(mu)^T r, mean removed.

Steps, in the paper's notation, with scipy.sparse as the matrix library:
  1. L_G~ = P(mu)^T L_G P(mu)                 (Eq. def:L_ell, sparse product)
  2. H~   = negative off-diagonals of L_G~, diagonal recomputed (Sec. 3.2)
  3. solve L_H~ y = P(mu)^T r with the last expanded node grounded (y = 0
     there; any solution differs by a constant, mapped by P(mu) to a
     constant that the final projection removes).  The grounded matrix is
     first scaled as S = D L_H~ D with D = diag(mu^-k) on level k, an exact
     diagonal similarity (y = D S^-1 D rhs) that keeps the pivots O(1).
  4. z = P(mu) y - mean.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def laplacian_sparse(n, u, v, w):
    """L_G = B^T W B."""
    m = len(u)
    B = sp.csr_matrix((np.concatenate([np.ones(m), -np.ones(m)]),
                       (np.concatenate([np.arange(m), np.arange(m)]),
                        np.concatenate([u, v]))), shape=(m, n))
    return (B.T @ sp.diags(np.asarray(w, dtype=np.float64)) @ B).tocsr()


def p_mu_sparse(aggs, n, mu):
    """P(mu) = [I, -mu P^2, ..., (-mu)^(l-1) P^l] as a sparse n x n~ matrix."""
    blocks = [sp.identity(n, format="csr")]
    Pk = sp.identity(n, format="csr")
    for k, a in enumerate(aggs, start=1):
        nc = int(np.max(a)) + 1
        Pstep = sp.csr_matrix((np.ones(len(a)), (np.arange(len(a)), a)),
                              shape=(len(a), nc))
        Pk = (Pk @ Pstep).tocsr()
        blocks.append(((-mu) ** k) * Pk)
    return sp.hstack(blocks).tocsr()


def positive_part(Gt):
    """H~ from L_G~: keep off-diagonal entries < 0, recompute the diagonal."""
    G = sp.coo_matrix(Gt)
    off = (G.row != G.col) & (G.data < 0.0)
    H = sp.csr_matrix((G.data[off], (G.row[off], G.col[off])), shape=G.shape)
    d = -np.asarray(H.sum(axis=1)).ravel()
    return (H + sp.diags(d)).tocsr()


class PEGP:
    """z = P(mu) pinv(L_H~) P(mu)^T r (mean-free) for a fixed hierarchy."""

    def __init__(self, n, u, v, w, aggs, mu, permc_spec="COLAMD"):
        self.n = int(n)
        self.mu = float(mu)
        L = laplacian_sparse(n, np.asarray(u), np.asarray(v), w)
        self.Pmu = p_mu_sparse(aggs, n, mu)
        self.Gt = (self.Pmu.T @ L @ self.Pmu).tocsr()
        self.Ht = positive_part(self.Gt)
        sizes = [n] + [int(np.max(a)) + 1 for a in aggs]
        self.sizes = sizes
        self.d = np.concatenate([np.full(s, mu ** (-k)) for k, s in enumerate(sizes)])
        D = sp.diags(self.d)
        S = (D @ self.Ht @ D).tocsc()
        self.nt = S.shape[0]
        # permc_spec: the fill ordering of the sparse LU (any ordering gives
        # the same solve up to rounding; tests use two to measure that spread)
        self._lu = spla.splu(S[:-1, :-1].tocsc(), permc_spec=permc_spec)

    @property
    def nnz_ht(self):
        return self.Ht.nnz

    def solve_expanded(self, bt):
        """Grounded solve of L_H~ y~ = b~ in the expanded space: the scaled
        system D L_H~ D (D y~') = D b~ with the last node grounded."""
        y = np.zeros(self.nt)
        y[:-1] = self._lu.solve((self.d * np.asarray(bt, dtype=np.float64))[:-1])
        return y * self.d

    def apply(self, r):
        rt = self.Pmu.T @ np.asarray(r, dtype=np.float64)
        y = np.zeros(self.nt)
        y[:-1] = self._lu.solve((self.d * rt)[:-1])
        y *= self.d
        z = self.Pmu @ y
        return z - z.mean()

    __call__ = apply
