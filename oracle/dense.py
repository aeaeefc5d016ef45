"""Dense definitions of the paper's objects for tiny graphs (oracle).

TEST INFRASTRUCTURE ONLY.  Every matrix is formed explicitly from its
definition, in FP64 numpy, so that a reader can check it against the paper:

  * L_G = B^T W B (Sec. 2.1);
  * P_{k}^{k+1}(i, j) = 1 iff node i is in aggregate j; P^k = P_1^2 ... P_{k-1}^k
    (Eq. def:P); P(mu) = [I, -mu P^2, mu^2 P^3, ...] (Sec. 2.2);
  * L_G~ = P(mu)^T L_G P(mu) (Eq. def:L_ell);
  * H~: the positively weighted edges of G~, i.e. the negative off-diagonal
    entries of L_G~, with the diagonal recomputed as a Laplacian (Sec. 3.2);
  * T~ (MSP): from H~ keep the top-level edges, the links between a node and
    its own aggregate on the next level, and the edges inside aggregates
    (Sec. 3.3; reading stated in the design notes);
  * kappa(pinv(B) A): largest over smallest nonzero eigenvalue (Sec. 3.2).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def laplacian(n, u, v, w):
    """L_G = B^T W B from the incidence matrix B (one row per edge)."""
    m = len(u)
    B = np.zeros((m, n))
    B[np.arange(m), u] = 1.0
    B[np.arange(m), v] = -1.0
    return B.T @ np.diag(np.asarray(w, dtype=np.float64)) @ B


def prolongation(agg, nc):
    """P_{k}^{k+1}(i, j) = 1 if node i is in aggregate j."""
    P = np.zeros((len(agg), nc))
    P[np.arange(len(agg)), agg] = 1.0
    return P


def composite(aggs, n):
    """[P^1 = I, P^2, ..., P^l] with P^(k+1) = P^k P_k^(k+1)."""
    Ps = [np.eye(n)]
    for a in aggs:
        nc = int(np.max(a)) + 1
        Ps.append(Ps[-1] @ prolongation(a, nc))
    return Ps


def p_mu(aggs, n, mu):
    """P(mu) = [I, (-mu) P^2, (-mu)^2 P^3, ..., (-mu)^(l-1) P^l]."""
    Ps = composite(aggs, n)
    return np.hstack([(-mu) ** k * P for k, P in enumerate(Ps)])


def level_sizes(aggs, n):
    return [n] + [int(np.max(a)) + 1 for a in aggs]


def expanded(L, Pmu):
    """L_G~ = P(mu)^T L_G P(mu)."""
    return Pmu.T @ L @ Pmu


def positive_subgraph(Gt):
    """H~: keep the off-diagonal entries < 0 (positive edges); diagonal =
    minus the sum of the kept off-diagonals of the row."""
    off = Gt - np.diag(np.diag(Gt))
    H = np.where(off < 0.0, off, 0.0)
    H[np.diag_indices_from(H)] = -H.sum(axis=1)
    return H


def negative_part(Gt):
    """L_mu^-: Laplacian of the dropped (negatively weighted) edges, so that
    L_G~ = L_H~ - L_mu^- (Lemma lem:upper)."""
    off = Gt - np.diag(np.diag(Gt))
    N = np.where(off > 0.0, -off, 0.0)
    N[np.diag_indices_from(N)] = -N.sum(axis=1)
    return N


def level_of(sizes):
    return np.concatenate([np.full(s, k) for k, s in enumerate(sizes)])


def msp_from_h(H, aggs, sizes):
    """T~ extracted from H~: edges inside an aggregate on every level below
    the top, links (i, agg(i)) between adjacent levels, all top-level edges."""
    nt = sum(sizes)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    lev = level_of(sizes)
    local = np.arange(nt) - offs[lev]
    top = len(sizes) - 1
    keep = np.zeros((nt, nt), dtype=bool)
    for i in range(nt):
        for j in range(nt):
            if i == j or H[i, j] == 0.0:
                continue
            ki, kj = lev[i], lev[j]
            if ki == kj:
                if ki == top or aggs[ki][local[i]] == aggs[ki][local[j]]:
                    keep[i, j] = True
            elif kj == ki + 1 and aggs[ki][local[i]] == local[j]:
                keep[i, j] = keep[j, i] = True
    T = np.where(keep, H, 0.0)
    T[np.diag_indices_from(T)] = 0.0
    T[np.diag_indices_from(T)] = -T.sum(axis=1)
    return T


def edges_to_dense(nt, u, v, w):
    """Laplacian of an edge list (used for oracle-built T~)."""
    A = np.zeros((nt, nt))
    for a, b, c in zip(u, v, w):
        A[a, b] -= c
        A[b, a] -= c
        A[a, a] += c
        A[b, b] += c
    return A


def pencil_eigs(A, B):
    """Eigenvalues of pinv(B) A for Laplacians A, B with null(B) = span{1}
    and A 1 = 0.

    With D = diag(B)^(-1/2), the pencil (D A D, D B D + u u^T), u = D^-1 1,
    has eigenvalue 0 on u and, on the D B D-orthogonal complement of u,
    exactly the eigenvalues of B v = lambda^-1 A v restricted to 1-perp,
    i.e. those of pinv(B) A.  The congruence by D changes no eigenvalue; it
    only keeps the entries O(1) when the levels are scaled by mu^(2k)."""
    d = 1.0 / np.sqrt(np.diag(B))
    u = 1.0 / d
    u /= np.linalg.norm(u)
    As = d[:, None] * A * d[None, :]
    Bs = d[:, None] * B * d[None, :]
    return sla.eigh(As, Bs + np.outer(u, u), eigvals_only=True)


def kappa(A, B, rel=1e-9):
    """kappa(pinv(B) A) = lambda_max / smallest nonzero lambda."""
    ev = np.abs(pencil_eigs(A, B))
    nz = ev[ev > rel * ev.max()]
    return nz.max() / nz.min()


def pinv_solve_operator(T, Pmu):
    """P(mu) pinv(L_T~) P(mu)^T with the mean removed on both sides."""
    n = Pmu.shape[0]
    M = Pmu @ np.linalg.pinv(T) @ Pmu.T
    J = np.eye(n) - np.ones((n, n)) / n
    return J @ M @ J


def stretch(T, H):
    """Total stretch of H's edges in T (Eqs. def:stretch-edge/graph), with
    the tree distance taken as the effective resistance through T (for a
    tree it is the path sum of 1/w; for the sparsifier it is a lower bound
    of the lightest path sum used by the paper)."""
    Tp = np.linalg.pinv(T)
    nt = T.shape[0]
    total = 0.0
    for i in range(nt):
        for j in range(i + 1, nt):
            if H[i, j] < 0.0:
                e = np.zeros(nt)
                e[i], e[j] = 1.0, -1.0
                total += -H[i, j] * (e @ Tp @ e)
    return total


def _highprec_expanded(n, u, v, w, aggs, mu, ctx):
    """(P(mu), L_G~, T~, mask of T~'s edges) in mpmath, from the definitions
    (the sign pattern of H~ and T~'s edge mask from the FP64 objects: which
    entries are kept is structural)."""
    mu_ = ctx.mpf(mu)
    sizes = level_sizes(aggs, n)
    nt = sum(sizes)
    Pm64 = p_mu(aggs, n, float(mu))
    Gt64 = expanded(laplacian(n, u, v, w), Pm64)
    T64 = msp_from_h(positive_subgraph(Gt64), aggs, sizes)
    keep = (T64 != 0.0) & ~np.eye(nt, dtype=bool)
    Pm = ctx.zeros(n, nt)
    col = 0
    for k, P in enumerate(composite(aggs, n)):
        f = (-mu_) ** k
        for i, j in zip(*np.nonzero(P)):
            Pm[int(i), col + int(j)] = f
        col += P.shape[1]
    Lg = ctx.zeros(n, n)
    for a, b, c in zip(u, v, w):
        c = ctx.mpf(float(c))
        a, b = int(a), int(b)
        Lg[a, a] += c
        Lg[b, b] += c
        Lg[a, b] -= c
        Lg[b, a] -= c
    Gt = Pm.T * Lg * Pm
    T = ctx.zeros(nt, nt)
    for i, j in zip(*np.nonzero(keep)):
        T[int(i), int(j)] = Gt[int(i), int(j)]
    for i in range(nt):
        T[i, i] = -ctx.fsum(T[i, j] for j in range(nt) if j != i)
    return Pm, Gt, T, keep


def _highprec_pinv(T, ctx):
    """pinv(L) = (L + J/t)^(-1) - J/t for a connected Laplacian of t nodes."""
    t = T.rows
    J = ctx.ones(t, t) / t
    return ctx.inverse(T + J) - J


def offtree_stretch_highprec(n, u, v, w, aggs, mu, pairs, dps=50):
    """Stretch in T~ of the H~ edges `pairs` (expanded indices i < j): the
    H~ weight w_ij = -L_G~(i, j) times the effective resistance
    (e_i - e_j)^T pinv(L_T~) (e_i - e_j), all in mpmath at `dps` digits
    (Sec. 3.3, def. stretch-edge with the resistance as the distance).  For
    tiny graphs only."""
    import mpmath as mpm
    ctx = mpm.mp.clone()
    ctx.dps = dps
    _, Gt, T, _ = _highprec_expanded(n, u, v, w, aggs, mu, ctx)
    Tp = _highprec_pinv(T, ctx)
    return np.array([float(-Gt[i, j] * (Tp[i, i] + Tp[j, j] - 2 * Tp[i, j])) for i, j in pairs])


def msp_apply_highprec(n, u, v, w, aggs, mu, r, dps=50):
    """z = P(mu) pinv(L_T~) P(mu)^T r - mean(.), every step of the
    definition carried out densely in mpmath at `dps` digits: P(mu)
    (Sec. 2.2), L_G~ = P(mu)^T L_G P(mu), H~ its positively weighted edges
    (Sec. 3.2), T~ the MSP edges of H~ (Sec. 3.3, same reading as
    msp_from_h), pinv(L) = (L + J/t)^(-1) - J/t for the connected T~ with t
    nodes (J the all-ones matrix).  For tiny graphs only (the expanded
    graph's size cubed mpmath operations): a reference whose rounding is far
    below FP64, for checking FP64 evaluations at any mu."""
    import mpmath as mpm
    ctx = mpm.mp.clone()
    ctx.dps = dps
    Pm, _, T, _ = _highprec_expanded(n, u, v, w, aggs, mu, ctx)
    Tp = _highprec_pinv(T, ctx)
    rm = ctx.matrix([ctx.mpf(float(t)) for t in r])
    z = Pm * (Tp * (Pm.T * rm))
    mean = ctx.fsum(z[i] for i in range(n)) / n
    return np.array([float(z[i] - mean) for i in range(n)])
