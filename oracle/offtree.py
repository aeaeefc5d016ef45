"""The MSP tree with off-tree edges added back (test infrastructure only).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may use this module; it shares no
code with the GPU library.

Sec. 3.3 bounds kappa(pinv(L_T~) L_G~) by the total stretch of H~'s edges
in the MSP tree T~ over 1 - rho, and notes that sparsifiers made by adding
off-tree edges back to a low-stretch tree are effective in practice; it
does not fix which edges.  The reading used here: the off-tree edges of H~
(its positive edges that are not in T~) are ranked by their stretch in T~
(def. stretch-edge, with the distance through T~ taken as the effective
resistance, as for the total stretch), the ceil(frac * count) largest are
added to T~ (ties to the smaller pair (i, j), i < j), and the result H_k~,
a subgraph of H~ that contains T~, is solved exactly like PEGP: the
grounded, scaled system D L_Hk~ D by a sparse LU.  frac = 0 gives the MSP
preconditioner, frac = 1 the PEGP one.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .pegp import laplacian_sparse, p_mu_sparse, positive_part


def offtree_edges(Ht, tree_u, tree_v):
    """The positive edges of H~ (pairs i < j and their weights) that are not
    edges of T~.  H~ here comes from sparse products, whose cancelling sums
    leave entries of rounding size (~1e-16 of the terms) where the exact
    H~ has none; an entry counts as an edge only above 1e-12 of the smaller
    degree of its two ends."""
    tree = {(min(a, b), max(a, b)) for a, b in zip(tree_u.tolist(), tree_v.tolist())}
    deg = Ht.diagonal()
    U = sp.triu(Ht, k=1).tocoo()
    out = [(int(i), int(j), -float(x)) for i, j, x in zip(U.row, U.col, U.data)
           if -x > 1e-12 * min(deg[i], deg[j]) and (int(i), int(j)) not in tree]
    out.sort()
    return out


def stretch_in_tree(edges, solve_tree, nt):
    """w_e times the effective resistance between the ends of e through T~,
    from grounded solves with L_T~ (any grounding gives the same
    difference y_i - y_j for a right-hand side e_i - e_j)."""
    s = np.empty(len(edges))
    for t, (i, j, w) in enumerate(edges):
        e = np.zeros(nt)
        e[i], e[j] = 1.0, -1.0
        y = solve_tree(e)
        s[t] = w * (y[i] - y[j])
    return s


def select(edges, stretch, frac):
    """Indices of the ceil(frac * count) off-tree edges of largest stretch,
    ties to the smaller pair."""
    k = int(math.ceil(frac * len(edges) - 1e-12))
    order = sorted(range(len(edges)), key=lambda t: (-stretch[t], edges[t][0], edges[t][1]))
    return sorted(order[:k])


def h_edges(Ht):
    """Every positive edge of H~ as (i, j, w), i < j, in (i, j) order (the
    same rounding-size filter as offtree_edges)."""
    return offtree_edges(Ht, np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64))


TIE_REL = 1e-9


def kruskal_order(edges):
    """The order Kruskal takes H~'s edges (i, j, w) in: heaviest first, and
    weights that agree to TIE_REL relative taken as equal (runs of sorted
    weights whose consecutive gaps are all within it), ordered by the
    smaller pair.  H~ has structurally equal weights (the pairs (i,
    parent(j)) and (j, parent(i)) of one fine edge, for one), which
    evaluations of H~ in FP64 may round apart by far less than that."""
    by_w = sorted(range(len(edges)), key=lambda t: -edges[t][2])
    group = {}
    g = 0
    for r, t in enumerate(by_w):
        if r and edges[by_w[r - 1]][2] - edges[t][2] > TIE_REL * edges[by_w[r - 1]][2]:
            g += 1
        group[t] = g
    return sorted(range(len(edges)), key=lambda t: (group[t], edges[t][0], edges[t][1]))


def max_weight_spanning_tree(nt, edges):
    """Kruskal's algorithm on H~'s edges (i, j, w) in kruskal_order; an
    edge joining two components is kept.  Returns the indices of the
    nt - 1 tree edges, in (i, j) order."""
    parent = list(range(nt))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    tree = []
    for t in kruskal_order(edges):
        i, j, _ = edges[t]
        ri, rj = find(i), find(j)
        if ri != rj:
            parent[ri] = rj
            tree.append(t)
    if len(tree) != nt - 1:
        raise ValueError("H~ is not connected")
    return sorted(tree)


def subgraph_laplacian(nt, edges):
    """L of the subgraph with the given (i, j, w) edges on nt nodes."""
    eu = [e[0] for e in edges]
    ev = [e[1] for e in edges]
    ew = [e[2] for e in edges]
    A = sp.coo_matrix((ew, (eu, ev)), shape=(nt, nt)).tocsr()
    A = A + A.T
    return (sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A).tocsr()


def grounded_solver(Lsub):
    """y with Lsub y = e (grounded at the last node); differences y_i - y_j
    do not depend on the grounding."""
    nt = Lsub.shape[0]
    lu = spla.splu(Lsub[:-1, :-1].tocsc())

    def solve(e):
        y = np.zeros(nt)
        y[:-1] = lu.solve(np.asarray(e, dtype=np.float64)[:-1])
        return y

    return solve


class _SubgraphPreconditioner:
    """z = P(mu) pinv(L_S) P(mu)^T r (mean-free) for a subgraph S of H~
    given by its edges, solved like PEGP: the grounded, scaled system
    D L_S D by a sparse LU."""

    def _factor(self, n, aggs, mu, edges, permc_spec):
        self.Hk = subgraph_laplacian(self.nt, edges)
        sizes = [n] + [int(np.max(a)) + 1 for a in aggs]
        self.d = np.concatenate([np.full(s, mu ** (-k)) for k, s in enumerate(sizes)])
        S = (sp.diags(self.d) @ self.Hk @ sp.diags(self.d)).tocsc()
        self._lu = spla.splu(S[:-1, :-1].tocsc(), permc_spec=permc_spec)

    def solve_expanded(self, bt):
        """Grounded solve of L_S y~ = b~ (the last node grounded)."""
        y = np.zeros(self.nt)
        y[:-1] = self._lu.solve((self.d * np.asarray(bt, dtype=np.float64))[:-1])
        return y * self.d

    def apply(self, r):
        y = self.solve_expanded(self.Pmu.T @ np.asarray(r, dtype=np.float64))
        z = self.Pmu @ y
        return z - z.mean()

    __call__ = apply


class SpanningOffTree(_SubgraphPreconditioner):
    """The other tree of Sec. 3.3's remark: a maximum-weight spanning tree
    of H~ (Kruskal), with its off-tree edges of largest stretch added back
    (stretch = w_e times the effective resistance between the ends through
    the tree, ranked and selected as for the MSP tree), solved like PEGP.
    frac = 1 gives PEGP."""

    def __init__(self, n, u, v, w, h, mu, frac, permc_spec="COLAMD"):
        self.n = int(n)
        self.mu = float(mu)
        aggs = h.aggs()
        L = laplacian_sparse(n, np.asarray(u), np.asarray(v), np.asarray(w, dtype=np.float64))
        self.Pmu = p_mu_sparse(aggs, n, mu)
        Ht = positive_part((self.Pmu.T @ L @ self.Pmu).tocsr())
        self.nt = Ht.shape[0]
        edges = h_edges(Ht)
        tree_idx = max_weight_spanning_tree(self.nt, edges)
        in_tree = np.zeros(len(edges), dtype=bool)
        in_tree[tree_idx] = True
        self.tree_edges = [edges[t] for t in tree_idx]
        self.off = [e for e, t in zip(edges, in_tree) if not t]
        solve_tree = grounded_solver(subgraph_laplacian(self.nt, self.tree_edges))
        self.stretch = stretch_in_tree(self.off, solve_tree, self.nt)
        self.kept = select(self.off, self.stretch, frac)
        self._factor(n, aggs, mu, self.tree_edges + [self.off[t] for t in self.kept],
                     permc_spec)


class OffTree:
    """z = P(mu) pinv(L_Hk~) P(mu)^T r (mean-free), H_k~ = T~ plus the
    selected off-tree edges of H~."""

    def __init__(self, n, u, v, w, h, mu, frac, permc_spec="COLAMD"):
        from . import MSP
        self.n = int(n)
        self.mu = float(mu)
        aggs = h.aggs()
        L = laplacian_sparse(n, np.asarray(u), np.asarray(v), np.asarray(w, dtype=np.float64))
        self.Pmu = p_mu_sparse(aggs, n, mu)
        Ht = positive_part((self.Pmu.T @ L @ self.Pmu).tocsr())
        self.nt = Ht.shape[0]
        tu, tv, tw = h.msp_edges(mu)
        self.tree = (tu, tv, tw)
        self.off = offtree_edges(Ht, tu, tv)
        msp = MSP(h, mu)
        self.stretch = stretch_in_tree(self.off, msp.solve_expanded, self.nt)
        self.kept = select(self.off, self.stretch, frac)
        # L_Hk~: the tree's edges with H~'s weights, and the kept edges
        Hc = Ht.tocsr()
        eu = [min(a, b) for a, b in zip(tu.tolist(), tv.tolist())]
        ev = [max(a, b) for a, b in zip(tu.tolist(), tv.tolist())]
        ew = [-float(Hc[a, b]) for a, b in zip(eu, ev)]
        for t in self.kept:
            i, j, x = self.off[t]
            eu.append(i)
            ev.append(j)
            ew.append(x)
        A = sp.coo_matrix((ew, (eu, ev)), shape=(self.nt, self.nt)).tocsr()
        A = A + A.T
        self.Hk = (sp.diags(np.asarray(A.sum(axis=1)).ravel()) - A).tocsr()
        sizes = [n] + [int(np.max(a)) + 1 for a in aggs]
        self.d = np.concatenate([np.full(s, mu ** (-k)) for k, s in enumerate(sizes)])
        S = (sp.diags(self.d) @ self.Hk @ sp.diags(self.d)).tocsc()
        self._lu = spla.splu(S[:-1, :-1].tocsc(), permc_spec=permc_spec)

    def solve_expanded(self, bt):
        """Grounded solve of L_Hk~ y~ = b~ (the last node grounded)."""
        y = np.zeros(self.nt)
        y[:-1] = self._lu.solve((self.d * np.asarray(bt, dtype=np.float64))[:-1])
        return y * self.d

    def apply(self, r):
        y = self.solve_expanded(self.Pmu.T @ np.asarray(r, dtype=np.float64))
        z = self.Pmu @ y
        return z - z.mean()

    __call__ = apply
