"""Pins of the off-tree sparsifier oracle (oracle/offtree.py).

H_k~ = T~ plus the off-tree edges of H~ with the largest stretch in T~
(Sec. 3.3).  Its two ends are other preconditioners computed by other
code: frac = 0 is MSP (the oracle's tree-ordered elimination in C) and
frac = 1 is PEGP (the grounded sparse LU of H~).  In between: each edge's
stretch against a dense pseudo-inverse of L_T~, the selection against a
brute-force ranking, and the pencil of nested subgraphs (T~ in H_k~ in
H~, all positive weights: the eigenvalues of pinv(L_Hk~) L_H~ are >= 1 and
their largest falls as edges are added, from at most the total stretch).
"""
import numpy as np
import pytest

import workloads as W


def _setup(case):
    from oracle import Graph, Hierarchy
    graphs = [W.grid2d(8, 5), W.ring(40), W.erdos_renyi(60, 4, 3), W.grid2d(4)]
    n, u, v = graphs[case]
    w = W.loguniform_weights(len(u), 31 + case, -1, 1)
    mu = [0.3, 0.6, 0.8, 0.5][case]
    h = Hierarchy(Graph(n, u, v, w))
    return n, u, v, w, h, mu


def _rhs(n, seed):
    r = np.random.default_rng(seed).standard_normal(n)
    return r - r.mean()


@pytest.mark.parametrize("case", range(3))
def test_no_offtree_edges_is_msp(oracle_lib, case):
    from oracle import MSP
    from oracle.offtree import OffTree
    n, u, v, w, h, mu = _setup(case)
    r = _rhs(n, case)
    z = OffTree(n, u, v, w, h, mu, 0.0).apply(r)
    z0 = MSP(h, mu).apply(r)
    assert np.linalg.norm(z - z0) <= 1e-10 * np.linalg.norm(z0)


@pytest.mark.parametrize("case", range(3))
def test_all_offtree_edges_is_pegp(oracle_lib, case):
    from oracle.offtree import OffTree
    from oracle.pegp import PEGP
    n, u, v, w, h, mu = _setup(case)
    r = _rhs(n, case)
    M = OffTree(n, u, v, w, h, mu, 1.0)
    assert len(M.kept) == len(M.off)
    z = M.apply(r)
    z0 = PEGP(n, u, v, w, h.aggs(), mu).apply(r)
    assert np.linalg.norm(z - z0) <= 1e-10 * np.linalg.norm(z0)


def _dense(n, u, v, w, h, mu):
    from oracle import dense
    L = dense.laplacian(n, u, v, w)
    Pm = dense.p_mu(h.aggs(), n, mu)
    H = dense.positive_subgraph(dense.expanded(L, Pm))
    T = dense.msp_from_h(H, h.aggs(), dense.level_sizes(h.aggs(), n))
    return H, T


@pytest.mark.parametrize("case", [1, 3])
def test_stretch_and_selection_against_dense(oracle_lib, case):
    from oracle.offtree import OffTree
    n, u, v, w, h, mu = _setup(case)
    H, T = _dense(n, u, v, w, h, mu)
    Tp = np.linalg.pinv(T)
    M = OffTree(n, u, v, w, h, mu, 0.25)
    assert len(M.off) > 4
    s_dense = []
    for (i, j, x) in M.off:
        assert abs(x + H[i, j]) <= 1e-13 * x           # an H~ edge with its weight
        assert T[i, j] == 0.0                           # not a T~ edge
        e = np.zeros(M.nt)
        e[i], e[j] = 1.0, -1.0
        s_dense.append(x * (e @ Tp @ e))
    s_dense = np.array(s_dense)
    np.testing.assert_allclose(M.stretch, s_dense, rtol=1e-9, atol=0)
    # the kept edges are the ceil(count / 4) of largest stretch
    k = int(np.ceil(0.25 * len(M.off)))
    top = set(np.argsort(-s_dense, kind="stable")[:k].tolist())
    assert set(M.kept) == top
    # off-tree plus tree edges are all of H~'s edges (above rounding size)
    deg = np.diag(H)
    nh = int((np.triu(-H, 1) > 1e-12 * np.minimum.outer(deg, deg)).sum())
    assert len(M.off) + len(M.tree[0]) == nh


@pytest.mark.parametrize("case", [1, 3])
def test_nested_sparsifier_pencils(oracle_lib, case):
    from oracle import dense
    from oracle.offtree import OffTree
    n, u, v, w, h, mu = _setup(case)
    H, T = _dense(n, u, v, w, h, mu)
    total = dense.stretch(T, H)
    prev = np.inf
    for frac in (0.0, 0.1, 0.3, 0.6, 1.0):
        Hk = OffTree(n, u, v, w, h, mu, frac).Hk.toarray()
        lam = dense.pencil_eigs(H, Hk)
        nz = lam[lam > 1e-9]
        assert nz.min() >= 1.0 - 1e-9, frac
        assert nz.max() <= prev * (1 + 1e-9), frac
        if frac == 0.0:
            np.testing.assert_allclose(Hk, T, rtol=0, atol=1e-14 * np.abs(T).max())
            assert nz.max() <= total * (1 + 1e-9)
        prev = nz.max()
    assert abs(prev - 1.0) <= 1e-9                      # frac = 1: H_k~ = H~


# The other tree: a maximum-weight spanning tree of H~ (oracle.offtree.SpanningOffTree).

@pytest.mark.parametrize("case", range(4))
def test_spanning_tree_is_a_maximum_weight_spanning_tree(oracle_lib, case):
    """nt - 1 edges of H~ that connect every node, and the largest total
    weight: against scipy's minimum spanning tree of the order-reversed
    weights (every spanning tree has nt - 1 edges, so maximising sum w is
    minimising sum (c - w))."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components, minimum_spanning_tree
    from oracle.offtree import SpanningOffTree, h_edges
    n, u, v, w, h, mu = _setup(case)
    M = SpanningOffTree(n, u, v, w, h, mu, 0.0)
    nt = M.nt
    assert len(M.tree_edges) == nt - 1
    T = sp.coo_matrix(([1.0] * (nt - 1), ([e[0] for e in M.tree_edges],
                                          [e[1] for e in M.tree_edges])), shape=(nt, nt))
    assert connected_components(T, directed=False)[0] == 1
    H, _ = _dense(n, u, v, w, h, mu)
    edges = h_edges(sp.csr_matrix(H))
    c = 1.0 + max(e[2] for e in edges)
    G = sp.coo_matrix(([c - e[2] for e in edges], ([e[0] for e in edges], [e[1] for e in edges])),
                      shape=(nt, nt)).tocsr()
    best = (nt - 1) * c - minimum_spanning_tree(G).sum()
    mine = sum(e[2] for e in M.tree_edges)
    assert abs(mine - best) <= 1e-12 * best
    # every tree edge is an edge of H~ with its weight
    for (i, j, x) in M.tree_edges:
        assert abs(x + H[i, j]) <= 1e-13 * x


@pytest.mark.parametrize("case", [1, 3])
def test_spanning_stretch_is_the_tree_path_resistance(oracle_lib, case):
    """Stretch w_e * R_tree(i, j): R summed along the tree path (1 / weight
    per edge), found by a breadth-first search, not by solves."""
    from collections import deque
    from oracle.offtree import SpanningOffTree
    n, u, v, w, h, mu = _setup(case)
    M = SpanningOffTree(n, u, v, w, h, mu, 0.3)
    adj = {k: [] for k in range(M.nt)}
    for (i, j, x) in M.tree_edges:
        adj[i].append((j, x))
        adj[j].append((i, x))
    for t, (i, j, x) in enumerate(M.off):
        res = {i: 0.0}
        q = deque([i])
        while q:
            a = q.popleft()
            for b, y in adj[a]:
                if b not in res:
                    res[b] = res[a] + 1.0 / y
                    q.append(b)
        assert abs(M.stretch[t] - x * res[j]) <= 1e-12 * x * res[j]
    # the kept edges are the largest stretches
    k = len(M.kept)
    assert k == int(np.ceil(0.3 * len(M.off) - 1e-12))
    thr = min(M.stretch[t] for t in M.kept)
    assert all(M.stretch[t] <= thr for t in range(len(M.off)) if t not in set(M.kept))


@pytest.mark.parametrize("case", range(3))
def test_spanning_ends_tree_alone_and_pegp(oracle_lib, case):
    """frac = 0: P(mu) pinv(L_tree) P(mu)^T r against a dense pseudo-inverse
    of the tree's Laplacian; frac = 1: every edge of H~ is back, PEGP."""
    from oracle import dense
    from oracle.offtree import SpanningOffTree
    from oracle.pegp import PEGP
    n, u, v, w, h, mu = _setup(case)
    r = _rhs(n, 40 + case)
    M0 = SpanningOffTree(n, u, v, w, h, mu, 0.0)
    Lt = np.zeros((M0.nt, M0.nt))
    for (i, j, x) in M0.tree_edges:
        Lt[i, j] -= x
        Lt[j, i] -= x
        Lt[i, i] += x
        Lt[j, j] += x
    Pm = dense.p_mu(h.aggs(), n, mu)
    z0 = Pm @ np.linalg.pinv(Lt) @ Pm.T @ r
    z0 -= z0.mean()
    z = M0.apply(r)
    assert np.linalg.norm(z - z0) <= 1e-9 * np.linalg.norm(z0)
    M1 = SpanningOffTree(n, u, v, w, h, mu, 1.0)
    assert len(M1.kept) == len(M1.off)
    z1 = PEGP(n, u, v, w, h.aggs(), mu).apply(r)
    assert np.linalg.norm(M1.apply(r) - z1) <= 1e-10 * np.linalg.norm(z1)


def test_kruskal_order_takes_near_equal_weights_as_ties():
    """Weights within 1e-9 relative are one run, ordered by pair; a larger
    gap starts a new run; heavier runs first."""
    from oracle.offtree import kruskal_order
    edges = [(0, 5, 1.0), (1, 2, 1.0 + 1e-13), (0, 3, 2.0), (2, 4, 1.0 - 3e-10),
             (3, 4, 1.0 - 5e-8)]
    order = kruskal_order(edges)
    assert [edges[t][:2] for t in order] == [(0, 3), (0, 5), (1, 2), (2, 4), (3, 4)]
