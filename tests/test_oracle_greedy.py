"""Pins of the oracle's greedy matching (lr_greedy_match), the aggregation
of the parallel setup.

The greedy matching by a strict total order on edges (weight descending,
then the smaller (i, j)) is characterised by domination: it is the only
matching M in which every edge outside M shares an end with an edge of M
that comes earlier in the order.  Checking that property on a graph
therefore checks the whole matching, independently of how it was computed
(the library computes it by rounds of locally dominant pairs instead).
Also: every maximal matching has at least half the weight of a maximum one
(brute force on tiny graphs), leftovers are pairwise non-adjacent and join
their heaviest neighbour (ties to the smaller id), and pair ids follow the
smaller end."""
import itertools

import numpy as np
import pytest

import workloads as W


def _key(w, i, j):
    a, b = min(i, j), max(i, j)
    return (-w, a, b)


def _edges(n, u, v, w):
    d = {}
    for a, b, c in zip(u.tolist(), v.tolist(), w.tolist()):
        k = (min(a, b), max(a, b))
        d[k] = d.get(k, 0.0) + c
    return d


def _graphs():
    out = []
    for s in range(6):
        n, u, v = W.erdos_renyi(40 + 10 * s, 4, 100 + s)
        # integer weights 1..3: many exact ties
        w = np.random.default_rng(s).integers(1, 4, len(u)).astype(float)
        out.append((f"er_{n}_ties", n, u, v, w))
    n, u, v = W.grid2d(9, 7)
    out.append(("grid_9x7_unit", n, u, v, W.unit_weights(len(u))))
    n, u, v = W.chung_lu(300, 6.0, 2.1, 9)
    out.append(("chunglu_300", n, u, v, W.uniform01_weights(len(u), 3)))
    return out


@pytest.mark.parametrize("case", _graphs(), ids=lambda c: c[0])
def test_greedy_matching_is_the_dominating_matching(oracle_lib, case):
    from oracle import Graph, greedy_match
    name, n, u, v, w = case
    g = Graph(n, u, v, w)
    agg, mt, nc = greedy_match(g)
    E = _edges(n, u, v, w)
    adj = {i: [] for i in range(n)}
    for (a, b), c in E.items():
        adj[a].append((b, c))
        adj[b].append((a, c))
    # the matching: aggregates of two matched vertices
    members = {}
    for i in range(n):
        members.setdefault(int(agg[i]), []).append(i)
    mate = {}
    for J, vs in members.items():
        pair = [i for i in vs if mt[i]]
        assert len(pair) == 2 and (min(pair), max(pair)) in E, (J, vs)
        mate[pair[0]], mate[pair[1]] = pair[1], pair[0]
    assert nc == len(members)
    # ids by the smaller end of each pair
    smaller = sorted(min(i, mate[i]) for i in mate if i < mate[i])
    assert [int(agg[i]) for i in smaller] == list(range(nc))
    # domination: every non-matching edge meets an earlier matching edge
    for (a, b), c in E.items():
        if mate.get(a) == b:
            continue
        dom = [_key(E[(min(x, mate[x]), max(x, mate[x]))], x, mate[x]) for x in (a, b)
               if x in mate]
        assert dom and min(dom) < _key(c, a, b), ((a, b), c)
    # leftovers: non-adjacent, in their heaviest neighbour's aggregate
    for i in range(n):
        if mt[i]:
            continue
        assert all(mt[j] for j, _ in adj[i])
        best = min(adj[i], key=lambda e: (-e[1], e[0]))[0]
        assert agg[i] == agg[best]


def test_greedy_half_of_maximum_weight(oracle_lib):
    """Brute force: a maximal matching weighs at least half a maximum one."""
    from oracle import Graph, greedy_match
    for s in range(5):
        n, u, v = W.erdos_renyi(9, 3, 200 + s)
        w = W.uniform01_weights(len(u), s)
        E = _edges(n, u, v, w)
        g = Graph(n, u, v, w)
        agg, mt, nc = greedy_match(g)
        got = sum(c for (a, b), c in E.items() if agg[a] == agg[b] and mt[a] and mt[b])
        keys = list(E)
        best = 0.0
        for r in range(1, n // 2 + 1):
            for sub in itertools.combinations(keys, r):
                ends = [x for e in sub for x in e]
                if len(set(ends)) == 2 * r:
                    best = max(best, sum(E[e] for e in sub))
        assert got >= 0.5 * best - 1e-12 and got <= best + 1e-12


def test_greedy_hierarchy_levels(oracle_lib):
    """The hierarchy with greedy matching: each level's aggregates are
    those of lr_greedy_match on the level's graph, the coarse graphs are
    Galerkin (P^T L P), and coarsening stops at two nodes."""
    from oracle import Graph, Hierarchy, greedy_match
    n, u, v = W.grid2d(12, 11)
    w = W.loguniform_weights(len(u), 4)
    g = Graph(n, u, v, w)
    h = Hierarchy(g, matching="greedy")
    assert h.sizes[-1] <= 3 and h.sizes[0] == n
    for k in range(h.nlev - 1):
        ptr, col, cw = h.level_csr(k)
        rows = np.repeat(np.arange(h.sizes[k]), np.diff(ptr))
        gk = Graph(h.sizes[k], rows[rows < col], col[rows < col], cw[rows < col])
        a, m, nc = greedy_match(gk)
        a2, m2 = h.agg(k)
        assert np.array_equal(a, a2) and np.array_equal(m, m2) and nc == h.sizes[k + 1]
        L = np.zeros((h.sizes[k],) * 2)
        L[rows, col] = -cw
        L[np.diag_indices_from(L)] = -L.sum(axis=1)
        P = np.zeros((h.sizes[k], nc))
        P[np.arange(h.sizes[k]), a] = 1.0
        ptr1, col1, cw1 = h.level_csr(k + 1)
        rows1 = np.repeat(np.arange(nc), np.diff(ptr1))
        C = np.zeros((nc, nc))
        C[rows1, col1] = -cw1
        C[np.diag_indices_from(C)] = -C.sum(axis=1)
        np.testing.assert_allclose(C, P.T @ L @ P, atol=1e-12 * np.abs(L).max())
