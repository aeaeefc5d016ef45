"""The off-tree sparsifier's selection (Sec. 3.3), host part of lap_setup
(LAP_PREC_OFFTREE and LAP_PREC_SPANNING, host only): the off-tree edges of
H~, their stretches in the tree (the MSP tree T~, or a maximum-weight
spanning tree of H~) and the edges added back.  For the spanning tree an
identical off-tree edge set also means an identical tree, and the unit-
weight grid (every weight a power of two at mu = 0.5, so no rounding in
either H~) has many equal weights, which the tie rule must order alike.

Against the oracle (oracle/offtree.py) at mu >= 0.5: the edge set must be
identical; stretches agree to 1e-9 relative; the kept sets must agree on
every edge whose stretch is not within 1e-9 of the selection threshold.
Below mu = 0.5 the oracle's effective resistances, from its elimination of
T~ with running diagonals, lose accuracy to cancellation (1.4e-8 relative
at mu = 1/8 on an 8 x 8 grid, 0.8 % at mu = 1/16 on 16 x 16), so there the
library's stretches are checked against the definition carried out in
50-digit arithmetic (oracle.dense.offtree_stretch_highprec) instead."""
import numpy as np
import pytest

import workloads as W

CASES = {
    "grid2d_24_loguniform_mu0.5": lambda: (*W.grid2d(24), W.loguniform_weights(1104, 7), 0.5),
    "chunglu_1500_mu0.8": lambda: (*W.chung_lu(1500, 8.0, 2.1, 5), None, 0.8),
    "grid2d_16_unit_mu0.5": lambda: (*W.grid2d(16), W.unit_weights(480), 0.5),
}
TREES = ["msp", "spanning"]


def _case(name):
    n, u, v, w, mu = CASES[name]()
    if w is None:
        w = W.uniform01_weights(len(u), 8)
    assert len(w) == len(u)
    return n, u, v, w, mu


@pytest.mark.parametrize("tree", TREES)
@pytest.mark.parametrize("frac", [0.0, 0.1, 0.3, 1.0])
@pytest.mark.parametrize("name", list(CASES))
def test_offtree_selection_matches_oracle(oracle_lib, name, frac, tree):
    import paper_2207_07847_amd as lap
    from oracle import Graph, Hierarchy
    from oracle.offtree import OffTree, SpanningOffTree
    n, u, v, w, mu = _case(name)
    h = Hierarchy(Graph(n, u, v, w))
    ot = (OffTree if tree == "msp" else SpanningOffTree)(n, u, v, w, h, mu, frac)
    pc = lap.LAP_PREC_OFFTREE if tree == "msp" else lap.LAP_PREC_SPANNING
    H = lap.lap_setup(n, u, v, w, lap.lap_default_params(
        mu=mu, precond=pc, offtree_frac=frac, flags=lap.LAP_FLAG_HOST_ONLY))
    try:
        E = lap.lap_export_offtree(H)
    finally:
        lap.lap_free(H)
    kept_o = set(ot.kept)
    ora = {(i, j): (s, t in kept_o) for t, ((i, j, _), s) in enumerate(zip(ot.off, ot.stretch))}
    gpu = {(int(a), int(b)): (s, bool(k)) for a, b, s, k in zip(E["a"], E["b"], E["stretch"],
                                                                E["kept"])}
    assert set(gpu) == set(ora), (len(gpu), len(ora))
    rel = max((abs(gpu[e][0] - ora[e][0]) / ora[e][0] for e in ora), default=0.0)
    assert rel <= 1e-9, rel
    assert sum(k for _, k in gpu.values()) == len(kept_o)
    if 0 < len(kept_o) < len(ora):
        thr = min(ora[e][0] for e in ora if ora[e][1])
        differ = [e for e in ora if ora[e][1] != gpu[e][1]]
        assert all(abs(ora[e][0] - thr) <= 1e-9 * thr for e in differ), differ[:5]
    # the weights are H~'s: the oracle forms H~ by the sparse products
    # P(mu)^T L P(mu), whose cancelling sums leave up to ~1e-10 relative on
    # small entries; the library sums the fine weights of each pair directly
    wo = {(i, j): x for i, j, x in ot.off}
    assert max((abs(wt - wo[(int(a), int(b))]) / wo[(int(a), int(b))]
                for a, b, wt in zip(E["a"], E["b"], E["w"])), default=0.0) <= 1e-9


def test_offtree_fraction_out_of_range():
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(6)
    for pc in (lap.LAP_PREC_OFFTREE, lap.LAP_PREC_SPANNING):
        for frac in (-0.1, 1.5, float("nan")):
            with pytest.raises(lap.LapError):
                lap.lap_setup(n, u, v, W.unit_weights(len(u)), lap.lap_default_params(
                    precond=pc, offtree_frac=frac, flags=lap.LAP_FLAG_HOST_ONLY))


@pytest.mark.slow
@pytest.mark.parametrize("a", [6, 8])
def test_offtree_stretch_small_mu_highprec(oracle_lib, a):
    """mu = 1/sqrt(n) (Tables 2-3): every off-tree edge's stretch against the
    50-digit definition, weights log-uniform in [0.1, 10]."""
    import paper_2207_07847_amd as lap
    from oracle import Graph, Hierarchy, dense
    n, u, v = W.grid2d(a)
    w = W.loguniform_weights(len(u), 3, -1, 1)
    mu = 1.0 / a
    h = Hierarchy(Graph(n, u, v, w))
    H = lap.lap_setup(n, u, v, w, lap.lap_default_params(
        mu=mu, precond=lap.LAP_PREC_OFFTREE, offtree_frac=0.2, flags=lap.LAP_FLAG_HOST_ONLY))
    try:
        E = lap.lap_export_offtree(H)
    finally:
        lap.lap_free(H)
    pairs = list(zip(E["a"].tolist(), E["b"].tolist()))
    ref = dense.offtree_stretch_highprec(n, u, v, w, h.aggs(), mu, pairs, dps=50)
    rel = np.max(np.abs(E["stretch"] - ref) / ref)
    print(a, "edges", len(pairs), "max rel stretch error", rel)
    assert len(pairs) > 0 and rel <= 1e-12
    # the selection is the top ceil(0.2 count) of these values
    k = int(np.ceil(0.2 * len(pairs) - 1e-12))
    thr = np.sort(ref)[::-1][k - 1]
    far = np.abs(ref - thr) > 1e-9 * thr
    assert np.array_equal(E["kept"][far] == 1, ref[far] >= thr)
