"""Graph construction of the setup on the device (LAP_FLAG_DEVICE_SETUP)
against the oracle and the host build.

The device builds the symmetric adjacency and every coarse graph P^T L P
(Sec. 2.2) by stable radix sorts and in-order run sums; the matching stays
on the host.  The hierarchy must be the oracle's bit for bit: level sizes,
aggregate ids, matched flags, and every level's graph with its FP64 weights
exactly (including parallel input edges summed in input order, and coarse
weights summed in fine CSR order).  Solves on the two hierarchies give the
same bits.

With LAP_FLAG_PARALLEL_MATCHING the matching runs on the device too, as
rounds of locally dominant pairs with a thread per vertex; its hierarchy is
compared, bit for bit, with the oracle's greedy matching (a global sort by
edge weight: the same matching by a different algorithm), and a solve on it
with the oracle's solve on that hierarchy.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


def _graphs():
    rng = np.random.default_rng(7)
    out = [("grid2d_17x9", W.grid2d(17, 9), None),
           ("grid3d_9", W.grid3d(9), "loguniform"),
           ("ring_101", W.ring(101), None),
           ("ws_300", W.watts_strogatz(300, 4, 0.1, 4), "loguniform"),
           ("chunglu_3000", W.chung_lu(3000, 8.0, 2.1, 5), "uniform"),
           ("rmat_10", W.rmat(10, 8, seed=6), "uniform"),
           ("complete_9", W.complete(9), None)]
    # parallel edges, both orientations, shuffled order
    n, u, v = W.erdos_renyi(400, 5, 1)
    dup = rng.integers(0, len(u), 300)
    u2 = np.concatenate([u, v[dup], u[dup[:50]]])
    v2 = np.concatenate([v, u[dup], v[dup[:50]]])
    perm = rng.permutation(len(u2))
    out.append(("er_400_parallel_shuffled", (n, u2[perm], v2[perm]), "uniform"))
    return out


def _weights(kind, m, seed):
    if kind is None:
        return W.unit_weights(m)
    if kind == "loguniform":
        return W.loguniform_weights(m, seed)
    return W.uniform01_weights(m, seed)


def _exports(lap, h, info):
    lv = [lap.lap_export_level(h, k, info["sizes"][k]) for k in range(info["nlev"] - 1)]
    gr = [lap.lap_export_graph(h, k, info["sizes"][k]) for k in range(info["nlev"])]
    return lv, gr


@pytest.mark.parametrize("case", range(8))
def test_device_setup_bit_exact(oracle_lib, case):
    from oracle import Graph, Hierarchy
    import paper_2207_07847_amd as lap
    name, (n, u, v), kind = _graphs()[case]
    w = _weights(kind, len(u), 300 + case)
    H = Hierarchy(Graph(n, u, v, w))
    G = GpuLap(n, u, v, w, flags=lap.LAP_FLAG_DEVICE_SETUP)
    try:
        info = G.info
        assert info["sizes"] == H.sizes, name
        lv, gr = _exports(lap, G.h, info)
        for k, (a, m) in enumerate(lv):
            a2, m2 = H.agg(k)
            np.testing.assert_array_equal(a, a2)
            np.testing.assert_array_equal(m, m2)
        for k, (pt, c, ww) in enumerate(gr):
            pt2, c2, w2 = H.level_csr(k)
            np.testing.assert_array_equal(pt, pt2)
            np.testing.assert_array_equal(c, c2)
            np.testing.assert_array_equal(ww, w2)
    finally:
        G.close()
    say(name, "levels", info["nlev"], "sizes", info["sizes"][:4])


def test_device_setup_same_solve(oracle_lib):
    """The same hierarchy: a solve on each gives the same bits."""
    import paper_2207_07847_amd as lap
    n, u, v = W.chung_lu(5000, 8.0, 2.1, 9)
    w = W.uniform01_weights(len(u), 10)
    b = W.gaussian_rhs(n, 11)
    out = []
    for flags in (0, lap.LAP_FLAG_DEVICE_SETUP):
        G = GpuLap(n, u, v, w, flags=flags, max_iter=2000)
        try:
            st, x, info = G.solve(b, 1e-8)
        finally:
            G.close()
        assert st == 0
        out.append((x, info["iterations"]))
    assert out[0][1] == out[1][1]
    np.testing.assert_array_equal(out[0][0], out[1][0])


def test_device_setup_rejects_bad_graph(oracle_lib):
    import paper_2207_07847_amd as lap
    n, u, v = 4, np.array([0, 1, 2]), np.array([1, 2, 2])
    p = lap.lap_default_params(flags=lap.LAP_FLAG_DEVICE_SETUP)
    with pytest.raises(lap.LapError) as e:
        lap.lap_setup(n, u, v, np.ones(3), p)
    assert e.value.status == lap.LAP_EINVAL


@pytest.mark.parametrize("case", range(8))
def test_device_parallel_matching_bit_exact(oracle_lib, case):
    from oracle import Graph, Hierarchy
    import paper_2207_07847_amd as lap
    name, (n, u, v), kind = _graphs()[case]
    w = _weights(kind, len(u), 300 + case)
    H = Hierarchy(Graph(n, u, v, w), matching="greedy")
    G = GpuLap(n, u, v, w, flags=lap.LAP_FLAG_DEVICE_SETUP | lap.LAP_FLAG_PARALLEL_MATCHING)
    try:
        info = G.info
        assert info["sizes"] == H.sizes, name
        lv, gr = _exports(lap, G.h, info)
        for k, (a, m) in enumerate(lv):
            a2, m2 = H.agg(k)
            np.testing.assert_array_equal(a, a2)
            np.testing.assert_array_equal(m, m2)
        for k, (pt, c, ww) in enumerate(gr):
            pt2, c2, w2 = H.level_csr(k)
            np.testing.assert_array_equal(pt, pt2)
            np.testing.assert_array_equal(c, c2)
            np.testing.assert_array_equal(ww, w2)
    finally:
        G.close()
    say(name, "greedy levels", info["nlev"], "sizes", info["sizes"][:4])


def test_parallel_matching_solve(oracle_lib):
    """A solve on the device-matched hierarchy against the oracle's solve on
    its greedy hierarchy: iterations inside the rounding band of the
    evaluation orders (widened by 1), the iterate at the same count within
    1e-7, true residual <= tol."""
    from oracle import Graph, Hierarchy, MSP, pcg
    from oracle.msp_closed import band, closed_form
    import paper_2207_07847_amd as lap
    n, u, v = W.chung_lu(5000, 8.0, 2.1, 9)
    w = W.uniform01_weights(len(u), 10)
    b = W.gaussian_rhs(n, 11)
    g = Graph(n, u, v, w)
    h = Hierarchy(g, matching="greedy")
    B = band(g, b, 1e-8, 2000, h=h, mu=0.8, precond=MSP(h, 0.8))
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=2000,
               flags=lap.LAP_FLAG_DEVICE_SETUP | lap.LAP_FLAG_PARALLEL_MATCHING)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    k = info["iterations"]
    same = pcg(g, b, 0.0, k, closed_form(h, 0.8))
    d = np.linalg.norm(x - same.x) / np.linalg.norm(same.x)
    msg = (f"greedy hierarchy: gpu {k} iterations, oracle {B['oracle']}, band "
           f"[{B['lo'] - 1}, {B['hi'] + 1}], relres {info['relres_true']:.3e}, diff {d:.2e}")
    say(msg)
    assert st == 0 and B["lo"] - 1 <= k <= B["hi"] + 1, msg
    assert info["relres_true"] <= 1e-8 and d <= 1e-7, msg
