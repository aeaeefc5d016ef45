"""GPU checks of the block (multi-right-hand-side) solve: up to 64 columns
advanced together, each with its own PCG scalars and stop test.

Every column must meet what a single solve promises: FP64 true residual
<= tol, recomputed on the host with the oracle's L, and a mean-free x.  On
a small weighted graph every column is also within 1e-7 (relative 2-norm)
of the oracle's solution at tol 1e-13, the solution bar of the single
solves (any iterate with relative residual tol lies within kappa(L) tol of
it; the GPU's are far closer).  Columns that are zero converge at once; a
non-finite column is rejected.
"""
import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


def _host_relres(g, B, X):
    out = []
    for b, x in zip(B, X):
        bh = b - b.mean()
        nb = np.linalg.norm(bh)
        out.append(np.linalg.norm(bh - g.apply(x)) / nb if nb > 0 else 0.0)
    return np.array(out)


CASES = {
    "grid3d_16_pairs": lambda: (*W.config_graph("grid3d_128", 16 / 128), "pairs"),
    "chunglu_20000_pairs": lambda: (*W.chung_lu(20000, 16.0, 2.1, 41),
                                    W.uniform01_weights(len(W.chung_lu(20000, 16.0, 2.1, 41)[1]),
                                                        42), "pairs"),
    "hub_21267_gauss": lambda: (*W.hub_graph(20000, 6000, 3000, 7),
                                W.uniform01_weights(len(W.hub_graph(20000, 6000, 3000, 7)[1]),
                                                    71), "gauss"),
}


def _rhs(kind, n, nrhs, seed):
    if kind == "pairs":
        return W.pair_rhs(n, nrhs, seed)
    return W.gaussian_rhs(n, seed, nrhs).reshape(nrhs, n) if nrhs > 1 else \
        W.gaussian_rhs(n, seed)[None, :]


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("name", list(CASES))
def test_block_residuals(oracle_lib, name, precision):
    import paper_2207_07847_amd as lap
    from oracle import Graph
    n, u, v, w, kind = CASES[name]()
    prec = lap.LAP_MIXED_FP32_FP64 if precision == "mixed" else lap.LAP_FP64
    B = _rhs(kind, n, 64, 51)
    G = GpuLap(n, u, v, w, mu=0.8, precision=prec, max_iter=20000,
               flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        st, X, info = G.solve_many(B, 1e-8)
    finally:
        G.close()
    g = Graph(n, u, v, w)
    rel = _host_relres(g, B, X)
    its = [i["iterations"] for i in info]
    say(name, precision, "status", st, "iterations", min(its), max(its),
        "refinements", info[0]["refinements"], "max host relres", rel.max(),
        "max gpu relres", max(i["relres_true"] for i in info))
    assert st == 0
    assert all(i["status"] == 0 and i["relres_true"] <= 1e-8 for i in info)
    assert rel.max() <= 1.01e-8
    assert np.all(np.abs(X.mean(axis=1)) <= 1e-12 * np.abs(X).max(axis=1))


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_block_matches_single_solves(oracle_lib, precision):
    """Each column of a block solve against the oracle solution at 1e-13,
    within 1e-7 (and the kappa * tol bound, reported)."""
    import paper_2207_07847_amd as lap
    from oracle import MSP, Graph, Hierarchy, pcg
    from oracle.dense import laplacian
    n, u, v = W.chung_lu(1500, 8.0, 2.1, 93)
    w = W.loguniform_weights(len(u), 94, -2.0, 2.0)
    B = W.pair_rhs(n, 64, 95)
    g = Graph(n, u, v, w)
    M = MSP(Hierarchy(g), 0.8)
    ev = np.linalg.eigvalsh(laplacian(n, u, v, w))
    kappa = ev[-1] / ev[1]
    prec = lap.LAP_MIXED_FP32_FP64 if precision == "mixed" else lap.LAP_FP64
    G = GpuLap(n, u, v, w, mu=0.8, precision=prec, max_iter=20000,
               flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        st, X, info = G.solve_many(B, 1e-8)
    finally:
        G.close()
    assert st == 0
    worst = 0.0
    for c in range(0, 64, 7):
        ref = pcg(g, B[c], 1e-13, 20000, M)
        d = np.linalg.norm(X[c] - ref.x) / np.linalg.norm(ref.x)
        worst = max(worst, d)
    msg = f"block {precision} vs oracle: worst diff {worst:.3e}, kappa*tol {kappa * 1e-8:.3e}"
    say(msg)
    assert worst <= 1e-7, msg


def test_block_ragged_columns_and_ld(oracle_lib):
    """70 columns (one full block of 64, then 6) with ld > n; a zero column."""
    import paper_2207_07847_amd as lap
    from oracle import Graph
    n, u, v, w = W.config_graph("grid3d_128", 12 / 128)
    B = W.pair_rhs(n, 70, 61)
    B[5] = 0.0
    G = GpuLap(n, u, v, w, mu=0.8, precision=lap.LAP_MIXED_FP32_FP64, max_iter=20000,
               flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        st, X, info = G.solve_many(B, 1e-8, ld=n + 37)
    finally:
        G.close()
    rel = _host_relres(Graph(n, u, v, w), B, X)
    say("ragged: status", st, "max relres", rel.max(), "zero column it", info[5]["iterations"])
    assert st == 0 and rel.max() <= 1.01e-8
    assert np.all(X[5] == 0.0) and info[5]["iterations"] == 0


def test_block_plain_cg(oracle_lib):
    import paper_2207_07847_amd as lap
    from oracle import Graph
    n, u, v, w = W.config_graph("grid2d_64")
    B = W.pair_rhs(n, 64, 71)
    G = GpuLap(n, u, v, w, precond=lap.LAP_PREC_NONE, precision=lap.LAP_MIXED_FP32_FP64,
               max_iter=50000, flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        st, X, info = G.solve_many(B, 1e-8)
    finally:
        G.close()
    rel = _host_relres(Graph(n, u, v, w), B, X)
    say("plain block: status", st, "max relres", rel.max())
    assert st == 0 and rel.max() <= 1.01e-8


def test_block_nonfinite_column_rejected(oracle_lib):
    import paper_2207_07847_amd as lap
    n, u, v, w = W.config_graph("grid2d_64")
    B = W.pair_rhs(n, 8, 81)
    B[3, 10] = np.nan
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=5000, flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        st, X, info = G.solve_many(B, 1e-8)
    finally:
        G.close()
    assert st == lap.LAP_EINVAL and info[3]["status"] == lap.LAP_EINVAL
    assert all(info[c]["status"] == 0 for c in range(8) if c != 3)


def _hub_case():
    n, u, v = W.hub_graph(20000, 6000, 3000, 7)
    return n, u, v, W.uniform01_weights(len(u), 71)


def test_block_autotuner_choice(oracle_lib):
    """The set-up autotuner picks, for the FP64 block engine and the FP32
    inner one, sizes among its candidates; a block solve with them meets the
    residual bar (a hub graph: rows long enough to be split)."""
    import paper_2207_07847_amd as lap
    from oracle import Graph
    n, u, v, w = _hub_case()
    B = W.gaussian_rhs(n, 52, 64).reshape(64, n)
    G = GpuLap(n, u, v, w, mu=0.8, precision=lap.LAP_MIXED_FP32_FP64, max_iter=20000,
               flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        d = G.info
        st, X, info = G.solve_many(B, 1e-8)
    finally:
        G.close()
    say("autotuner: chunk", d["mm_chunk"], "grid", d["mm_grid"], "seg", d["mm_seg"],
        "seconds", d["mm_tune_seconds"])
    for k in (0, 1):
        assert d["mm_chunk"][k] in (32, 64, 128, 256, 512)
        assert d["mm_grid"][k] in (256, 512, 1024, 2048)
        assert d["mm_seg"][k] in (32, 64, 128, 256)
    assert d["mm_tune_seconds"] > 0.0
    rel = _host_relres(Graph(n, u, v, w), B, X)
    assert st == 0 and rel.max() <= 1.01e-8


@pytest.mark.parametrize("sizes", [(32, 256, 32), (512, 2048, 256)])
def test_block_pinned_sizes(oracle_lib, monkeypatch, sizes):
    """Sizes pinned through the environment are used as given (no tuning)
    and the solve meets the bar with either extreme decomposition."""
    import paper_2207_07847_amd as lap
    from oracle import Graph
    c, g, s = sizes
    monkeypatch.setenv("LAPGPU_MM_CHUNK", str(c))
    monkeypatch.setenv("LAPGPU_MM_GRID", str(g))
    monkeypatch.setenv("LAPGPU_MM_SEG", str(s))
    n, u, v, w = _hub_case()
    B = W.pair_rhs(n, 64, 53)
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=20000, flags=lap.LAP_FLAG_MULTI_RHS)
    try:
        d = G.info
        st, X, info = G.solve_many(B, 1e-8)
    finally:
        G.close()
    say("pinned", sizes, "reported", d["mm_chunk"][0], d["mm_grid"][0], d["mm_seg"][0])
    assert (d["mm_chunk"][0], d["mm_grid"][0], d["mm_seg"][0]) == (c, g, s)
    assert d["mm_chunk"][1] == 0
    rel = _host_relres(Graph(n, u, v, w), B, X)
    assert st == 0 and rel.max() <= 1.01e-8


def test_block_bad_pinned_grid(monkeypatch):
    """A pinned workgroup count outside 1..2048 is rejected by lap_setup."""
    import paper_2207_07847_amd as lap
    from gpu_util import torch_cuda
    torch = torch_cuda()
    monkeypatch.setenv("LAPGPU_MM_GRID", "4096")
    n, u, v, w = W.config_graph("grid2d_64")
    p = lap.lap_default_params(flags=lap.LAP_FLAG_MULTI_RHS)
    with pytest.raises(lap.LapError) as ei:
        lap.lap_setup(n, u, v, w, p, torch.cuda.current_stream().cuda_stream)
    assert ei.value.status == lap.LAP_EINVAL
