"""GPU checks of the off-tree sparsifiers (Sec. 3.3): a tree with the
off-tree edges of H~ of largest stretch added back, solved like PEGP on
that subgraph (explicit operator or factor, both tested) and applied
through the lifting of Sec. 3.1; the tree is the MSP tree T~
(LAP_PREC_OFFTREE) or a maximum-weight spanning tree of H~
(LAP_PREC_SPANNING).

Against the oracle (oracle/offtree.py), at mu where its stretches are
accurate (the host tests check the selection itself): the applied
preconditioner within 100 x the rounding spread of the oracle's own direct
solve under two fill orderings (the PEGP bar), at frac 0.1 and 0.3 and at
the two ends (frac 0: the MSP tree alone; frac 1: all of H~, the PEGP
preconditioner); whole solves with the iterate at the same count within
1e-7 and the true residual <= tol, and iteration counts inside the range
that rounding order alone gives, widened by 1: the oracle's solve, the same
operator formed explicitly (columns M (e_j - 1/n)) and its symmetric part,
each with the rounding model's eight seeds and with correctly rounded sums
(on the weighted grid at mu = 0.5 these span 499 to 509 iterations)."""
import contextlib
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu

CASES = {
    "grid2d_24_loguniform_mu0.5": lambda: (*W.grid2d(24), "log", 0.5),
    "chunglu_1500_mu0.8": lambda: (*W.chung_lu(1500, 8.0, 2.1, 5), "u01", 0.8),
}


def _case(name):
    n, u, v, kind, mu = CASES[name]()
    w = W.loguniform_weights(len(u), 7) if kind == "log" else W.uniform01_weights(len(u), 8)
    return n, u, v, w, mu


@contextlib.contextmanager
def _mode(mode):
    old = os.environ.get("LAPGPU_PEGP_OPERATOR")
    os.environ["LAPGPU_PEGP_OPERATOR"] = "1" if mode == "operator" else "0"
    try:
        yield
    finally:
        if old is None:
            del os.environ["LAPGPU_PEGP_OPERATOR"]
        else:
            os.environ["LAPGPU_PEGP_OPERATOR"] = old


TREES = ["msp", "spanning"]


def _oracle_cls(tree):
    from oracle.offtree import OffTree, SpanningOffTree
    return OffTree if tree == "msp" else SpanningOffTree


def _gpu(n, u, v, w, mu, frac, mode, tree="msp", **kw):
    import paper_2207_07847_amd as lap
    pc = lap.LAP_PREC_OFFTREE if tree == "msp" else lap.LAP_PREC_SPANNING
    with _mode(mode):
        return GpuLap(n, u, v, w, mu=mu, precond=pc, offtree_frac=frac, **kw)


@pytest.mark.parametrize("tree", TREES)
@pytest.mark.parametrize("mode", ["operator", "factor"])
@pytest.mark.parametrize("frac", [0.0, 0.1, 0.3, 1.0])
@pytest.mark.parametrize("name", list(CASES))
def test_offtree_apply_parity(oracle_lib, name, frac, mode, tree):
    from oracle import Graph, Hierarchy
    n, u, v, w, mu = _case(name)
    h = Hierarchy(Graph(n, u, v, w))
    M = _oracle_cls(tree)(n, u, v, w, h, mu, frac)
    M2 = _oracle_cls(tree)(n, u, v, w, h, mu, frac, permc_spec="MMD_AT_PLUS_A")
    r = np.random.default_rng(13).standard_normal(n)
    r -= r.mean()
    z0 = M.apply(r)
    spread = np.linalg.norm(M2.apply(r) - z0) / np.linalg.norm(z0)
    G = _gpu(n, u, v, w, mu, frac, mode, tree)
    try:
        z = G.apply_precond(r)
    finally:
        G.close()
    err = np.linalg.norm(z - z0) / np.linalg.norm(z0)
    msg = (f"{name} {tree} frac {frac} ({mode}): kept {len(M.kept)} of {len(M.off)} off-tree edges, "
           f"rel err {err:.3e}, oracle ordering spread {spread:.3e}")
    say(msg)
    assert err <= max(100 * spread, 1e-14), msg


@pytest.mark.parametrize("tree", TREES)
@pytest.mark.parametrize("name,frac", [("grid2d_24_loguniform_mu0.5", 0.1),
                                       ("chunglu_1500_mu0.8", 0.3)])
def test_offtree_solve(oracle_lib, name, frac, tree):
    from oracle import Graph, Hierarchy, iteration_band, pcg
    n, u, v, w, mu = _case(name)
    g = Graph(n, u, v, w)
    M = _oracle_cls(tree)(n, u, v, w, Hierarchy(g), mu, frac)
    b = W.gaussian_rhs(n, 44)
    ref = pcg(g, b, 1e-8, 2000, M)
    D = np.empty((n, n))
    for j in range(n):
        e = np.full(n, -1.0 / n)
        e[j] += 1.0
        D[:, j] = M.apply(e)
    Ds = 0.5 * (D + D.T)
    from oracle.msp_closed import pcg_exact_sums
    its = []
    for op in (M.apply, lambda r: D @ r, lambda r: Ds @ r):
        its += list(iteration_band(g, b, 1e-8, 2000, op))
        its.append(pcg_exact_sums(g, op, b, 1e-8, 2000)[0])
    lo, hi = min(its), max(its)
    G = _gpu(n, u, v, w, mu, frac, "operator", tree, max_iter=2000)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    k = info["iterations"]
    same = pcg(g, b, 0.0, k, M)
    d = np.linalg.norm(x - same.x) / np.linalg.norm(same.x)
    bh = b - b.mean()
    host = np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)
    msg = (f"{name} {tree} frac {frac}: gpu status {st} iterations {k}, oracle {ref.iterations}, "
           f"band [{lo - 1}, {hi + 1}]; relres {info['relres_true']:.3e} host {host:.3e}; "
           f"iterate diff at the same count {d:.2e}")
    say(msg)
    assert st == 0 and lo - 1 <= k <= hi + 1, msg
    assert info["relres_true"] <= 1e-8 and host <= 1.01e-8 and d <= 1e-7, msg
