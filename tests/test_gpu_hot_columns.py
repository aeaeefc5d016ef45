"""GPU checks of the hot-column copy of the separate-p SpMV.

On graphs without locality (solved in the tree order of the hierarchy, the
SpMV forming p in a pass of its own), the most referenced columns of L are
read from a compact copy of p.  The copy is formed from the same inputs by
the same fused multiply-add as p itself, so every gathered value, and with
it the whole solve, is the same bit for bit with or without it.  Checked on
a hub graph (a row far above the slice width, read by the heavy-row path)
and a Chung-Lu graph, in FP64 and in mixed precision, with copies of
several sizes (one value, a few, more than the block of the copy kernel,
and every column), and the FP64 solve against the oracle's iteration band
as in the other parity tests.
"""
import contextlib
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def _env(**kv):
    old = {k: os.environ.get(k) for k in kv}
    os.environ.update({k: str(v) for k, v in kv.items()})
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v


def _chunglu():
    n, u, v = W.chung_lu(40000, 16.0, 2.1, 21)
    return n, u, v, W.uniform01_weights(len(u), 22)


def _hub():
    n, u, v = W.hub_graph(20000, 6000, 3000, 7)
    return n, u, v, W.uniform01_weights(len(u), 71)


def _solve(n, u, v, w, b, hot, **params):
    with _env(LAPGPU_SPMV_ORDER="tree", LAPGPU_HOT_COLS=hot):
        G = GpuLap(n, u, v, w, **params)
    try:
        return G.solve(b, 1e-8)
    finally:
        G.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("make", [_chunglu, _hub])
def test_hot_copy_is_bit_identical(oracle_lib, make, precision):
    import paper_2207_07847_amd as lap
    n, u, v, w = make()
    b = W.gaussian_rhs(n, 5)
    prec = lap.LAP_FP64 if precision == "fp64" else lap.LAP_MIXED_FP32_FP64
    st0, x0, i0 = _solve(n, u, v, w, b, 0, precision=prec, max_iter=3000)
    assert st0 == 0, i0
    for hot in (1, 37, 300, n):
        st, x, info = _solve(n, u, v, w, b, hot, precision=prec, max_iter=3000)
        msg = (f"{make.__name__} {precision} hot {hot}: iterations {info['iterations']} vs "
               f"{i0['iterations']}, max |dx| {np.max(np.abs(x - x0)):.3e}")
        say(msg)
        assert st == 0 and info["iterations"] == i0["iterations"], msg
        assert np.array_equal(x, x0), msg


def test_hot_copy_solve_parity(oracle_lib):
    """The FP64 solve with a hot copy of 5,000 columns: true residual <= tol
    on the host and the iterate at the same count equal to the oracle's
    within 1e-7."""
    from oracle import MSP, Graph, Hierarchy, pcg
    n, u, v, w = _chunglu()
    b = W.gaussian_rhs(n, 5)
    st, x, info = _solve(n, u, v, w, b, 5000, max_iter=3000)
    g = Graph(n, u, v, w)
    bh = b - b.mean()
    host = np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)
    ref = pcg(g, b, 0.0, info["iterations"], MSP(Hierarchy(g), 0.8))
    d = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
    msg = f"hot 5000: iterations {info['iterations']} host relres {host:.3e} diff {d:.2e}"
    say(msg)
    assert st == 0 and host <= 1.01e-8 and d <= 1e-7, msg
