"""GPU checks of the request server (continuous batching over resident
hierarchies): every request's solution meets its tolerance (FP64 true
residual recomputed on the host with the oracle's L), and each result is
the same whether the request ran alone or in a mix with others admitted
and retired around it (columns never mix: the same PCG run per column)."""
import time

import numpy as np
import pytest

import workloads as W
from gpu_util import say, torch_cuda

pytestmark = pytest.mark.gpu


def _pool():
    out = []
    n, u, v = W.grid2d(32)
    out.append((n, u, v, W.unit_weights(len(u))))
    n, u, v = W.grid3d(12, 11, 10)
    out.append((n, u, v, W.loguniform_weights(len(u), 5)))
    n, u, v = W.chung_lu(3000, 12.0, 2.1, 6)
    out.append((n, u, v, W.uniform01_weights(len(u), 7)))
    n, u, v = W.hub_graph(2000, 500, 300, 8)
    out.append((n, u, v, W.uniform01_weights(len(u), 9)))
    return out


class Server:
    def __init__(self, graphs, budget=0):
        import paper_2207_07847_amd as lap
        self.torch = torch_cuda()
        self.lap = lap
        self.graphs = graphs
        self.hs = []
        s = self.torch.cuda.current_stream().cuda_stream
        for (n, u, v, w) in graphs:
            p = lap.lap_default_params(mu=0.8, max_iter=20000, flags=lap.LAP_FLAG_MULTI_RHS)
            self.hs.append(lap.lap_setup(n, u, v, w, p, s))
        self.torch.cuda.synchronize()
        self.srv = lap.lap_server_create(budget)
        self.gid = [lap.lap_server_add(self.srv, h) for h in self.hs]
        self.keep = {}

    def submit(self, tag, g, B, tol):
        n = self.graphs[g][0]
        b = np.ascontiguousarray(B, dtype=np.float64)
        x = np.full(b.shape, np.nan)
        self.keep[tag] = (b, x)
        st = self.lap.lap_server_submit(self.srv, self.gid[g], b.ctypes.data, x.ctypes.data,
                                        b.shape[0], tol, tag)
        assert st == 0
        return x

    def collect(self, count, timeout=120.0):
        res = {}
        t0 = time.time()
        while len(res) < count:
            for r in self.lap.lap_server_poll(self.srv, 256, 100):
                res[r["tag"]] = r
            assert time.time() - t0 < timeout, f"server stalled: {len(res)}/{count}"
        return res

    def close(self):
        self.lap.lap_server_destroy(self.srv)
        for h in self.hs:
            self.lap.lap_free(h)


def _requests(pool, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(count):
        g = int(rng.integers(len(pool)))
        n = pool[g][0]
        m = int(rng.integers(1, 17))
        tol = 1e-8 if rng.random() < 0.5 else 1e-6
        B = rng.standard_normal((m, n)) if rng.random() < 0.5 else W.pair_rhs(n, m, seed + k)
        reqs.append((k, g, B, tol))
    return reqs


def _relres(graph, B, X):
    from oracle import Graph
    n, u, v, w = graph
    g = Graph(n, u, v, w)
    out = []
    for b, x in zip(B, X):
        bh = b - b.mean()
        out.append(np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh))
    return max(out)


def test_serving_mix_equals_alone(oracle_lib):
    pool = _pool()
    reqs = _requests(pool, 48, 2024)
    S = Server(pool)
    try:
        xs = {}
        for k, g, B, tol in reqs:            # all at once: they mix on the GPU
            xs[k] = S.submit(k, g, B, tol)
        res = S.collect(len(reqs))
        assert all(r["status"] == 0 for r in res.values())
        worst = 0.0
        for k, g, B, tol in reqs:
            rel = _relres(pool[g], B, xs[k])
            worst = max(worst, rel / tol)
            assert rel <= 1.01 * tol, (k, rel, tol)
        say("mix: worst relres/tol", worst,
            "max queue", max(r["queue_seconds"] for r in res.values()))
        # the same requests again, one at a time
        diffs = []
        for k, g, B, tol in reqs[::5]:
            x1 = S.submit(10_000 + k, g, B, tol)
            S.collect(1)
            d = np.abs(x1 - xs[k]).max() / np.abs(xs[k]).max()
            diffs.append(d)
        say("alone vs mix: max relative difference", max(diffs))
        assert max(diffs) <= 1e-12
    finally:
        S.close()


def test_serving_small_budget(oracle_lib):
    """A budget that holds one request's staging at a time: requests wait
    for memory, and all complete."""
    pool = _pool()[:2]
    S0 = Server(pool)
    resident = sum(S0.lap.lap_hierarchy_info(h)["device_bytes"] for h in S0.hs)
    S0.close()
    n_max = max(p[0] for p in pool)
    budget = resident + 2 * n_max * 16 * 8 + 1024
    S = Server(pool, budget=budget)
    try:
        reqs = _requests(pool, 12, 7)
        xs = {k: S.submit(k, g, B, tol) for k, g, B, tol in reqs}
        res = S.collect(len(reqs))
        assert all(r["status"] == 0 for r in res.values())
        for k, g, B, tol in reqs:
            assert _relres(pool[g], B, xs[k]) <= 1.01 * tol
    finally:
        S.close()


def test_serving_rejects_bad_requests(oracle_lib):
    pool = _pool()[:1]
    S = Server(pool)
    try:
        lap = S.lap
        n = pool[0][0]
        b = np.zeros((65, n))
        x = np.zeros_like(b)
        assert lap.lap_server_submit(S.srv, 0, b.ctypes.data, x.ctypes.data, 65, 1e-8, 1) \
            == lap.LAP_EINVAL
        assert lap.lap_server_submit(S.srv, 7, b.ctypes.data, x.ctypes.data, 1, 1e-8, 1) \
            == lap.LAP_EINVAL
        assert lap.lap_server_submit(S.srv, 0, b.ctypes.data, x.ctypes.data, 1, 0.0, 1) \
            == lap.LAP_EINVAL
    finally:
        S.close()
