"""Seeded synthetic inputs: graphs, edge weights and right-hand sides.

This module only *draws* inputs.  It holds none of the solver's arithmetic
(no Laplacian, no aggregation, no preconditioner), so both the FP64 oracle
under ``oracle/`` and the GPU library may be fed from it without sharing any
code of the method.

Every generator is a pure function of its arguments and an integer seed
(numpy's PCG64 bit generator).  Graphs are returned as undirected edge lists
``(n, u, v)`` with ``u < v``, no self-loops and no duplicate pairs.

The graph families follow the paper's experiments: 2D regular grids and ring
graphs of average degree 4 (Sec. 3.2, Tables 1-2; Sec. 4.1, Table 3),
Watts-Strogatz rings (Sec. 4.2) and, standing in for the SNAP / UF real-world
graphs of Sec. 4.3 (not available here), seeded Chung-Lu and R-MAT power-law
graphs reduced to their largest connected component with self-loops dropped,
which is the preprocessing that section describes.
"""
from __future__ import annotations

import numpy as np

MASTER_SEED = 20220715

__all__ = [
    "MASTER_SEED", "grid2d", "grid3d", "path", "cycle", "ring", "complete",
    "erdos_renyi", "watts_strogatz", "chung_lu", "rmat", "largest_component",
    "unit_weights", "loguniform_weights", "uniform01_weights", "gaussian_rhs",
    "lowfreq_rhs", "pair_rhs", "config_graph",
]


def _canon(n, u, v):
    """Canonical simple undirected edge list: u<v, unique, sorted."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(n) + hi)
    return int(n), key // n, key % n


# ---------------------------------------------------------------- structured


def grid2d(a, b=None):
    """a x b 5-point grid, row-major ids, edges (i,i+1) in rows and (i,i+a)."""
    b = a if b is None else b
    idx = np.arange(a * b, dtype=np.int64).reshape(b, a)
    u = [idx[:, :-1].ravel(), idx[:-1, :].ravel()]
    v = [idx[:, 1:].ravel(), idx[1:, :].ravel()]
    return _canon(a * b, np.concatenate(u), np.concatenate(v))


def grid3d(a, b=None, c=None):
    """a x b x c 7-point grid, ids x + a*(y + b*z)."""
    b = a if b is None else b
    c = a if c is None else c
    idx = np.arange(a * b * c, dtype=np.int64).reshape(c, b, a)
    u = [idx[:, :, :-1].ravel(), idx[:, :-1, :].ravel(), idx[:-1, :, :].ravel()]
    v = [idx[:, :, 1:].ravel(), idx[:, 1:, :].ravel(), idx[1:, :, :].ravel()]
    return _canon(a * b * c, np.concatenate(u), np.concatenate(v))


def path(n):
    i = np.arange(n - 1, dtype=np.int64)
    return _canon(n, i, i + 1)


def cycle(n):
    i = np.arange(n, dtype=np.int64)
    return _canon(n, i, (i + 1) % n)


def ring(n, k=2):
    """Ring lattice of average degree 2k: edges (i, i+d mod n), d=1..k."""
    i = np.arange(n, dtype=np.int64)
    u = np.concatenate([i] * k)
    v = np.concatenate([(i + d) % n for d in range(1, k + 1)])
    return _canon(n, u, v)


def complete(n):
    u, v = np.triu_indices(n, 1)
    return _canon(n, u, v)


# ---------------------------------------------------------------- random


def largest_component(n, u, v, w=None):
    """Keep the largest connected component, relabelled by ascending old id."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.coo_matrix((np.ones(len(u)), (u, v)), shape=(n, n))
    ncomp, lab = connected_components(a, directed=False)
    if ncomp == 1:
        return (n, u, v) if w is None else (n, u, v, w)
    big = np.argmax(np.bincount(lab))
    keep = lab == big
    newid = np.full(n, -1, dtype=np.int64)
    newid[keep] = np.arange(int(keep.sum()), dtype=np.int64)
    ek = keep[u] & keep[v]
    out = (int(keep.sum()), newid[u[ek]], newid[v[ek]])
    return out if w is None else out + (w[ek],)


def erdos_renyi(n, mean_degree, seed):
    rng = np.random.default_rng(seed)
    m = int(round(n * mean_degree / 2))
    u = rng.integers(0, n, m)
    v = rng.integers(0, n, m)
    n2, u2, v2 = _canon(n, u, v)
    return largest_component(n2, u2, v2)


def watts_strogatz(n, k, beta, seed):
    """Ring lattice of degree k (k even), each edge's far end rewired with
    probability beta to a uniform vertex (loops and duplicates dropped)."""
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.int64)
    u = np.concatenate([i] * (k // 2))
    v = np.concatenate([(i + d) % n for d in range(1, k // 2 + 1)])
    rew = rng.random(len(u)) < beta
    v = v.copy()
    v[rew] = rng.integers(0, n, int(rew.sum()))
    n2, u2, v2 = _canon(n, u, v)
    return largest_component(n2, u2, v2)


def chung_lu(n, mean_degree=16.0, gamma=2.1, seed=0):
    """Chung-Lu power-law graph.

    Expected degrees w_i ~ (i+1)^(-1/(gamma-1)) scaled to the requested mean,
    capped at sqrt(n*mean); n*mean/2 endpoint pairs are drawn with both ends
    proportional to w; duplicates and loops dropped; largest component kept.
    """
    rng = np.random.default_rng(seed)
    wdeg = (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))
    wdeg *= mean_degree / wdeg.mean()
    np.minimum(wdeg, np.sqrt(n * mean_degree), out=wdeg)
    cdf = np.cumsum(wdeg)
    cdf /= cdf[-1]
    m = int(round(n * mean_degree / 2))
    # inverse-CDF draws of both endpoints; sorted queries make the searches
    # cache-friendly, and a random permutation of the second end pairs them
    u = np.searchsorted(cdf, np.sort(rng.random(m)), side="right")
    v = np.searchsorted(cdf, np.sort(rng.random(m)), side="right")[rng.permutation(m)]
    np.minimum(u, n - 1, out=u)
    np.minimum(v, n - 1, out=v)
    n2, u2, v2 = _canon(n, u, v)
    return largest_component(n2, u2, v2)


def hub_graph(n_base, hub_links, pendants, seed=0):
    """A Chung-Lu graph on n_base ids plus one hub vertex linked to
    `hub_links` random base vertices and to `pendants` new degree-1
    vertices: a row far above any slice width, and an aggregate with
    thousands of children (the pendants can only join the hub)."""
    rng = np.random.default_rng(seed)
    n0, u0, v0 = chung_lu(n_base, 8.0, 2.1, seed)
    hub = n0
    links = rng.choice(n0, size=min(hub_links, n0), replace=False)
    pend = np.arange(n0 + 1, n0 + 1 + pendants)
    u = np.concatenate([u0, np.full(len(links), hub), np.full(pendants, hub)])
    v = np.concatenate([v0, links, pend])
    return _canon(n0 + 1 + pendants, u, v)


def rmat(scale, edge_factor=16, abcd=(0.57, 0.19, 0.19, 0.05), seed=0):
    """R-MAT graph on 2^scale ids with edge_factor*2^scale samples."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    a, b, c, _ = abcd
    u = np.zeros(m, dtype=np.int64)
    v = np.zeros(m, dtype=np.int64)
    for bit in range(scale):
        r = rng.random(m)
        ubit = r >= a + b                      # quadrants c or d
        vbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
        u |= ubit.astype(np.int64) << bit
        v |= vbit.astype(np.int64) << bit
    n2, u2, v2 = _canon(n, u, v)
    return largest_component(n2, u2, v2)


# ---------------------------------------------------------------- weights


def unit_weights(m):
    return np.ones(m, dtype=np.float64)


def loguniform_weights(m, seed, lo_exp=-3.0, hi_exp=3.0):
    """w = 10^U(lo_exp, hi_exp)."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(lo_exp, hi_exp, m)


def uniform01_weights(m, seed):
    """w ~ U(0,1] drawn as 1 - U[0,1)."""
    rng = np.random.default_rng(seed)
    return 1.0 - rng.random(m)


# ---------------------------------------------------------------- right-hand sides


def gaussian_rhs(n, seed, nrhs=1):
    """Standard normal entries; the solver projects out the mean itself."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((nrhs, n))
    return b[0] if nrhs == 1 else b


def lowfreq_rhs(n):
    """b = [1, 1, ..., 1, 1-n] (the paper's low-frequency RHS, Sec. 4)."""
    b = np.ones(n, dtype=np.float64)
    b[-1] = 1.0 - n
    return b


def pair_rhs(n, nrhs, seed):
    """nrhs columns e_i - e_j for uniformly drawn distinct pairs (i, j)."""
    rng = np.random.default_rng(seed)
    b = np.zeros((nrhs, n), dtype=np.float64)
    for k in range(nrhs):
        i, j = rng.choice(n, 2, replace=False)
        b[k, i] = 1.0
        b[k, j] = -1.0
    return b


# ---------------------------------------------------------------- named workloads


def config_graph(name, scale=1.0):
    """Named workloads with their full sizes (scale<1 shrinks the linear size).

    grid2d_64      : 64x64 5-point grid, unit weights (PEGP, mu = 1/64)
    grid3d_128     : 128^3 7-point grid, weights 10^U(-3,3) (MSP, mu = 0.8)
    chunglu_4m     : Chung-Lu, 4M ids, mean degree 16, gamma 2.1, U(0,1]
    rmat_20        : R-MAT scale 20, 16 samples/id, U(0,1]
    Returns (n, u, v, w).
    """
    if name == "grid2d_64":
        a = max(2, int(round(64 * scale)))
        n, u, v = grid2d(a)
        return n, u, v, unit_weights(len(u))
    if name == "grid3d_128":
        a = max(2, int(round(128 * scale)))
        n, u, v = grid3d(a)
        return n, u, v, loguniform_weights(len(u), MASTER_SEED + 2)
    if name == "chunglu_4m":
        n0 = max(64, int(round(4_000_000 * scale)))
        n, u, v = chung_lu(n0, 16.0, 2.1, MASTER_SEED + 4)
        return n, u, v, uniform01_weights(len(u), MASTER_SEED + 4 + 1000)
    if name == "rmat_20":
        sc = max(6, int(round(20 + np.log2(scale))))
        n, u, v = rmat(sc, 16, seed=MASTER_SEED + 5)
        return n, u, v, uniform01_weights(len(u), MASTER_SEED + 5 + 1000)
    raise KeyError(name)
