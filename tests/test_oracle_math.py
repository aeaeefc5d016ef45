"""Pins of the FP64 oracle against closed forms, invariants and brute force.

These check the oracle against facts fixed by mathematics rather than by
its own formulas: Laplacian spectra of paths, cycles and grids; the null
spaces stated in Sec. 3.1 and Lemma lem:dim_G_tilde; the lifting theorem;
the spectral bounds of Lemma lem:upper and of the sparsifier (Sec. 3.3);
dense pseudo-inverse solves on tiny graphs; structural properties of the
matching (Sec. 2.2); error handling of invalid input.
"""
import numpy as np
import pytest

import workloads as W


def _graph(n, u, v, w=None):
    from oracle import Graph
    return Graph(n, u, v, np.ones(len(u)) if w is None else w)


# ------------------------------------------------------------- Laplacian


@pytest.mark.parametrize("n", [2, 7, 64])
def test_path_spectrum(oracle_lib, n):
    """Path P_n: eigenpairs 2 - 2 cos(pi k/n), cos(pi k (i + 1/2)/n)."""
    g = _graph(*W.path(n))
    i = np.arange(n)
    for k in range(n):
        x = np.cos(np.pi * k * (i + 0.5) / n)
        lam = 2 - 2 * np.cos(np.pi * k / n)
        np.testing.assert_allclose(g.apply(x), lam * x, atol=1e-12)


@pytest.mark.parametrize("n", [3, 8, 65])
def test_cycle_spectrum(oracle_lib, n):
    """Cycle C_n: eigenpairs 2 - 2 cos(2 pi k/n), cos(2 pi k i/n)."""
    g = _graph(*W.cycle(n))
    i = np.arange(n)
    for k in range(n):
        x = np.cos(2 * np.pi * k * i / n)
        np.testing.assert_allclose(g.apply(x), (2 - 2 * np.cos(2 * np.pi * k / n)) * x,
                                   atol=1e-12)


def test_grid_spectrum(oracle_lib):
    """a x b grid = Kronecker sum of paths: eigenvalues add, vectors multiply."""
    a, b = 5, 4
    g = _graph(*W.grid2d(a, b))
    xs, ys = np.meshgrid(np.arange(a), np.arange(b))
    for p in range(a):
        for q in range(b):
            x = (np.cos(np.pi * p * (xs + 0.5) / a) * np.cos(np.pi * q * (ys + 0.5) / b)).ravel()
            lam = 4 - 2 * np.cos(np.pi * p / a) - 2 * np.cos(np.pi * q / b)
            np.testing.assert_allclose(g.apply(x), lam * x, atol=1e-12)


def test_laplacian_matches_incidence_definition(oracle_lib):
    """L_G = B^T W B (Sec. 2.1) with random weights; constants map to 0 exactly."""
    from oracle import dense
    n, u, v = W.erdos_renyi(40, 5, 1)
    w = W.loguniform_weights(len(u), 2)
    g = _graph(n, u, v, w)
    L = dense.laplacian(n, u, v, w)
    x = np.random.default_rng(0).standard_normal(n)
    np.testing.assert_allclose(g.apply(x), L @ x, rtol=1e-13, atol=1e-12)
    assert np.all(g.apply(np.full(n, 3.7)) == 0.0)


def test_parallel_edges_summed(oracle_lib):
    from oracle import Graph
    g1 = Graph(3, [0, 1, 0], [1, 2, 1], [1.0, 2.0, 0.5])
    g2 = Graph(3, [0, 1], [1, 2], [1.5, 2.0])
    x = np.array([1.0, -2.0, 0.25])
    np.testing.assert_array_equal(g1.apply(x), g2.apply(x))


@pytest.mark.parametrize("bad", [
    dict(u=[0, 1], v=[1, 1], w=[1.0, 1.0]),       # self-loop
    dict(u=[0, 1], v=[1, 3], w=[1.0, 1.0]),       # id out of range
    dict(u=[0, 1], v=[1, 2], w=[1.0, 0.0]),       # zero weight
    dict(u=[0, 1], v=[1, 2], w=[1.0, -1.0]),      # negative weight
    dict(u=[0, 1], v=[1, 2], w=[1.0, np.nan]),    # NaN
    dict(u=[0, 1], v=[1, 2], w=[1.0, np.inf]),    # Inf
])
def test_invalid_graph_rejected(oracle_lib, bad):
    from oracle import EINVAL, Graph, OracleError
    with pytest.raises(OracleError) as e:
        Graph(3, bad["u"], bad["v"], bad["w"])
    assert e.value.code == EINVAL


def test_disconnected_rejected(oracle_lib):
    from oracle import EDISCONNECTED, Graph, Hierarchy, OracleError
    g = Graph(4, [0, 2], [1, 3], [1.0, 1.0])
    assert not g.connected()
    with pytest.raises(OracleError) as e:
        Hierarchy(g)
    assert e.value.code == EDISCONNECTED


# ------------------------------------------------------------ aggregation


def _check_matching(g_edges, agg, matched):
    n, u, v, w = g_edges
    nbr = [dict() for _ in range(n)]
    for a, b, c in zip(u, v, w):
        nbr[a][b] = nbr[a].get(b, 0.0) + c
        nbr[b][a] = nbr[b].get(a, 0.0) + c
    nc = agg.max() + 1
    for J in range(nc):
        mem = np.flatnonzero(agg == J)
        pair = mem[matched[mem]]
        assert len(pair) == 2, "each aggregate holds exactly one matched pair"
        assert pair[1] in nbr[pair[0]], "matched nodes are adjacent"
        for x in mem[~matched[mem]]:
            # a leftover: all neighbours matched; it joined its heaviest one
            assert all(matched[y] for y in nbr[x])
            best = max(nbr[x].items(), key=lambda kv: (kv[1], -kv[0]))[0]
            assert agg[best] == J


@pytest.mark.parametrize("seed", [0, 11])
def test_mwm_structure(oracle_lib, seed):
    """Sec. 2.2: pairs joined by an edge, leftovers to the heaviest neighbour."""
    from oracle import Hierarchy
    n, u, v = W.erdos_renyi(300, 3, 5)
    w = W.uniform01_weights(len(u), 6)
    g = _graph(n, u, v, w)
    h = Hierarchy(g, seed=seed)
    agg, matched = h.agg(0)
    _check_matching((n, u, v, w), agg, matched)
    assert h.sizes[-1] >= 2 and all(a > b for a, b in zip(h.sizes, h.sizes[1:]))


def test_mwm_natural_order_greedy(oracle_lib):
    """Natural order on a weighted path 0-1-2-3 with w=(1,3,2): vertex 0
    pairs with 1 (its only free neighbour), then 2 with 3."""
    g = _graph(4, np.array([0, 1, 2]), np.array([1, 2, 3]), np.array([1.0, 3.0, 2.0]))
    nc, agg, matched = g.mwm()
    assert nc == 2 and list(agg) == [0, 0, 1, 1] and matched.all()


def test_mwm_heaviest_free_neighbour(oracle_lib):
    """Star centre 0 visited first picks its heaviest neighbour (ties to the
    smaller id); the other leaves become leftovers of that aggregate."""
    g = _graph(5, np.array([0, 0, 0, 0]), np.array([1, 2, 3, 4]), np.array([1.0, 5.0, 5.0, 2.0]))
    nc, agg, matched = g.mwm()
    assert nc == 1 and list(agg) == [0, 0, 0, 0, 0]
    assert list(matched) == [True, False, True, False, False]


def test_galerkin_coarse_graph(oracle_lib):
    """Coarse Laplacians equal (P^k)^T L_G P^k (Sec. 3.1 block diagonal)."""
    from oracle import Hierarchy, dense
    n, u, v = W.erdos_renyi(120, 4, 9)
    w = W.loguniform_weights(len(u), 3)
    g = _graph(n, u, v, w)
    h = Hierarchy(g)
    L = dense.laplacian(n, u, v, w)
    Ps = dense.composite(h.aggs(), n)
    for k in range(1, h.nlev):
        ptr, col, cw = h.level_csr(k)
        nk = h.sizes[k]
        A = np.zeros((nk, nk))
        for i in range(nk):
            for q in range(ptr[i], ptr[i + 1]):
                A[i, col[q]] -= cw[q]
                A[i, i] += cw[q]
        np.testing.assert_allclose(A, Ps[k].T @ L @ Ps[k], rtol=1e-12, atol=1e-12)


def test_never_one_node_top(oracle_lib):
    """A 3-node level is not coarsened into one node."""
    from oracle import Hierarchy
    g = _graph(*W.path(3))
    assert Hierarchy(g).sizes == [3]
    g = _graph(*W.path(6))
    assert Hierarchy(g).sizes[-1] >= 2


# ----------------------------------------------------- expanded operators


def _expanded(n, u, v, w, mu, **kw):
    from oracle import Hierarchy, dense
    g = _graph(n, u, v, w)
    h = Hierarchy(g, **kw)
    L = dense.laplacian(n, u, v, w)
    Pm = dense.p_mu(h.aggs(), n, mu)
    Gt = dense.expanded(L, Pm)
    return g, h, L, Pm, Gt


@pytest.mark.parametrize("mu", [0.2, 0.8])
def test_expanded_null_space(oracle_lib, mu):
    """Sec. 3.1: P(mu) 1 = c 1 and L_G~ 1 = 0; Lemma lem:dim_G_tilde:
    dim Null(L_G~) = n~ - n + 1."""
    n, u, v = W.grid2d(6, 5)
    w = W.loguniform_weights(len(u), 4, -1, 1)
    g, h, L, Pm, Gt = _expanded(n, u, v, w, mu)
    nt = h.ntilde
    c = sum((-mu) ** k for k in range(h.nlev))
    np.testing.assert_allclose(Pm @ np.ones(nt), c * np.ones(n), atol=1e-14)
    np.testing.assert_allclose(Gt @ np.ones(nt), 0.0, atol=1e-12)
    ev = np.linalg.eigvalsh(Gt)
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == nt - n + 1


def test_restrict_prolong_are_transposes(oracle_lib):
    from oracle import Hierarchy, dense
    n, u, v = W.ring(50)
    g = _graph(n, u, v)
    h = Hierarchy(g)
    mu = 0.6
    Pm = dense.p_mu(h.aggs(), n, mu)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(n)
    y = rng.standard_normal(h.ntilde)
    np.testing.assert_allclose(h.restrict_mu(mu, r), Pm.T @ r, atol=1e-13)
    np.testing.assert_allclose(h.prolong_mu(mu, y), Pm @ y, atol=1e-13)


def test_lifting_theorem(oracle_lib):
    """Theorem of Sec. 3.1: L_G~ x~ = P(mu)^T b implies L_G P(mu) x~ = b."""
    n, u, v = W.erdos_renyi(50, 4, 2)
    w = W.uniform01_weights(len(u), 2)
    g, h, L, Pm, Gt = _expanded(n, u, v, w, 0.7)
    b = np.random.default_rng(1).standard_normal(n)
    b -= b.mean()
    xt = np.linalg.pinv(Gt) @ (Pm.T @ b)
    np.testing.assert_allclose(L @ (Pm @ xt), b, atol=1e-10)


@pytest.mark.parametrize("mu", [0.1, 0.5, 0.9])
def test_pegp_spectral_bounds(oracle_lib, mu):
    """Lemma lem:upper: eigenvalues of pinv(L_H~) L_G~ lie in [0, 1];
    L_G~ = L_H~ - L_mu^- with L_mu^- positive semidefinite."""
    from oracle import dense
    n, u, v = W.watts_strogatz(60, 4, 0.2, 8)
    w = W.loguniform_weights(len(u), 8, -1, 1)
    g, h, L, Pm, Gt = _expanded(n, u, v, w, mu)
    H = dense.positive_subgraph(Gt)
    N = dense.negative_part(Gt)
    np.testing.assert_allclose(H - N, Gt, atol=1e-12)
    assert np.linalg.eigvalsh(N).min() > -1e-10
    off = H - np.diag(np.diag(H))
    assert off.max() <= 0.0
    ev = dense.pencil_eigs(Gt, H)
    assert ev.max() <= 1.0 + 1e-9 and ev.min() >= -1e-9


def test_msp_subgraph_and_stretch(oracle_lib):
    """Sec. 3.3: T~ is a subgraph of H~ with positive weights, so the
    eigenvalues of pinv(L_T~) L_H~ are >= 1; its largest one is bounded by
    the total stretch (here sum of w_e times the effective resistance of e
    in T~, a lower bound of the path-sum stretch)."""
    from oracle import dense
    n, u, v = W.grid2d(5, 4)
    w = W.loguniform_weights(len(u), 5, -1, 1)
    mu = 0.5
    g, h, L, Pm, Gt = _expanded(n, u, v, w, mu)
    H = dense.positive_subgraph(Gt)
    eu, ev_, ew = h.msp_edges(mu)
    T = dense.edges_to_dense(h.ntilde, eu, ev_, ew)
    assert np.all(ew > 0)
    # every T~ edge is an H~ edge with the same weight
    for a, b, c in zip(eu, ev_, ew):
        assert abs(-H[a, b] - c) <= 1e-14 * c
    lam = dense.pencil_eigs(H, T)
    nz = lam[lam > 1e-9]
    assert nz.min() >= 1.0 - 1e-9
    assert nz.max() <= dense.stretch(T, H) * (1 + 1e-9)


@pytest.mark.parametrize("case", range(4))
def test_msp_edges_equal_extraction_from_h(oracle_lib, case):
    """T~ built from the hierarchy equals T~ extracted from the dense H~."""
    from oracle import dense
    graphs = [W.grid2d(4), W.grid2d(8, 5), W.ring(40), W.erdos_renyi(60, 4, 3)]
    n, u, v = graphs[case]
    w = W.loguniform_weights(len(u), 7 + case, -1, 1)
    mu = [0.8, 0.3, 0.6, 0.95][case]
    g, h, L, Pm, Gt = _expanded(n, u, v, w, mu)
    H = dense.positive_subgraph(Gt)
    T = dense.msp_from_h(H, h.aggs(), h.sizes)
    eu, ev_, ew = h.msp_edges(mu)
    T2 = dense.edges_to_dense(h.ntilde, eu, ev_, ew)
    np.testing.assert_allclose(T2, T, rtol=0, atol=1e-15 * np.abs(T).max())


@pytest.mark.parametrize("case", range(4))
def test_msp_elimination_equals_pinv(oracle_lib, case):
    """The tree-ordered elimination of L_T~ gives P(mu) pinv(L_T~) P(mu)^T r."""
    from oracle import MSP, dense
    graphs = [W.grid2d(4), W.grid2d(8, 5), W.ring(40), W.erdos_renyi(60, 4, 3)]
    n, u, v = graphs[case]
    w = W.loguniform_weights(len(u), 7 + case, -1, 1)
    mu = [0.8, 0.3, 0.6, 0.95][case]
    g, h, L, Pm, Gt = _expanded(n, u, v, w, mu)
    H = dense.positive_subgraph(Gt)
    T = dense.msp_from_h(H, h.aggs(), h.sizes)
    M = MSP(h, mu)
    r = np.random.default_rng(case).standard_normal(n)
    r -= r.mean()            # M acts on residuals, which are mean-free
    z = M.apply(r)
    z2 = dense.pinv_solve_operator(T, Pm) @ r
    np.testing.assert_allclose(z, z2, rtol=0, atol=1e-11 * np.abs(z2).max())
    assert abs(z.mean()) < 1e-12 * np.abs(z).max()


def test_msp_no_fill_on_grids(oracle_lib):
    """Sec. 3.3: eliminating the aggregates of a grid hierarchy, leftovers
    first, creates (almost) no fill: only where a pair member has no link to
    its parent (ext = 0)."""
    from oracle import MSP, Hierarchy
    n, u, v = W.grid2d(32)
    g = _graph(n, u, v)
    M = MSP(Hierarchy(g), 0.8)
    assert M.fill <= n // 100


# ------------------------------------------------------------------- PCG


@pytest.mark.parametrize("kind", ["none", "msp", "pegp"])
def test_pcg_matches_pseudoinverse(oracle_lib, kind):
    """Tiny graphs: the PCG solution equals pinv(L_G) (b - mean b) within the
    bound kappa(L) * tol."""
    from oracle import MSP, Hierarchy, dense, pcg
    from oracle.pegp import PEGP
    n, u, v = W.erdos_renyi(80, 4, 12)
    w = W.loguniform_weights(len(u), 12, -1.5, 1.5)
    g = _graph(n, u, v, w)
    h = Hierarchy(g)
    prec = {"none": None, "msp": MSP(h, 0.8), "pegp": PEGP(n, u, v, w, h.aggs(), 0.3)}[kind]
    b = np.random.default_rng(2).standard_normal(n)
    res = pcg(g, b, 1e-10, 2000, prec)
    assert res.status == 0
    L = dense.laplacian(n, u, v, w)
    xs = np.linalg.pinv(L) @ (b - b.mean())
    ev = np.linalg.eigvalsh(L)
    kap = ev[-1] / ev[1]
    assert np.linalg.norm(res.x - xs) <= 2 * kap * 1e-10 * np.linalg.norm(xs)
    assert abs(res.x.mean()) < 1e-12 * np.abs(res.x).max()
    assert res.relres_true <= 1e-9


def test_pcg_breakdown_and_noconv(oracle_lib):
    from oracle import ENOCONV, pcg
    n, u, v = W.grid2d(8)
    g = _graph(n, u, v)
    res = pcg(g, np.random.default_rng(0).standard_normal(n), 1e-12, 3, None)
    assert res.status == ENOCONV and res.iterations == 3
    res = pcg(g, np.full(n, 2.0), 1e-8, 10, None)   # b^ = 0
    assert res.status == 0 and res.iterations == 0 and np.all(res.x == 0)


def test_cg_plain_on_path_counts(oracle_lib):
    """Unpreconditioned CG in exact arithmetic ends in at most (number of
    distinct eigenvalues) steps; on the path P_8 that is 7 nonzero ones."""
    from oracle import pcg
    g = _graph(*W.path(8))
    res = pcg(g, np.random.default_rng(0).standard_normal(8), 1e-12, 100, None)
    assert res.status == 0 and res.iterations <= 7
