"""Pins of the MSP closed form and of the rounding-order variants of the
oracle (oracle.msp_closed).

The MSP is M = P(mu) pinv(L_T~) P(mu)^T (Sec. 3.1, Sec. 3.3).  The oracle
evaluates it two ways: by eliminating T~ in the expanded space (lapref.c)
and by the closed form sum_j theta_j P^j D_j^+ (P^j)^T.  Here both are
checked against the definition carried out densely in 40-digit arithmetic
(oracle.dense.msp_apply_highprec), at the mu values the paper uses: the
closed form agrees to rounding at every mu, while the elimination loses
accuracy as mu shrinks (its grounded expanded solution carries offsets of
order mu^(-2(l-1)) that P(mu) cancels).  A dropped level, a wrong theta_j
or sign, or a transposed aggregation map fails these by orders of
magnitude.
"""
import numpy as np
import pytest

import workloads as W


def _setup(n, u, v, w):
    from oracle import Graph, Hierarchy
    g = Graph(n, u, v, w)
    return g, Hierarchy(g)


HIGHPREC = [("ring_64", lambda: W.ring(64), 64 ** -0.5),
            ("grid2d_8", lambda: W.grid2d(8), 64 ** -0.25),
            ("grid3d_4", lambda: W.grid3d(4, 4, 4), 0.8)]


@pytest.mark.slow
@pytest.mark.parametrize("name,make,mu", HIGHPREC, ids=[c[0] for c in HIGHPREC])
def test_closed_form_matches_highprec_definition(oracle_lib, name, make, mu):
    from oracle import MSP, dense
    from oracle.msp_closed import closed_form
    n, u, v = make()
    w = W.loguniform_weights(len(u), 3, -1, 1)
    g, h = _setup(n, u, v, w)
    r = np.random.default_rng(2).standard_normal(n)
    r -= r.mean()
    zm = dense.msp_apply_highprec(n, u, v, w, h.aggs(), mu, r, dps=40)
    nz = np.linalg.norm(zm)
    e_closed = np.linalg.norm(closed_form(h, mu)(r) - zm) / nz
    e_elim = np.linalg.norm(MSP(h, mu).apply(r) - zm) / nz
    print(name, "mu", mu, "closed", e_closed, "elimination", e_elim)
    assert e_closed <= 1e-14
    # the elimination is exact in exact arithmetic; its FP64 rounding grows
    # as mu shrinks but stays far below O(1) on these small hierarchies
    assert e_elim <= 1e-5


@pytest.mark.parametrize("case", range(4))
def test_closed_form_equals_dense_pinv(oracle_lib, case):
    """Same graphs and mu as the elimination's dense pin."""
    from oracle import dense
    from oracle.msp_closed import closed_form
    graphs = [W.grid2d(4), W.grid2d(8, 5), W.ring(40), W.erdos_renyi(60, 4, 3)]
    n, u, v = graphs[case]
    w = W.loguniform_weights(len(u), 7 + case, -1, 1)
    mu = [0.8, 0.3, 0.6, 0.95][case]
    g, h = _setup(n, u, v, w)
    Pm = dense.p_mu(h.aggs(), n, mu)
    Gt = dense.expanded(dense.laplacian(n, u, v, w), Pm)
    T = dense.msp_from_h(dense.positive_subgraph(Gt), h.aggs(), h.sizes)
    r = np.random.default_rng(case).standard_normal(n)
    r -= r.mean()
    z = closed_form(h, mu)(r)
    z2 = dense.pinv_solve_operator(T, Pm) @ r
    np.testing.assert_allclose(z, z2, rtol=0, atol=1e-11 * np.abs(z2).max())
    assert abs(z.mean()) < 1e-12 * np.abs(z).max()


def test_closed_form_single_level(oracle_lib):
    """A star cannot be coarsened: M = pinv(L_G) (theta_1 = 1)."""
    from oracle import dense
    from oracle.msp_closed import closed_form
    n = 13
    u, v = np.zeros(12, dtype=np.int64), np.arange(1, 13)
    w = W.uniform01_weights(12, 4)
    g, h = _setup(n, u, v, w)
    assert h.nlev == 1
    r = np.random.default_rng(1).standard_normal(n)
    r -= r.mean()
    z = closed_form(h, 0.5)(r)
    np.testing.assert_allclose(z, np.linalg.pinv(dense.laplacian(n, u, v, w)) @ r,
                               rtol=0, atol=1e-13)


def test_pcg_exact_sums_solves(oracle_lib):
    """The exact-sum PCG solves L x = b^: against pinv(L) b on a tiny graph,
    with and without a preconditioner."""
    from oracle import dense
    from oracle.msp_closed import closed_form, pcg_exact_sums
    n, u, v = W.grid2d(7, 6)
    w = W.loguniform_weights(len(u), 9, -1, 1)
    g, h = _setup(n, u, v, w)
    b = W.gaussian_rhs(n, 10)
    xs = np.linalg.pinv(dense.laplacian(n, u, v, w)) @ (b - b.mean())
    for M in (lambda r: r.copy(), closed_form(h, 0.8)):
        k, x = pcg_exact_sums(g, M, b, 1e-12, 500)
        assert 0 < k < 500
        assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert pcg_exact_sums(g, closed_form(h, 0.8), np.full(n, 2.0), 1e-8, 10)[0] == 0


def test_pcg_exact_sums_noise_model(oracle_lib):
    """The rounding model of the exact-sum PCG: noise 0 is the unperturbed
    run bit for bit; relative noise 4e-16 on L p and M r moves the solution
    only at rounding level (the converged x agrees with the unperturbed one
    and with pinv(L) b^), different seeds perturb differently, and a large
    noise visibly changes the iteration count's path (the model is live)."""
    from oracle import dense
    from oracle.msp_closed import closed_form, pcg_exact_sums
    n, u, v = W.grid2d(7, 6)
    w = W.loguniform_weights(len(u), 9, -1, 1)
    g, h = _setup(n, u, v, w)
    b = W.gaussian_rhs(n, 10)
    M = closed_form(h, 0.8)
    xs = np.linalg.pinv(dense.laplacian(n, u, v, w)) @ (b - b.mean())
    k0, x0 = pcg_exact_sums(g, M, b, 1e-12, 500)
    k0b, x0b = pcg_exact_sums(g, M, b, 1e-12, 500, noise=0.0, seed=5)
    assert k0 == k0b and np.array_equal(x0, x0b)
    k1, x1 = pcg_exact_sums(g, M, b, 1e-12, 500, noise=4e-16, seed=1)
    k2, x2 = pcg_exact_sums(g, M, b, 1e-12, 500, noise=4e-16, seed=2)
    assert abs(k1 - k0) <= 2 and abs(k2 - k0) <= 2
    for x in (x1, x2):
        assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    assert not np.array_equal(x1, x0) and not np.array_equal(x1, x2)
    k3, _ = pcg_exact_sums(g, M, b, 1e-12, 500, noise=0.3, seed=1)
    assert k3 != k0


def test_band_and_the_cause_of_lower_counts(oracle_lib):
    """The rounding band holds the oracle's own count, and on these two
    workloads the more accurate evaluations (closed form, correctly rounded
    sums) take fewer iterations than the oracle's elimination with
    sequential sums: more accurate FP64 arithmetic converges faster here,
    so a count below the oracle's noise band alone is not a defect."""
    from oracle import MSP
    from oracle.msp_closed import band
    from cases import case
    for name in ("grid2d_64_lowfreq", "ring_1024"):
        n, u, v, w, mu, b = case(name)
        g, h = _setup(n, u, v, w)
        B = band(g, b, 1e-8, 20000, h=h, mu=mu, precond=MSP(h, mu))
        runs = dict(B["runs"])
        print(name, B["lo"], B["hi"], runs["elim"], runs["closed+exact_sums"])
        assert B["lo"] <= B["oracle"] <= B["hi"]
        assert runs["closed+exact_sums"] < runs["elim"]
        noise_hi = max(k for t, k in B["runs"] if t.startswith("elim"))
        assert noise_hi - B["lo"] <= 0.1 * B["oracle"]
