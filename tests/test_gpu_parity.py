"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Kernel level, element by element: L x within the sum's forward error
bound; M r within 1e-12 of the oracle's closed-form MSP, which is pinned to
the definition P(mu) pinv(L_T~) P(mu)^T in 40-digit arithmetic at every mu
(tests/test_oracle_closed.py), and, for mu >= 0.5, within the rounding of
the oracle's elimination of T~.

Whole solves, per case:
  * iteration count inside the case's rounding band widened by 1 on each
    side.  The band (tests/golden/iteration_bands.json, written from the
    oracle alone) is the range of counts over FP64 evaluations that differ
    only in rounding order: the oracle's elimination and the closed form,
    each with sequential sums plus eight runs of the rounding model and
    with correctly rounded sums.  CG counts are not sharp in FP64: on these
    cases the band spans 0 to 20 % of the count;
  * the GPU iterate within 1e-7 (relative 2-norm) of the oracle's iterate
    after the same number of iterations (the oracle rerun with tol = 0 and
    max_iter = the GPU's count), and of the oracle's solution at tol 1e-13;
  * true relative residual <= tol on the GPU and recomputed on the host.
Every assertion message carries the GPU's and the oracle's figures.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from cases import ELIM_MIN_MU, PCG_CASES, case, plain_cg_case
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


def precond_tolerance(mu, nlev):
    """Relative 2-norm bar for M r.  M = sum_j theta_j P^j D_j^+ P^jT with
    theta_j ~ mu^(-2j): level contributions spanning theta_max/theta_min are
    added in different orders by the two sides, so the difference scales with
    eps * mu^(-2(nlev-1)) on top of a base level of cancellation in the
    mean projection."""
    return 1e-10 + 1e3 * np.finfo(float).eps * mu ** (-2.0 * (nlev - 1))


_BANDS = None


def iteration_band(name):
    """(lo, hi): the stored rounding band of a case widened by 1 each side."""
    global _BANDS
    if _BANDS is None:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                            "iteration_bands.json")
        with open(path) as f:
            _BANDS = json.load(f)["cases"]
    b = _BANDS[name]
    return b["lo"] - 1, b["hi"] + 1


def reference_msp(h, mu):
    """The oracle's MSP in closed form (accurate to FP64 rounding at any mu)."""
    from oracle.msp_closed import closed_form
    return closed_form(h, mu)


def _oracle(n, u, v, w):
    from oracle import Graph, Hierarchy
    g = Graph(n, u, v, w)
    return g, Hierarchy(g)


@pytest.mark.parametrize("name", ["grid2d_64_lowfreq", "grid3d_12x10x7_loguniform",
                                  "er_3000_uniform", "chunglu_6000", "star_61", "path_2"])
def test_spmv_parity(oracle_lib, name):
    """q = L_G x element by element (sum order differs: rounding only)."""
    n, u, v, w, mu, _ = case(name)
    say("spmv", name, n)
    g, _ = _oracle(n, u, v, w)
    G = GpuLap(n, u, v, w, mu=mu)
    try:
        x = np.random.default_rng(1).standard_normal(n)
        y = G.apply_laplacian(x)
        y0 = g.apply(x)
        ax = np.abs(x)
        scale = (np.bincount(u, w * (ax[u] + ax[v]), minlength=n)
                 + np.bincount(v, w * (ax[u] + ax[v]), minlength=n))
        np.testing.assert_allclose(y, y0, rtol=0, atol=1e-15 * 16 * scale.max())
        # constants are in the null space exactly
        assert np.all(G.apply_laplacian(np.full(n, 1.25)) == 0.0)
    finally:
        G.close()


PRECOND_CASES = ["grid2d_64_lowfreq", "grid3d_12x10x7_loguniform", "grid3d_16_loguniform",
                 "er_3000_uniform", "chunglu_6000", "ring_1024", "grid2d_64_mu05", "star_61",
                 "ring_1024_quarter", "ring_1024_mu03", "grid3d_12_quarter", "grid2d_32_invsqrt"]


@pytest.mark.parametrize("name", PRECOND_CASES)
def test_precond_parity(oracle_lib, name):
    """z = P(mu) L_T~^+ P(mu)^T r - mean: GPU against the oracle's closed
    form (every mu), and against its elimination of T~ where that is
    accurate (mu >= 0.5)."""
    from oracle import MSP
    n, u, v, w, mu, _ = case(name)
    say("precond", name, n, "mu", mu)
    g, h = _oracle(n, u, v, w)
    G = GpuLap(n, u, v, w, mu=mu)
    try:
        r = np.random.default_rng(2).standard_normal(n)
        r -= r.mean()
        z = G.apply_precond(r)
    finally:
        G.close()
    zc = reference_msp(h, mu)(r)
    err_c = np.linalg.norm(z - zc) / np.linalg.norm(zc)
    msg = f"{name}: mu {mu} levels {h.nlev} rel err vs closed form {err_c:.3e}"
    if mu >= ELIM_MIN_MU:
        z0 = MSP(h, mu).apply(r)
        err_e = np.linalg.norm(z - z0) / np.linalg.norm(z0)
        tol_e = precond_tolerance(mu, h.nlev)
        msg += f", vs elimination {err_e:.3e} (bar {tol_e:.1e})"
    say("  " + msg)
    assert err_c <= 1e-12, msg
    np.testing.assert_allclose(z, zc, rtol=0, atol=1e-12 * np.abs(zc).max(), err_msg=msg)
    if mu >= ELIM_MIN_MU:
        assert err_e <= tol_e, msg


@pytest.mark.parametrize("name", PCG_CASES)
def test_pcg_parity(oracle_lib, name):
    """Whole solve against the oracle (bars in the module docstring)."""
    from oracle import pcg
    n, u, v, w, mu, b = case(name)
    tol = 1e-8
    say("pcg", name, n, "mu", mu)
    g, h = _oracle(n, u, v, w)
    M = reference_msp(h, mu)
    ref = pcg(g, b, tol, 20000, M)
    tight = pcg(g, b, 1e-13, 60000, M)
    lo, hi = iteration_band(name)
    G = GpuLap(n, u, v, w, mu=mu, max_iter=20000)
    try:
        st, x, info = G.solve(b, tol)
    finally:
        G.close()
    k = info["iterations"]
    same = pcg(g, b, 0.0, k, M)
    d_same = np.linalg.norm(x - same.x) / np.linalg.norm(same.x)
    d_tight = np.linalg.norm(x - tight.x) / np.linalg.norm(tight.x)
    bh = b - b.mean()
    host = np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)
    msg = (f"{name}: gpu status {st} iterations {k} (replacements {info['refinements']}), "
           f"oracle {ref.iterations}, band [{lo}, {hi}]; relres gpu {info['relres_true']:.3e} "
           f"host {host:.3e} oracle {ref.relres_true:.3e}; iterate diff at the same count "
           f"{d_same:.2e}, vs tol-1e-13 solution {d_tight:.2e}")
    say("  " + msg)
    assert st == 0 and ref.status == 0, msg
    assert lo <= k <= hi, msg
    assert info["relres_true"] <= tol and host <= tol * 1.01, msg
    assert d_same <= 1e-7 and d_tight <= 1e-7, msg
    assert abs(x.mean()) <= 1e-12 * np.abs(x).max(), msg


def test_plain_cg_parity(oracle_lib):
    """LAP_PREC_NONE: unpreconditioned CG against the oracle's."""
    from oracle import pcg
    import paper_2207_07847_amd as lap
    n, u, v, w, _, b = plain_cg_case()
    say("cg none", n)
    g, _ = _oracle(n, u, v, w)
    ref = pcg(g, b, 1e-8, 5000, None)
    tight = pcg(g, b, 1e-13, 20000, None)
    lo, hi = iteration_band("plain_cg_grid2d_32x20")
    G = GpuLap(n, u, v, w, precond=lap.LAP_PREC_NONE, max_iter=5000)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    k = info["iterations"]
    same = pcg(g, b, 0.0, k, None)
    d_same = np.linalg.norm(x - same.x) / np.linalg.norm(same.x)
    d_tight = np.linalg.norm(x - tight.x) / np.linalg.norm(tight.x)
    msg = (f"plain CG: gpu {k} oracle {ref.iterations} band [{lo}, {hi}] relres "
           f"{info['relres_true']:.3e}; diff same count {d_same:.2e}, tight {d_tight:.2e}")
    say("  " + msg)
    assert st == 0 and info["relres_true"] <= 1e-8, msg
    assert lo <= k <= hi, msg
    assert d_same <= 1e-7 and d_tight <= 1e-7, msg


def test_noconv_status(oracle_lib):
    """max_iter reached: LAP_ENOCONV with x written; after 40 iterations x is
    within 10x the spread of the oracle's rounding model around the oracle's
    own 40th iterate, and so is the recursive residual."""
    from oracle import MSP, pcg
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(64)
    w = W.unit_weights(len(u))
    b = W.lowfreq_rhs(n)
    say("noconv", n)
    g, h = _oracle(n, u, v, w)
    M = MSP(h, 0.8)
    ref = pcg(g, b, 0.0, 40, M)
    ens = [pcg(g, b, 0.0, 40, M, noise=1e-15, seed=s) for s in range(1, 5)]
    spread_x = max(np.linalg.norm(e.x - ref.x) for e in ens) / np.linalg.norm(ref.x)
    spread_r = max(abs(e.relres_recursive - ref.relres_recursive) for e in ens)
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=40)
    try:
        st, x, info = G.solve(b, 1e-12)
        dx = np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)
        dr = abs(info["relres_recursive"] - ref.relres_recursive)
        say("  dx", dx, "spread", spread_x, "dr", dr, "spread", spread_r)
        assert st == lap.LAP_ENOCONV and info["iterations"] == 40
        assert np.all(np.isfinite(x))
        assert dx <= 10 * spread_x + 1e-12
        assert dr <= 10 * spread_r + 1e-12
    finally:
        G.close()


def test_zero_and_constant_rhs():
    """b = constant projects to zero: x = 0 after 0 iterations."""
    n, u, v = W.grid2d(16)
    say("const rhs", n)
    G = GpuLap(n, u, v, W.unit_weights(len(u)))
    try:
        st, x, info = G.solve(np.full(n, 3.0), 1e-8)
        assert st == 0 and info["iterations"] == 0 and np.all(x == 0.0)
    finally:
        G.close()


def test_nonfinite_rhs_rejected():
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(8)
    say("nan rhs", n)
    G = GpuLap(n, u, v, W.unit_weights(len(u)))
    try:
        b = np.ones(n)
        b[3] = np.nan
        st, x, info = G.solve(b, 1e-8)
        assert st == lap.LAP_EINVAL
    finally:
        G.close()


def test_deterministic(oracle_lib):
    """Two solves of the same system are bitwise identical."""
    n, u, v, w, mu, b = case("chunglu_6000")
    say("determinism", n)
    G = GpuLap(n, u, v, w, mu=mu)
    try:
        st1, x1, i1 = G.solve(b, 1e-8)
        st2, x2, i2 = G.solve(b, 1e-8)
        assert st1 == st2 == 0 and i1["iterations"] == i2["iterations"]
        assert np.array_equal(x1, x2)
    finally:
        G.close()
