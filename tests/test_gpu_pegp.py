"""GPU checks of the PEGP preconditioner (Sec. 3.1-3.2): z = P(mu) L_H~^+
P(mu)^T r through the grounded, scaled system S = D L_H~ D factored on the
host.  Two device paths, each tested: the explicit operator M (formed at
set-up through the factor, applied as one matrix-vector product; the
default up to 8192 fine nodes), and the factor itself (the sparse levels by
one workgroup, the dense tail, the last-eliminated rows, by blocked
substitution over the whole device).

The applied preconditioner is compared with the oracle's (scipy sparse
products and a sparse LU of the same grounded, scaled matrix) in the
relative 2-norm, within the backward-stable-solve bound c * nt * eps *
kappa(S) (kappa from a dense spectrum where the system is small enough).
Whole solves reproduce the PCG step counts the paper prints in Table 3
(grids, level = max with mu = 1/sqrt(n), level = 2 with mu = n^(-1/4)).
"""
import contextlib
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu


MODES = ["operator", "factor"]


@contextlib.contextmanager
def _mode(mode):
    """The device path of PEGP hierarchies set up inside the block."""
    old = os.environ.get("LAPGPU_PEGP_OPERATOR")
    os.environ["LAPGPU_PEGP_OPERATOR"] = "1" if mode == "operator" else "0"
    try:
        yield
    finally:
        if old is None:
            del os.environ["LAPGPU_PEGP_OPERATOR"]
        else:
            os.environ["LAPGPU_PEGP_OPERATOR"] = old


def _oracle_pegp(n, u, v, w, mu, max_levels=0):
    from oracle import Graph, Hierarchy
    from oracle.pegp import PEGP
    g = Graph(n, u, v, w)
    h = Hierarchy(g, max_levels=max_levels) if max_levels else Hierarchy(g)
    return g, h, PEGP(n, u, v, w, h.aggs(), mu)


CASES = {
    "grid2d_16_mu1/16": lambda: (*W.grid2d(16), None, 1 / 16.0),
    "grid2d_32_mu1/32": lambda: (*W.grid2d(32), None, 1 / 32.0),
    "grid2d_64_mu1/64": lambda: (*W.grid2d(64), None, 1 / 64.0),
    "grid2d_24_loguniform_mu0.5": lambda: (*W.grid2d(24), "log", 0.5),
    "er_1500_mu0.8": lambda: (*W.erdos_renyi(1500, 6, 3), "u01", 0.8),
}


def _weights(kind, m, seed):
    if kind is None:
        return W.unit_weights(m)
    if kind == "log":
        return W.loguniform_weights(m, seed)
    return W.uniform01_weights(m, seed)


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", list(CASES))
def test_pegp_apply_parity(oracle_lib, name, mode):
    """The bar is the rounding spread of the direct solve itself: the oracle
    solved with two fill orderings (the same grounded system, different
    elimination orders) differs by `spread`; the GPU's elimination order is a
    third one, and its result must lie within 100 x that spread (and 1e-14)."""
    import paper_2207_07847_amd as lap
    from oracle.pegp import PEGP
    n, u, v, kind, mu = CASES[name]()
    w = _weights(kind, len(u), 11)
    g, h, M = _oracle_pegp(n, u, v, w, mu)
    M2 = PEGP(n, u, v, w, h.aggs(), mu, permc_spec="MMD_AT_PLUS_A")
    r = np.random.default_rng(12).standard_normal(n)
    r -= r.mean()
    z0 = M.apply(r)
    spread = np.linalg.norm(M2.apply(r) - z0) / np.linalg.norm(z0)
    with _mode(mode):
        G = GpuLap(n, u, v, w, mu=mu, precond=lap.LAP_PREC_PEGP)
    try:
        z = G.apply_precond(r)
    finally:
        G.close()
    err = np.linalg.norm(z - z0) / np.linalg.norm(z0)
    msg = f"{name} ({mode}): nt {M.nt} rel err {err:.3e}, oracle ordering spread {spread:.3e}"
    say(msg)
    assert err <= max(100 * spread, 1e-14), msg


# Shapes of the dense tail on small grids (grid side, level setting):
# the whole factor in the tail with no sparse level, no tail at all, one
# superblock that is mostly padding, and one that is full but for two rows.
TAIL_SHAPES = {
    "grid2d_6_level_max_all_tail": (6, 0),
    "grid2d_6_level2_no_tail": (6, 2),
    "grid2d_8_level2_one_superblock": (8, 2),
    "grid2d_12_level_max_one_full_superblock": (12, 0),
}


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("name", list(TAIL_SHAPES))
def test_pegp_apply_tail_shapes(oracle_lib, name, mode):
    """The same bar as above, on tails that the larger cases do not have."""
    import paper_2207_07847_amd as lap
    from oracle.pegp import PEGP
    a, ml = TAIL_SHAPES[name]
    n, u, v = W.grid2d(a)
    w = W.unit_weights(len(u))
    mu = n ** -0.25 if ml else 1.0 / a
    g, h, M = _oracle_pegp(n, u, v, w, mu, ml)
    M2 = PEGP(n, u, v, w, h.aggs(), mu, permc_spec="MMD_AT_PLUS_A")
    r = np.random.default_rng(22).standard_normal(n)
    r -= r.mean()
    z0 = M.apply(r)
    spread = np.linalg.norm(M2.apply(r) - z0) / np.linalg.norm(z0)
    with _mode(mode):
        G = GpuLap(n, u, v, w, mu=mu, precond=lap.LAP_PREC_PEGP, max_levels=ml)
    try:
        z = G.apply_precond(r)
    finally:
        G.close()
    err = np.linalg.norm(z - z0) / np.linalg.norm(z0)
    msg = f"{name} ({mode}): nt {M.nt} rel err {err:.3e}, oracle ordering spread {spread:.3e}"
    say(msg)
    assert err <= max(100 * spread, 1e-14), msg


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("a", [16, 32, 64])
def test_pegp_table3_steps(oracle_lib, a, mode):
    """Table 3: PEGP, tol 1e-8, b = [1,...,1,1-n]: the paper's step counts."""
    import paper_2207_07847_amd as lap
    from oracle import Graph
    pins = {(256, 0): 7, (1024, 0): 6, (4096, 0): 5, (256, 2): 12, (1024, 2): 10, (4096, 2): 9}
    n, u, v = W.grid2d(a)
    w = np.ones(len(u))
    b = W.lowfreq_rhs(n)
    g = Graph(n, u, v, w)
    for ml, mu in [(0, 1 / np.sqrt(n)), (2, n ** -0.25)]:
        with _mode(mode):
            G = GpuLap(n, u, v, w, mu=mu, max_levels=ml, precond=lap.LAP_PREC_PEGP,
                       max_iter=1000)
        try:
            st, x, info = G.solve(b, 1e-8)
        finally:
            G.close()
        bh = b - b.mean()
        host = np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)
        say("table3", n, "levels", ml or "max", "steps", info["iterations"], "pin", pins[(n, ml)],
            "relres", host)
        assert st == 0 and info["iterations"] == pins[(n, ml)]
        assert host <= 1.01e-8


@pytest.mark.parametrize("mode", MODES)
def test_pegp_c1_solve(oracle_lib, mode):
    """64x64 grid, unit weights, mu = 1/64, Gaussian right-hand side: the
    oracle's PEGP-PCG iteration count, FP64 residual <= tol."""
    import paper_2207_07847_amd as lap
    from oracle import pcg
    n, u, v = W.grid2d(64)
    w = W.unit_weights(len(u))
    b = W.gaussian_rhs(n, W.MASTER_SEED + 1)
    g, h, M = _oracle_pegp(n, u, v, w, 1 / 64.0)
    ref = pcg(g, b, 1e-8, 1000, M)
    with _mode(mode):
        G = GpuLap(n, u, v, w, mu=1 / 64.0, precond=lap.LAP_PREC_PEGP, max_iter=1000)
    try:
        st, x, info = G.solve(b, 1e-8)
    finally:
        G.close()
    bh = b - b.mean()
    host = np.linalg.norm(bh - g.apply(x)) / np.linalg.norm(bh)
    diff = np.linalg.norm(x - pcg(g, b, 0.0, info["iterations"], M).x) / np.linalg.norm(x)
    msg = (f"C1 pegp ({mode}): gpu {info} oracle it {ref.iterations} host relres {host:.3e} "
           f"iterate diff {diff:.2e}")
    say(msg)
    assert st == 0 and info["iterations"] == ref.iterations, msg
    assert host <= 1.01e-8 and diff <= 1e-7, msg


def test_pegp_operator_profile_part(oracle_lib):
    """The operator's matrix-vector product is timed on its own
    (LAP_KERNEL_PEGP_OP), with 8 n^2 + 20 n algorithmic bytes; a hierarchy
    that runs through the factor has no such part."""
    import paper_2207_07847_amd as lap
    n, u, v = W.grid2d(32)
    w = W.unit_weights(len(u))
    for mode in MODES:
        with _mode(mode):
            G = GpuLap(n, u, v, w, mu=1 / 32.0, precond=lap.LAP_PREC_PEGP)
        try:
            opn = G.info["pegp_operator_n"]
            if mode == "operator":
                assert opn == n
                ms, by = lap.lap_profile_kernel(G.h, lap.LAP_KERNEL_PEGP_OP, 10, G.stream())
                say(f"pegp operator n {n}: {ms * 1e3:.1f} us, {by / 1e6:.2f} MB")
                assert by == 8.0 * n * n + 20.0 * n and 0.0 < ms < 10.0
            else:
                assert opn == 0
                with pytest.raises(lap.LapError):
                    lap.lap_profile_kernel(G.h, lap.LAP_KERNEL_PEGP_OP, 10, G.stream())
        finally:
            G.close()
