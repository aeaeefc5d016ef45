"""Pins of the oracle's stop rule on the original system (Sec. 4): the
recurrence's residual is only a recursive estimate, so a converged run forms
the true residual b^ - L x and, while it is above tol, restarts from x on it
(residual replacement), at most three times.

Independent checks: the true residual is recomputed here from the dense
Laplacian B^T W B (Sec. 2.1) built in numpy; a restart is compared with the
composition it stands for (PCG from zero on the residual equation L d = t,
then x + d); a hopeless tolerance must end in LR_ENOCONV after exactly three
replacements.
"""
import numpy as np
import pytest

import workloads as W


def _dense_laplacian(n, u, v, w):
    L = np.zeros((n, n))
    np.add.at(L, (u, v), -w)
    np.add.at(L, (v, u), -w)
    L[np.arange(n), np.arange(n)] = -L.sum(axis=1)
    return L


@pytest.fixture(scope="module")
def grid(oracle_lib):
    from oracle import MSP, Graph, Hierarchy
    n, u, v = W.grid2d(32)
    w = W.loguniform_weights(len(u), 5)
    b = W.gaussian_rhs(n, 6)
    g = Graph(n, u, v, w)
    return dict(n=n, b=b, bh=b - b.mean(), g=g, M=MSP(Hierarchy(g), 0.8),
                L=_dense_laplacian(n, u, v, w))


def _true(d, x):
    bh = d["bh"]
    return np.linalg.norm(bh - d["L"] @ x) / np.linalg.norm(bh)


def test_residuals_part_and_a_replacement_recovers(grid):
    """At tol 1e-12 the recurrence meets tol while the true residual is
    about 5x above it; one replacement brings the true residual under tol."""
    from oracle import ENOCONV, OK, pcg
    tol = 1e-12
    r0 = pcg(grid["g"], grid["b"], tol, 20000, grid["M"], restarts=0)
    r3 = pcg(grid["g"], grid["b"], tol, 20000, grid["M"])
    t0, t3 = _true(grid, r0.x), _true(grid, r3.x)
    assert r0.relres_recursive <= tol < t0
    assert r0.status == ENOCONV and r0.restarts == 0
    assert r3.status == OK and 1 <= r3.restarts <= 3
    assert t3 <= tol
    assert abs(r3.relres_true - t3) <= 1e-2 * t3
    assert abs(r0.relres_true - t0) <= 1e-2 * t0
    assert r3.iterations > r0.iterations


def test_restart_is_pcg_on_the_residual_equation(grid):
    """The restarted run equals: the first run's x, plus PCG from zero on
    t = b^ - L x stopped at ||r|| <= tol ||b^||."""
    from oracle import pcg
    tol = 1e-12
    g, M, bh = grid["g"], grid["M"], grid["bh"]
    r0 = pcg(g, grid["b"], tol, 20000, M, restarts=0)
    r3 = pcg(g, grid["b"], tol, 20000, M)
    assert r3.restarts == 1
    t = bh - grid["L"] @ r0.x
    th = t - t.mean()
    d = pcg(g, t, tol * np.linalg.norm(bh) / np.linalg.norm(th), 20000, M, restarts=0)
    xc = r0.x + d.x
    xc -= xc.mean()
    # t here comes from the dense product, in the run from the sparse one:
    # the two differ by rounding, which may move the stop by one iteration
    assert abs(r3.iterations - (r0.iterations + d.iterations)) <= 1
    assert np.linalg.norm(xc - r3.x) <= 1e-9 * np.linalg.norm(r3.x)


def test_unreachable_tolerance_ends_after_three_replacements(grid):
    from oracle import ENOCONV, pcg
    tol = 1e-15
    r = pcg(grid["g"], grid["b"], tol, 20000, grid["M"])
    assert r.status == ENOCONV and r.restarts == 3
    assert _true(grid, r.x) > tol
    assert r.iterations < 20000


def test_no_replacement_when_the_true_residual_meets_tol(grid):
    """At tol 1e-8 the true residual already meets tol: with and without
    replacements the runs are the same, bit for bit."""
    from oracle import OK, pcg
    r0 = pcg(grid["g"], grid["b"], 1e-8, 20000, grid["M"], restarts=0)
    r3 = pcg(grid["g"], grid["b"], 1e-8, 20000, grid["M"])
    assert r0.status == r3.status == OK and r3.restarts == 0
    assert r0.iterations == r3.iterations
    assert np.array_equal(r0.x, r3.x)
    assert _true(grid, r3.x) <= 1e-8
