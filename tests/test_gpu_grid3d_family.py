"""GPU solves of the 3D grid family of the benchmark workload against the
oracle's own full solves.

The workload: 7-point a x a x a grids, weights 10^U(-3,3), Gaussian
right-hand side, MSP mu = 0.8, level = max, tol 1e-8 (Sec. 3.3, Sec. 4).
tests/golden/grid3d_<a>_mu08.json holds what tests/golden/
make_grid3d_golden.py wrote from oracle/ only: the converged solve
(iterations, residuals, x at a seeded sample of 4096 vertices), the
iterate after k iterations at fixed checkpoints, and, for 40^3 and 48^3,
the oracle's rounding band (its unperturbed run and eight runs with
relative noise 4e-16 on L p and M r).

Checked here, for 40^3 and 48^3:
  * the GPU's iteration count lies in the oracle's band widened by one;
  * the GPU's iterate after each checkpoint's k iterations equals the
    oracle's at the sample within 1e-7 relative (the solution bar of the
    parity tests: what differs is the rounding order);
  * the converged GPU solution equals the oracle's converged solution at
    the sample within 1e-7 relative, and its true residual is <= tol.
The 128^3 workload itself is checked the same way in test_gpu_fullsize.py.
"""
import json
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import GpuLap, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(a):
    path = os.path.join(GOLDEN, f"grid3d_{a}_mu08.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written (tests/golden/make_grid3d_golden.py)")
    with open(path) as f:
        d = json.load(f)
    n = d["n"]
    if n <= d["sample_size"]:
        idx = np.arange(n)
    else:
        rng = np.random.default_rng(d["sample_seed"])
        idx = np.sort(rng.choice(n, size=d["sample_size"], replace=False))
    return d, idx


def problem(a):
    n, u, v, w = W.config_graph("grid3d_128", a / 128)
    return n, u, v, w, W.gaussian_rhs(n, W.MASTER_SEED + 3)


def rel(x, ref):
    ref = np.asarray(ref)
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def run_gpu(n, u, v, w, b, tol, max_iter):
    G = GpuLap(n, u, v, w, mu=0.8, max_iter=max_iter)
    try:
        return G.solve(b, tol)
    finally:
        G.close()


@pytest.mark.parametrize("a", [40, 48])
def test_count_in_oracle_band_and_solution(oracle_lib, a):
    d, idx = golden(a)
    n, u, v, w, b = problem(a)
    assert n == d["n"]
    st, x, info = run_gpu(n, u, v, w, b, 1e-8, 60000)
    lo, hi = d["band"]
    dx = rel(x[idx], d["x"])
    msg = (f"grid3d {a}^3: gpu {info['iterations']} iterations ({info['refinements']} "
           f"replacements, relres true {info['relres_true']:.3e}); oracle {d['iterations']}, "
           f"band [{lo}, {hi}] +-1; x vs oracle at the sample {dx:.2e}")
    say(msg)
    assert st == 0 and info["relres_true"] <= 1e-8, msg
    assert lo - 1 <= info["iterations"] <= hi + 1, msg
    assert dx <= 1e-7, msg


@pytest.mark.parametrize("a", [40, 48])
def test_checkpoint_iterates(oracle_lib, a):
    d, idx = golden(a)
    n, u, v, w, b = problem(a)
    for ck in d["checkpoints"]:
        k = ck["k"]
        # tol 1e-30 is never met: exactly k iterations, x written
        st, x, info = run_gpu(n, u, v, w, b, 1e-30, k)
        dx = rel(x[idx], ck["x"])
        msg = (f"grid3d {a}^3 after {k} iterations: gpu {info['iterations']} (status {st}), "
               f"x vs oracle at the sample {dx:.2e}; recursive relres gpu "
               f"{info['relres_recursive']:.3e} oracle {ck['relres_recursive']:.3e}")
        say(msg)
        assert info["iterations"] == k, msg
        assert dx <= 1e-7, msg
