"""Write the oracle's reference solves of the 3D grid workload family.

The workload: a 7-point a x a x a grid with edge weights 10^U(-3,3) and a
mean-zero Gaussian right-hand side (the seeds of ``workloads``), solved by
MSP-preconditioned CG at mu = 0.8, tol 1e-8, level max (Sec. 3.3, Sec. 4).
For each size this records, from the oracle only:

  * the converged solve: iterations, residual replacements, status, the
    recursive and true relative residuals, ||x||_2 and x at a fixed seeded
    sample of vertices;
  * checkpoints: the iterate after k iterations (tol 0, so no stop and no
    replacement) at the same sample, and its recursive residual, so that a
    GPU run capped at k iterations can be compared at the same count;
  * for the smaller sizes, the iteration band of the oracle's rounding model
    (``oracle.iteration_band``: the unperturbed run and eight runs with
    relative noise 4e-16 on L p and M r).

Run from the repository root:  python tests/golden/make_grid3d_golden.py [a ...]
(default 40 48 128; 128 takes about 3.5 hours of one core for the
converged solve).  Output: tests/golden/grid3d_<a>_mu08.json.

    python tests/golden/make_grid3d_golden.py --band a [seeds]
adds the rounding band (noise runs 1..seeds, default 8, one process each)
to an existing grid3d_<a>_mu08.json (128: about 4 hours a run).

    python tests/golden/make_grid3d_golden.py --exact seeds a [a ...]
adds to grid3d_<a>_mu08_exact.json the same solve with every inner product
and mean summed exactly (math.fsum, oracle.msp_closed.pcg_exact_sums),
with the oracle's elimination of T~ and with the MSP's closed form, each
unperturbed (seed 0) and with the noise model for seeds 1..seeds:
iterations and x at the sample.  On these grids the oracle's sequential
sums over n terms of widely spread magnitude are the largest rounding in
the solve, so these runs show how far the count moves with it.
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

MU, TOL, MAXIT = 0.8, 1e-8, 60000
SAMPLE = 4096
CHECKPOINTS = {40: [100, 1000], 48: [100, 1000], 128: [100, 1000, 5000]}
BAND = {40, 48}
SEEDS = 8
NOISE = 4e-16


def sample_index(n):
    rng = np.random.default_rng(W.MASTER_SEED + 77)
    if n <= SAMPLE:
        return np.arange(n)
    return np.sort(rng.choice(n, size=SAMPLE, replace=False))


def _problem(a):
    from oracle import MSP, Graph, Hierarchy
    n, u, v, w = W.config_graph("grid3d_128", a / 128)
    b = W.gaussian_rhs(n, W.MASTER_SEED + 3)
    g = Graph(n, u, v, w)
    h = Hierarchy(g)
    return n, b, g, h, MSP(h, MU)


def task(job):
    from oracle import pcg
    a, kind, arg = job
    t0 = time.time()
    n, b, g, h, M = _problem(a)
    idx = sample_index(n)
    if kind == "final":
        r = pcg(g, b, TOL, MAXIT, M)
        out = dict(iterations=r.iterations, restarts=r.restarts, status=r.status,
                   relres_recursive=r.relres_recursive, relres_true=r.relres_true,
                   xnorm=float(np.linalg.norm(r.x)), x=[float(t) for t in r.x[idx]],
                   nlev=h.nlev, n=n)
    elif kind == "ck":
        r = pcg(g, b, 0.0, arg, M)
        out = dict(k=arg, relres_recursive=r.relres_recursive, relres_true=r.relres_true,
                   xnorm=float(np.linalg.norm(r.x)), x=[float(t) for t in r.x[idx]])
    else:
        r = pcg(g, b, TOL, MAXIT, M, noise=NOISE, seed=arg)
        out = dict(seed=arg, iterations=r.iterations)
    print(f"grid3d {a}: {kind} {arg} done in {time.time() - t0:.0f} s", flush=True)
    return a, kind, arg, out


def main(sizes):
    jobs = []
    for a in sizes:
        jobs.append((a, "final", 0))
        jobs += [(a, "ck", k) for k in CHECKPOINTS.get(a, [100])]
        if a in BAND:
            jobs += [(a, "band", s) for s in range(1, SEEDS + 1)]
    res = {a: dict(checkpoints=[], band_runs=[]) for a in sizes}
    with mp.get_context("fork").Pool(min(7, len(jobs))) as pool:
        for a, kind, arg, out in pool.imap_unordered(task, jobs):
            if kind == "final":
                res[a].update(out)
            elif kind == "ck":
                res[a]["checkpoints"].append(out)
            else:
                res[a]["band_runs"].append(out["iterations"])
    for a in sizes:
        d = res[a]
        d["checkpoints"].sort(key=lambda c: c["k"])
        d.update(workload=f"grid3d {a}^3, weights 10^U(-3,3) seed MASTER_SEED+2, "
                 "Gaussian rhs seed MASTER_SEED+3",
                 mu=MU, tol=TOL, maxit=MAXIT, sample_seed=W.MASTER_SEED + 77,
                 sample_size=len(sample_index(d["n"])))
        if d["band_runs"]:
            its = [d["iterations"]] + d["band_runs"]
            d["band"] = [min(its), max(its)]
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"grid3d_{a}_mu08.json")
        with open(path, "w") as f:
            json.dump(d, f, indent=0)
        print("wrote", path, flush=True)


def exact_task(job):
    from oracle.msp_closed import closed_form, pcg_exact_sums
    a, kind, seed = job
    t0 = time.time()
    n, b, g, h, M = _problem(a)
    idx = sample_index(n)
    apply = M.apply if kind == "elimination" else closed_form(h, MU)
    it, x = pcg_exact_sums(g, apply, b, TOL, MAXIT, noise=NOISE if seed else 0.0, seed=seed)
    print(f"grid3d {a}: exact sums, {kind}, seed {seed}: {it} iterations in "
          f"{time.time() - t0:.0f} s", flush=True)
    return a, dict(precond=kind, seed=seed, iterations=it, xnorm=float(np.linalg.norm(x)),
                   x=[float(t) for t in x[idx]])


def add_exact(seeds, sizes, procs, first=0):
    jobs = [(a, kind, s) for a in sizes for kind in ("elimination", "closed_form")
            for s in range(first, seeds + 1)]
    res = {a: [] for a in sizes}
    with mp.get_context("fork").Pool(min(procs, len(jobs))) as pool:
        for a, out in pool.imap_unordered(exact_task, jobs):
            res[a].append(out)
    for a in sizes:
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"grid3d_{a}_mu08_exact.json")
        runs = res[a]
        if os.path.exists(path):
            with open(path) as f:
                old = json.load(f)["runs"]
            have = {(r["precond"], r.get("seed", 0)) for r in runs}
            runs += [r for r in old if (r["precond"], r.get("seed", 0)) not in have]
        runs.sort(key=lambda r: (r["precond"], r.get("seed", 0)))
        with open(path, "w") as f:
            json.dump(dict(workload=f"grid3d {a}^3, as grid3d_{a}_mu08.json", mu=MU, tol=TOL,
                           noise=NOISE, sample_seed=W.MASTER_SEED + 77, runs=runs), f, indent=0)
        print("wrote", path, flush=True)


def add_band(a, seeds=SEEDS):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"grid3d_{a}_mu08.json")
    with open(path) as f:
        d = json.load(f)
    jobs = [(a, "band", s) for s in range(1, seeds + 1)]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        d["band_runs"] = sorted(out["iterations"] for _, _, _, out in pool.imap_unordered(task, jobs))
    its = [d["iterations"]] + d["band_runs"]
    d["band"] = [min(its), max(its)]
    with open(path, "w") as f:
        json.dump(d, f, indent=0)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    if sys.argv[1:2] == ["--band"]:
        add_band(int(sys.argv[2]), int(sys.argv[3]) if len(sys.argv) > 3 else SEEDS)
    elif sys.argv[1:2] == ["--exact"]:
        add_exact(int(sys.argv[2]), [int(t) for t in sys.argv[3:]],
                  int(os.environ.get("GOLDEN_PROCS", "8")),
                  int(os.environ.get("GOLDEN_FIRST_SEED", "0")))
    else:
        main([int(t) for t in sys.argv[1:]] or [40, 48, 128])
