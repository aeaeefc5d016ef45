#!/usr/bin/env python3
"""Benchmark: MSP-preconditioned CG solves of a graph Laplacian on one MI355X.

A step is one whole solve (setup excluded) of the weighted 3D 7-point grid
128^3 (2,097,152 vertices, 6,242,304 edges, weights 10^U(-3,3)), MSP with
mu = 0.8 at level = max, FP64, one mean-free Gaussian right-hand side,
relative residual 1e-8; inputs resident in HBM before the timed region.

Prints one JSON line: solves/s, per-solve latency p50/p99, the roofline of
the dominant kernel (sliced-ELL SpMV fused with the p update and p^T q,
timed live with HIP events on the solve stream), and the FP64 oracle timed
on this host's cores over a bounded sample of the same solve.

    python bench.py [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solves/sec + SpMV HBM GB/s at rel-res 1e-8; p50/p99 solve latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


WORKLOADS = {
    "grid2d_64": "grid2d 64x64 5-point, unit weights, PEGP mu=1/64 level=max, 1 Gaussian RHS, "
                 "tol 1e-8",
    "grid3d_128": "grid3d_128^3 7-point, w=10^U(-3,3), MSP mu=0.8 level=max, 1 Gaussian RHS, tol 1e-8",
    "chunglu_4m": "Chung-Lu 4M ids (LCC), mean degree 16, gamma 2.1, w=U(0,1], MSP mu=0.8 "
                  "level=max, 1 Gaussian RHS, tol 1e-8",
    "rmat_20": "R-MAT scale 20 (LCC), (0.57,0.19,0.19,0.05), 16 samples/id, w=U(0,1], MSP mu=0.8 "
               "level=max, tol 1e-8",
}


def workload(name, scale, nrhs=1):
    """Graph, right-hand side(s) and solver settings.  nrhs > 1: columns
    e_i - e_j for seeded random pairs (shape (nrhs, n))."""
    import numpy as np

    import workloads as W
    if name not in WORKLOADS:
        raise SystemExit(f"unknown workload {name}")
    n, u, v, w = W.config_graph(name, scale)
    if nrhs > 1:
        b = W.pair_rhs(n, nrhs, W.MASTER_SEED + 6)
    else:
        b = W.gaussian_rhs(n, W.MASTER_SEED + (1 if name == "grid2d_64" else 3))
    if name == "grid2d_64":
        # the paper's grid workload: PEGP with mu = 1/sqrt(n)
        return dict(n=n, u=u, v=v, w=w, b=b, mu=1.0 / np.sqrt(n), tol=1e-8, precond="pegp")
    return dict(n=n, u=u, v=v, w=w, b=b, mu=0.8, tol=1e-8, precond="msp")


def pmc_traffic(workload_name, scale, kernel, precision):
    """HBM bytes per launch of `kernel` (names joined by '+' are summed)
    from the committed rocprofv3 counter summary of that kernel on this
    workload (profiles/<last kernel>_<workload>_pmc.txt), when it was taken
    at this precision and on the kernel sources as they are now; None
    otherwise."""
    import hashlib
    if scale != 1.0:
        return None
    path = os.path.join(ROOT, "profiles", f"{kernel.split('+')[-1]}_{workload_name}_pmc.txt")
    csrc = os.path.join(ROOT, "paper_2207_07847_amd", "csrc")
    try:
        text = open(path).read()
        h = hashlib.sha256()
        for f in sorted(os.listdir(csrc)):
            if f.endswith((".hip", ".hpp", ".cpp")):
                with open(os.path.join(csrc, f), "rb") as fh:
                    h.update(fh.read())
    except OSError:
        return None
    per, sha, prec = {}, None, None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch "):
            k, v = line[len("traffic_bytes_per_launch "):].split(":")
            per[k.strip()] = float(v)
        elif line.startswith("kernel source sha256[:16]"):
            sha = line.split(":")[-1].strip()
        elif line.startswith("precision:"):
            prec = line.split(":")[1].strip()
    names = kernel.split("+")
    if sha != h.hexdigest()[:16] or prec != precision or any(k not in per for k in names):
        return None
    return sum(per[k] for k in names)


def cpu_baseline_fgmres(wl, budget_s):
    """The oracle's FGMRES on the expanded system (PEGP), whole solves
    repeated for about budget_s seconds."""
    from oracle import Graph, Hierarchy
    from oracle.fgmres import fgmres_expanded
    from oracle.pegp import PEGP
    t0 = time.time()
    h = Hierarchy(Graph(wl["n"], wl["u"], wl["v"], wl["w"]))
    M = PEGP(wl["n"], wl["u"], wl["v"], wl["w"], h.aggs(), wl["mu"])
    setup_s = time.time() - t0
    t0 = time.time()
    k = 0
    while True:
        res = fgmres_expanded(wl["n"], wl["u"], wl["v"], wl["w"], h.aggs(), wl["mu"], wl["b"],
                              M.solve_expanded, tol=wl["tol"])
        k += 1
        if time.time() - t0 >= budget_s or k >= 1000:
            break
    dt = time.time() - t0
    return {
        "value": k / dt,
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{k} whole FGMRES solves ({res.iterations} steps each) in {dt:.1f} s, "
                   f"setup {setup_s:.1f} s untimed"),
    }


def oracle_iterations(name, scale, mu):
    """The oracle's own iteration count for the whole solve, where a
    committed script under tests/golden/ (calling only oracle/) has stored
    it; None elsewhere."""
    if name != "grid3d_128" or scale != 1.0 or mu != 0.8:
        return None
    path = os.path.join(ROOT, "tests", "golden", "grid3d_128_mu08.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    return int(d["iterations"]) if d.get("status") == 0 else None


def cpu_baseline(wl, iters, budget_s, whose):
    """The oracle (single thread) on a bounded number of PCG iterations of
    the same solve, scaled to solves/s by the iteration count the solve
    needs (`whose`: where that count comes from)."""
    from oracle import MSP, Graph, Hierarchy, pcg
    t0 = time.time()
    g = Graph(wl["n"], wl["u"], wl["v"], wl["w"])
    M = MSP(Hierarchy(g), wl["mu"])
    setup_s = time.time() - t0
    t0 = time.time()
    pcg(g, wl["b"], 0.0, 2, M)
    per_it = max((time.time() - t0) / 2.0, 1e-6)
    k = max(3, int(budget_s / per_it))
    t0 = time.time()
    res = pcg(g, wl["b"], 0.0, k, M)
    dt = time.time() - t0
    per_it = dt / res.iterations
    return {
        "value": 1.0 / (per_it * iters),
        "unit": "solves/s",
        "cores": 1,
        "kind": "oracle",
        "sample": (f"{res.iterations} PCG iterations of the same solve in {dt:.1f} s "
                   f"({per_it * 1e3:.1f} ms/iteration, setup {setup_s:.1f} s untimed), "
                   f"scaled by the {iters} iterations the solve takes ({whose})"),
    }, per_it


def _cpu_worker(name, scale, mu, k, barrier, out):
    """One single-threaded oracle process of the all-cores baseline: its
    own hierarchy (untimed), then k PCG iterations once every process is
    ready."""
    from oracle import MSP, Graph, Hierarchy, pcg
    wl = workload(name, scale)
    g = Graph(wl["n"], wl["u"], wl["v"], wl["w"])
    M = MSP(Hierarchy(g), mu)
    barrier.wait()
    t0 = time.time()
    res = pcg(g, wl["b"], 0.0, k, M)
    out.put((time.time() - t0) / res.iterations)


def cpu_baseline_all_cores(name, scale, mu, iters, per_it1, budget_s, whose):
    """The oracle on all host cores the run may use (at most 16, the host
    share of one GPU): one single-threaded oracle process per core, each on
    the same bounded sample, started together; whole-host throughput is the
    sum of the processes' rates.  Spawned interpreters that never touch the
    GPU."""
    import multiprocessing as mp
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    k = max(3, int(budget_s / per_it1))
    ctx = mp.get_context("spawn")
    barrier, out = ctx.Barrier(cores), ctx.Queue()
    procs = [ctx.Process(target=_cpu_worker, args=(name, scale, mu, k, barrier, out))
             for _ in range(cores)]
    for p in procs:
        p.start()
    per = [out.get() for _ in procs]
    for p in procs:
        p.join()
    rate = sum(1.0 / (t * iters) for t in per)
    return {
        "value": rate,
        "unit": "solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{cores} single-threaded oracle processes, {k} PCG iterations of the same "
                   f"solve each, started together ({min(per) * 1e3:.1f}-{max(per) * 1e3:.1f} "
                   f"ms/iteration; setup untimed), each scaled by the {iters} iterations the "
                   f"solve takes ({whose})"),
    }


def device_copy_rate(torch, nbytes=2 * 2**30, reps=20):
    """GB/s (bytes read plus written) of a plain device-to-device copy moving
    nbytes per launch, 2 GiB by default: far beyond the 256 MB Infinity
    Cache, so it measures what HBM gives a read-write stream on this GPU,
    beside the kernels' rates (a copy that fits the cache runs faster)."""
    half = max(1, int(nbytes // 16))
    src = torch.ones(half, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    dt = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 16.0 * half / dt / 1e9


def measure(lap, h, bd, xd, n, tol, steps, warmup, sh, stream, capped, nrhs=1):
    """Warm-up solves, then `steps` timed solves (of nrhs columns each);
    per-solve latency from HIP events on the solve stream."""
    import torch

    def one():
        st, inf = lap.lap_solve(h, bd.data_ptr(), xd.data_ptr(), n, tol, nrhs=nrhs,
                                stream=sh)
        if st == lap.LAP_ENOCONV and capped:
            return inf[0]
        if st != 0:
            raise SystemExit(f"solve failed: {lap.lap_status_str(st)} {inf[:2]}")
        worst = max(inf, key=lambda i: i["relres_true"])
        return dict(worst, iterations=max(i["iterations"] for i in inf))

    for i in range(warmup):
        inf = one()
        log(f"warmup {i}: {inf['iterations']} it, {inf['refinements']} ref, "
            f"relres {inf['relres_true']:.3e}, {inf['seconds']:.3f}s")
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        inf = one()
        e1.record(stream)
        e1.synchronize()
        lat.append(e0.elapsed_time(e1))
        log(f"step {i}: {inf['iterations']} it, {inf['refinements']} ref, "
            f"relres {inf['relres_true']:.3e}, {lat[-1]:.1f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    return dict(elapsed=elapsed, lat=lat, info=inf)


def serve_pool(count, n_min, n_max, seed):
    """Graphs of the serving stream: half 2D/3D grids (unit weights, as the
    paper's grids), half Chung-Lu (mean degree 16, exponent 2.1, U(0,1]
    weights), sizes log-uniform in [n_min, n_max]."""
    import numpy as np

    import workloads as W
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(count):
        target = float(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        if i % 2 == 0:
            if i % 4 == 0:
                a = max(4, int(round(target ** 0.5)))
                n, u, v = W.grid2d(a)
            else:
                a = max(3, int(round(target ** (1 / 3))))
                n, u, v = W.grid3d(a)
            w = W.unit_weights(len(u))
            kind = "grid"
        else:
            n, u, v = W.chung_lu(max(64, int(target)), 16.0, 2.1, seed + i)
            w = W.uniform01_weights(len(u), seed + 1000 + i)
            kind = "chung-lu"
        pool.append(dict(n=n, u=u, v=v, w=w, kind=kind))
    return pool


def serve(args):
    """Serving stream: Poisson arrivals of requests (1-16 Gaussian right-hand
    sides, tol 1e-6 or 1e-8) over a pool of resident hierarchies, through
    the continuous-batching server; latency per request, throughput in
    right-hand sides solved per second."""
    import numpy as np
    import torch

    import paper_2207_07847_amd as lap

    torch.cuda.set_device(0)
    sh = torch.cuda.current_stream().cuda_stream
    t0 = time.time()
    pool = serve_pool(args.serve_graphs, args.serve_nmin, args.serve_nmax, 20220715 + 7)
    log(f"pool: {len(pool)} graphs, n {min(g['n'] for g in pool)}..{max(g['n'] for g in pool)} "
        f"({time.time() - t0:.1f}s)")
    t0 = time.time()
    hs = []
    for g in pool:
        p = lap.lap_default_params(mu=0.8, max_iter=20000, flags=lap.LAP_FLAG_MULTI_RHS)
        hs.append(lap.lap_setup(g["n"], g["u"], g["v"], g["w"], p, sh))
    torch.cuda.synchronize()
    resident = sum(lap.lap_hierarchy_info(h)["device_bytes"] for h in hs)
    log(f"setup {time.time() - t0:.1f}s, resident {resident / 2**30:.1f} GiB")
    rng = np.random.default_rng(20220715 + 8)
    reqs = []
    for k in range(args.serve_requests):
        gi = int(rng.integers(len(pool)))
        m = int(rng.integers(1, 17))
        tol = 1e-8 if rng.random() < 0.5 else 1e-6
        reqs.append(dict(g=gi, tol=tol, m=m))
    arrivals = np.cumsum(rng.exponential(1.0 / args.serve_rate, len(reqs)))

    def rhs(k):
        # request k's right-hand sides from its own seed, drawn when it is
        # submitted (a long stream's b and x would not fit host memory)
        r = reqs[k]
        return np.random.default_rng(20220715 + 9 + k).standard_normal((r["m"],
                                                                        pool[r["g"]]["n"]))

    # plain FP64 single solves of a sample of the requests' columns, on the
    # same hierarchies before they are handed to the server
    sample = reqs[:args.serve_compare]
    cols = 0
    t0 = time.perf_counter()
    for i, r in enumerate(sample):
        g = pool[r["g"]]
        b = rhs(i)
        for j in range(r["m"]):
            bd = torch.tensor(b[j], dtype=torch.float64, device="cuda")
            xd = torch.empty_like(bd)
            st, _ = lap.lap_solve(hs[r["g"]], bd.data_ptr(), xd.data_ptr(), g["n"], r["tol"],
                                  stream=sh)
            cols += 1
    torch.cuda.synchronize()
    single_rate = cols / (time.perf_counter() - t0)
    log(f"plain FP64 single solves: {cols} right-hand sides, {single_rate:.1f} /s")
    srv = lap.lap_server_create(args.serve_budget_gib * 2**30 if args.serve_budget_gib else 0)
    gids = [lap.lap_server_add(srv, h) for h in hs]
    res = {}
    t_start = time.perf_counter()
    t_log = t_start
    k = 0
    while len(res) < len(reqs):
        now = time.perf_counter() - t_start
        if now > args.serve_limit_s:
            log(f"time limit: {len(reqs) - len(res)} requests unfinished")
            break
        if time.perf_counter() - t_log > 5.0:
            t_log = time.perf_counter()
            log(f"  {now:6.1f}s: submitted {k}, completed {len(res)}")
        while k < len(reqs) and arrivals[k] <= now:
            r = reqs[k]
            r["b"] = rhs(k)
            r["x"] = np.empty_like(r["b"])
            st = lap.lap_server_submit(srv, gids[r["g"]], r["b"].ctypes.data, r["x"].ctypes.data,
                                       r["m"], r["tol"], k)
            if st != 0:
                raise SystemExit(f"submit failed: {lap.lap_status_str(st)}")
            k += 1
        for o in lap.lap_server_poll(srv, 512, 1 if k == len(reqs) else 0):
            res[o["tag"]] = o
            # the server is done with the request's buffers
            reqs[o["tag"]].pop("b", None)
            reqs[o["tag"]].pop("x", None)
        if k < len(reqs) and arrivals[k] > now:
            time.sleep(min(0.0005, arrivals[k] - now))
    elapsed = time.perf_counter() - t_start
    lap.lap_server_destroy(srv)
    for h in hs:
        lap.lap_free(h)
    done = sorted(res)
    lat = np.array([res[i]["total_seconds"] for i in done]) * 1e3
    qlat = np.array([res[i]["queue_seconds"] for i in done]) * 1e3
    bad = [i for i in done if res[i]["status"] != 0]
    ncols = sum(reqs[i]["m"] for i in done)
    worst = max(res[i]["relres_max"] / reqs[i]["tol"] for i in done)
    unfinished = len(reqs) - len(done)
    log(f"served {len(done)} requests ({ncols} right-hand sides) in {elapsed:.2f}s, "
        f"p50 {np.percentile(lat, 50):.1f} ms, p99 {np.percentile(lat, 99):.1f} ms, "
        f"failed {len(bad)}, worst relres/tol {worst:.3f}")
    line = {
        "metric": METRIC,
        "value": ncols / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(done),
        "warmup": 0,
        "ms_per_step": elapsed / max(1, len(done)) * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"serving stream: {len(reqs)} requests, Poisson arrivals at "
                        f"{args.serve_rate:g}/s, {len(pool)} graphs (half 2D/3D grids, half "
                        f"Chung-Lu) of {args.serve_nmin}..{args.serve_nmax} vertices (grids: unit "
                        f"weights; Chung-Lu: U(0,1]), 1-16 "
                        f"Gaussian RHS per request, tol 1e-6 or 1e-8, MSP mu=0.8, FP64",
            "right_hand_sides": ncols, "resident_gib": resident / 2**30,
            "failed_requests": len(bad), "unfinished_requests": unfinished,
            "worst_relres_over_tol": worst,
        },
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "queue_p50_ms": float(np.percentile(qlat, 50)),
        "queue_p99_ms": float(np.percentile(qlat, 99)),
        "requests_per_s": len(done) / elapsed,
        "fp64_same_gpu": {"value": single_rate, "unit": "solves/s",
                          "what": f"plain FP64 PCG, one right-hand side per solve, "
                                  f"{cols} columns of the first {len(sample)} requests"},
        "speedup_vs_fp64": (ncols / elapsed) / single_rate,
    }
    print(json.dumps(line), flush=True)


def auto_mu(lap, wl, args, bd, xd, sh):
    """The same workload with mu chosen by lap_select_mu: the choice, its
    cost, and one solve at the chosen mu (after an untimed one)."""
    import torch
    n = wl["n"]
    mus = [float(x) for x in args.auto_mu_candidates.split(",")]
    t0 = time.time()
    st, best, kap = lap.lap_select_mu(n, wl["u"], wl["v"], wl["w"], mus, bd.data_ptr(),
                                      args.select_steps,
                                      lap.lap_default_params(max_iter=args.max_iter), sh)
    torch.cuda.synchronize()
    sel_s = time.time() - t0
    if st != 0:
        return {"status": lap.lap_status_str(st)}
    mu = mus[best]
    h = lap.lap_setup(n, wl["u"], wl["v"], wl["w"],
                      lap.lap_default_params(mu=mu, max_iter=args.max_iter), sh)
    lap.lap_solve(h, bd.data_ptr(), xd.data_ptr(), n, wl["tol"], stream=sh)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, inf = lap.lap_solve(h, bd.data_ptr(), xd.data_ptr(), n, wl["tol"], stream=sh)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    lap.lap_free(h)
    log(f"auto mu: {mu} chosen in {sel_s:.2f}s; {inf[0]['iterations']} iterations, {dt:.3f}s")
    return {"mu": mu, "candidates": mus, "kappa_estimates": [float(k) for k in kap],
            "selection_s": sel_s, "solves_per_s": 1.0 / dt if st == 0 else 0.0,
            "iterations": inf[0]["iterations"], "relres_true": inf[0]["relres_true"],
            "status": lap.lap_status_str(st),
            "what": "the same solve with mu chosen by the smallest estimated kappa of M L "
                    "(lap_select_mu, Lanczos from PCG coefficients); value above keeps mu = 0.8"}


def select_mu(args):
    """mu chosen by the smallest estimated kappa of M L (lap_select_mu), then
    one full solve at every candidate: the choice against the fastest."""
    import numpy as np
    import torch

    import paper_2207_07847_amd as lap
    torch.cuda.set_device(0)
    wl = workload(args.workload, args.scale)
    n = wl["n"]
    sh = torch.cuda.current_stream().cuda_stream
    mus = [float(x) for x in args.mu_candidates.split(",")]
    pc = lap.LAP_PREC_PEGP if wl["precond"] == "pegp" else lap.LAP_PREC_MSP
    params = lap.lap_default_params(max_iter=args.max_iter, precond=pc)
    bd = torch.tensor(np.ascontiguousarray(wl["b"]), dtype=torch.float64, device="cuda")
    xd = torch.empty_like(bd)
    t0 = time.time()
    st, best, kap = lap.lap_select_mu(n, wl["u"], wl["v"], wl["w"], mus, bd.data_ptr(),
                                      args.select_steps, params, sh)
    torch.cuda.synchronize()
    sel_s = time.time() - t0
    if st != 0:
        raise SystemExit(f"lap_select_mu: {lap.lap_status_str(st)}")
    log(f"selection {sel_s:.2f}s: mu {mus[best]}; kappa estimates "
        + ", ".join(f"{m}: {k:.1f}" for m, k in zip(mus, kap)))
    runs = []
    for m in mus:
        h = lap.lap_setup(n, wl["u"], wl["v"], wl["w"],
                          lap.lap_default_params(mu=m, max_iter=args.max_iter, precond=pc), sh)
        lap.lap_solve(h, bd.data_ptr(), xd.data_ptr(), n, wl["tol"], stream=sh)  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, inf = lap.lap_solve(h, bd.data_ptr(), xd.data_ptr(), n, wl["tol"], stream=sh)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        lap.lap_free(h)
        runs.append(dict(mu=m, status=lap.lap_status_str(st), iterations=inf[0]["iterations"],
                         seconds=dt, relres_true=inf[0]["relres_true"]))
        log(f"mu {m}: {inf[0]['iterations']} iterations, {dt:.3f}s, "
            f"{lap.lap_status_str(st)}")
    ok = [r for r in runs if r["status"] == lap.lap_status_str(0)]
    fastest = min(ok, key=lambda r: r["seconds"]) if ok else None
    chosen = runs[best]
    ref = [r for r in runs if abs(r["mu"] - wl["mu"]) < 1e-12]
    out = {
        "metric": "solves/s at the mu chosen by estimated kappa (lap_select_mu)",
        "value": 1.0 / chosen["seconds"] if chosen["status"] == lap.lap_status_str(0) else 0.0,
        "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload].replace(f"mu={wl['mu']:g}", "mu chosen"),
                   "candidates": mus, "estimate_steps": args.select_steps},
        "chosen_mu": mus[best], "selection_s": sel_s,
        "kappa_estimates": [float(k) for k in kap],
        "fastest_mu": fastest["mu"] if fastest else None,
        "per_mu": runs,
        "vs_default_mu": (ref[0]["seconds"] / chosen["seconds"]) if ref and ref[0]["status"] ==
        lap.lap_status_str(0) else None,
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="grid3d_128", choices=sorted(WORKLOADS))
    ap.add_argument("--solver", default="pcg", choices=["pcg", "fgmres"],
                    help="pcg on the original system, or FGMRES on the expanded system "
                         "(the paper's solver; FP64)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "both"],
                    help="both: mixed precision timed, plain FP64 timed beside it")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--mu", type=float, default=0.0,
                    help="mu in (0, 1) instead of the workload's (0: the workload's)")
    ap.add_argument("--nrhs", type=int, default=1,
                    help="right-hand sides per solve (> 1: the 64-column block solve)")
    ap.add_argument("--compare-cols", type=int, default=8,
                    help="with --nrhs > 1: columns timed as single FP64 solves beside it")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-all-cores", action=argparse.BooleanOptionalAction, default=True,
                    help="also time the oracle in one process per host core (at most 16)")
    ap.add_argument("--profile-reps", type=int, default=100)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--serve", action="store_true",
                    help="the serving stream instead of single solves")
    ap.add_argument("--serve-requests", type=int, default=600)
    ap.add_argument("--serve-rate", type=float, default=15.0, help="arrivals per second")
    ap.add_argument("--serve-graphs", type=int, default=32)
    ap.add_argument("--serve-nmin", type=int, default=1000)
    ap.add_argument("--serve-nmax", type=int, default=1000000)
    ap.add_argument("--serve-budget-gib", type=float, default=0.0)
    ap.add_argument("--serve-limit-s", type=float, default=240.0,
                    help="stop waiting after this long; unfinished requests are reported")
    ap.add_argument("--serve-compare", type=int, default=20,
                    help="requests whose columns are also timed as single FP64 solves")
    ap.add_argument("--select-mu", action="store_true",
                    help="choose mu by the smallest estimated kappa (lap_select_mu) and "
                         "solve at every candidate to check the choice")
    ap.add_argument("--mu-candidates", default="0.7,0.8,0.9,0.95,0.98")
    ap.add_argument("--device-setup", action="store_true",
                    help="build the hierarchy's graphs on the device (LAP_FLAG_DEVICE_SETUP)")
    ap.add_argument("--no-auto-mu", action="store_true",
                    help="skip the auto_mu field (the same solve at the mu lap_select_mu "
                         "chooses)")
    ap.add_argument("--auto-mu-candidates", default="0.8,0.9,0.95,0.98,0.99,0.995")
    ap.add_argument("--select-steps", type=int, default=40,
                    help="PCG steps of each candidate's spectrum estimate")
    ap.add_argument("--max-iter", type=int, default=200000,
                    help="cap per solve (profiling runs); a capped solve is not a valid step")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solve is "
              f"not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve(args)
        return
    if args.select_mu:
        select_mu(args)
        return

    import numpy as np
    import torch

    import paper_2207_07847_amd as lap

    torch.cuda.set_device(0)
    t0 = time.time()
    wl = workload(args.workload, args.scale, args.nrhs)
    if args.mu > 0.0:
        wl["mu"] = args.mu
    log(f"workload {args.workload}: n={wl['n']} edges={len(wl['u'])} ({time.time() - t0:.1f}s)")
    n = wl["n"]
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    prec = lap.LAP_FP64 if args.precision == "fp64" else lap.LAP_MIXED_FP32_FP64
    t0 = time.time()
    flags = lap.LAP_FLAG_MULTI_RHS if args.nrhs > 1 else 0
    if args.device_setup:
        flags |= lap.LAP_FLAG_DEVICE_SETUP
    if args.solver == "fgmres":
        flags |= lap.LAP_FLAG_FGMRES
    pc = lap.LAP_PREC_PEGP if wl["precond"] == "pegp" else lap.LAP_PREC_MSP
    h = lap.lap_setup(n, wl["u"], wl["v"], wl["w"],
                      lap.lap_default_params(mu=wl["mu"], max_iter=args.max_iter,
                                             precision=prec, flags=flags, precond=pc), sh)
    setup_s = time.time() - t0
    info = lap.lap_hierarchy_info(h)
    log(f"setup {setup_s:.2f}s levels={info['nlev']} tail={info['tail_level']} "
        f"sizes={info['sizes'][:4]}...{info['sizes'][-2:]}")
    bd = torch.tensor(np.ascontiguousarray(wl["b"]).ravel(), dtype=torch.float64, device="cuda")
    xd = torch.empty_like(bd)
    capped = args.max_iter < 200000
    base = None
    if args.nrhs > 1:
        # single FP64 solves of the first columns, on the same hierarchy
        lap.lap_set_precision(h, lap.LAP_FP64)
        k = min(args.compare_cols, args.nrhs)
        log(f"plain FP64 single solves of {k} columns beside it:")
        t0 = time.perf_counter()
        its = []
        for c in range(k):
            st, inf = lap.lap_solve(h, bd.data_ptr() + 8 * c * n, xd.data_ptr() + 8 * c * n, n,
                                    wl["tol"], nrhs=1, stream=sh)
            torch.cuda.synchronize()
            if st != 0 and not (capped and st == lap.LAP_ENOCONV):
                raise SystemExit(f"single solve failed: {lap.lap_status_str(st)}")
            its.append(inf[0]["iterations"])
        dt = time.perf_counter() - t0
        log(f"  {k} single FP64 solves: {dt:.3f}s, iterations {min(its)}..{max(its)}")
        base = dict(elapsed=dt / k * args.nrhs, lat=[dt / k * 1e3], info=dict(
            iterations=max(its), relres_true=inf[0]["relres_true"]), cols=k)
        if args.precision != "fp64":
            lap.lap_set_precision(h, lap.LAP_MIXED_FP32_FP64)
    elif args.precision == "both":
        lap.lap_set_precision(h, lap.LAP_FP64)
        log("plain FP64 beside it:")
        base = measure(lap, h, bd, xd, n, wl["tol"], args.steps, args.warmup, sh, stream, capped)
        lap.lap_set_precision(h, lap.LAP_MIXED_FP32_FP64)
    res = measure(lap, h, bd, xd, n, wl["tol"], args.steps, args.warmup, sh, stream, capped,
                  args.nrhs)
    inf = res["info"]

    if args.calib_copy_mb:
        src = torch.ones(args.calib_copy_mb * 131072, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # kernels timed inside iterations on the solve stream (the engine the
    # timed solves used: FP32 for mixed precision)
    kern = {}
    parts = [(lap.LAP_KERNEL_SPMV, "spmv_p"), (lap.LAP_KERNEL_UPDATE, "update_up0"),
             (lap.LAP_KERNEL_DOWN0, "down0"), (lap.LAP_KERNEL_PRECOND, "update_precond"),
             (lap.LAP_KERNEL_ITER, "iteration")]
    pegp_op = wl["precond"] == "pegp" and info["pegp_operator_n"] > 0
    if wl["precond"] == "pegp":
        # the PEGP application has no MSP level parts to time; with the
        # explicit operator, its matrix-vector product is the dominant kernel
        parts = [parts[0]] + ([(lap.LAP_KERNEL_PEGP_OP, "pegp_op")] if pegp_op else []) + \
            [parts[-1]]
    for kid, name in parts:
        ms, by = lap.lap_profile_kernel(h, kid, args.profile_reps, sh)
        kern[name] = {"avg_us": ms * 1e3, "alg_bytes": by, "gbs": by / (ms * 1e-3) / 1e9}
        log(f"kernel {name}: {ms * 1e3:.1f} us, {by / 1e6:.1f} MB, {kern[name]['gbs']:.0f} GB/s")
    if args.nrhs > 1:
        for kid, name in [(lap.LAP_KERNEL_BLOCK_SPMM, "block_spmm"),
                          (lap.LAP_KERNEL_BLOCK_ITER, "block_iteration")]:
            ms, by = lap.lap_profile_kernel(h, kid, max(3, args.profile_reps // 10), sh)
            kern[name] = {"avg_us": ms * 1e3, "alg_bytes": by,
                          "gbs": by / (ms * 1e-3) / 1e9 if by else None}
            log(f"kernel {name}: {ms * 1e3:.1f} us, {by / 1e6:.1f} MB")
    lap.lap_free(h)

    spmv = kern["spmv_p"] if args.nrhs == 1 else kern["block_spmm"]
    dom, dom_name = (kern["pegp_op"], "k_pegp_op") if pegp_op else \
        (spmv, "k_mm_spmm" if args.nrhs > 1 else
         "k_spmv_p" if info["spmv_fused"] else "k_pupd+k_spmv_q")
    steps = args.steps * args.nrhs       # right-hand sides solved
    dtype = "f64" if args.precision == "fp64" else "f32+f64"
    line = {
        "metric": METRIC,
        "value": steps / res["elapsed"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": res["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": (WORKLOADS[args.workload].replace("^3", f"^3 (scale {args.scale})")
                         if args.scale != 1.0 else WORKLOADS[args.workload]).replace(
                "mu=0.8", f"mu={wl['mu']:g}").replace("mu=1/64", f"mu={wl['mu']:g}"
                                                     if args.mu > 0.0 else "mu=1/64"),
            "precision": "FP64" if args.precision == "fp64" else
                         "FP32 SpMV/preconditioner inside FP64 iterative refinement",
            "solver": "FGMRES on the expanded system" if args.solver == "fgmres" else
                      "PCG on the original system",
            "n": n, "edges": int(len(wl["u"])), "levels": info["nlev"], "nrhs": args.nrhs,
            "iterations": inf["iterations"], "refinements": inf["refinements"],
            "relres_true": inf["relres_true"],
        },
        "p50_ms": float(np.percentile(res["lat"], 50)),
        "p99_ms": float(np.percentile(res["lat"], 99)),
        "spmv_gbs": spmv["gbs"],
        "iteration_us": kern["iteration"]["avg_us"],
        "kernels": kern,
        "setup_s": setup_s,
        "roofline": {
            "bound": "hbm",
            "kernel": dom_name,
            "achieved": dom["gbs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": dom["gbs"] / HBM_PEAK_GBS,
            "traffic": pmc_traffic(args.workload, args.scale, dom_name, args.precision),
        },
    }
    copy = device_copy_rate(torch) if not capped else float("nan")
    line["device_copy"] = {
        "gbs": copy, "bytes": 2 * 2**30,
        "kernel_over_copy": dom["gbs"] / copy,
        "what": "torch device-to-device copy of 1 GiB into 1 GiB (2 GiB read plus written "
                "per launch, beyond the 256 MB Infinity Cache), back to back: the rate HBM "
                "gives a plain read-write stream on this GPU, beside the dominant kernel's"}
    if capped:
        del line["device_copy"]     # capped runs (counter passes) time no copy
    else:
        log(f"device copy (2 GiB moved): {copy:.0f} GB/s; kernel / copy {dom['gbs'] / copy:.3f}")
    if pegp_op:
        line["roofline"]["note"] = (
            "the operator (opn^2 FP64 entries, 134 MB here) is smaller than the 256 MB "
            "last-level cache, so part of each read may be served there: the L2 fetches "
            "it once per launch either way")
    elif wl["precond"] == "pegp":
        line["roofline"]["note"] = (
            "the SpMV is a small part of a PEGP iteration applied by the factor: its "
            "time is in the preconditioner's level and dense-tail solves, chains of "
            "dependent steps bound by latency")
    if args.nrhs > 1:
        k = 1 if args.precision != "fp64" else 0
        line["autotuned"] = {"spmm_entries_per_item": info["mm_chunk"][k],
                             "spmm_workgroups": info["mm_grid"][k],
                             "level_children_per_item": info["mm_seg"][k],
                             "tune_s": info["mm_tune_seconds"]}
    if base is not None:
        bi = base["info"]
        line["fp64_same_gpu"] = {
            "value": steps / base["elapsed"] if args.nrhs == 1 else args.nrhs / base["elapsed"],
            "unit": "solves/s",
            "ms_per_step": base["elapsed"] / (args.steps if args.nrhs == 1 else 1) * 1e3,
            "iterations": bi["iterations"], "relres_true": bi["relres_true"],
            "p50_ms": float(np.percentile(base["lat"], 50)),
            "what": "plain FP64 PCG, one right-hand side per solve" +
                    (f" (timed on {base['cols']} of the columns)" if args.nrhs > 1 else ""),
        }
        line["speedup_vs_fp64"] = (base["elapsed"] / res["elapsed"]) if args.nrhs == 1 else \
            (base["elapsed"] / (res["elapsed"] / args.steps))
    if not capped:
        # the same set-up with the graphs built on the device (bit-identical
        # hierarchy), timed beside the host build above
        t0 = time.time()
        h2 = lap.lap_setup(n, wl["u"], wl["v"], wl["w"],
                           lap.lap_default_params(mu=wl["mu"], max_iter=args.max_iter,
                                                  precision=prec,
                                                  flags=flags ^ lap.LAP_FLAG_DEVICE_SETUP,
                                                  precond=pc), sh)
        torch.cuda.synchronize()
        other_s = time.time() - t0
        lap.lap_free(h2)
        # and with the matching on the device as well (the locally dominant
        # matching: a different hierarchy, not the one timed above)
        t0 = time.time()
        h3 = lap.lap_setup(n, wl["u"], wl["v"], wl["w"],
                           lap.lap_default_params(mu=wl["mu"], max_iter=args.max_iter,
                                                  precision=prec,
                                                  flags=flags | lap.LAP_FLAG_DEVICE_SETUP |
                                                  lap.LAP_FLAG_PARALLEL_MATCHING,
                                                  precond=pc), sh)
        torch.cuda.synchronize()
        par_s = time.time() - t0
        lap.lap_free(h3)
        line["setup_graphs"] = {
            "host_s": other_s if args.device_setup else setup_s,
            "device_s": setup_s if args.device_setup else other_s,
            "device_parallel_matching_s": par_s,
            "what": "lap_setup with the adjacency and coarse graphs built on the host, and on "
                    "the device (LAP_FLAG_DEVICE_SETUP), the rest of the set-up on the host in "
                    "both; and with the locally dominant matching on the device too "
                    "(LAP_FLAG_PARALLEL_MATCHING, a different hierarchy)"}
        log(f"setup: host graphs {line['setup_graphs']['host_s']:.2f}s, device graphs "
            f"{line['setup_graphs']['device_s']:.2f}s, device graphs and matching {par_s:.2f}s")
    if (not args.no_auto_mu and wl["precond"] == "msp" and args.nrhs == 1 and
            args.precision == "fp64" and args.solver == "pcg" and not capped):
        line["auto_mu"] = auto_mu(lap, wl, args, bd, xd, sh)
    if not args.no_cpu:
        if args.workload == "grid3d_128" and args.scale == 1.0 and args.solver == "pcg":
            log("cpu baseline (oracle) ...")
            it = oracle_iterations(args.workload, args.scale, wl["mu"])
            whose = "the oracle's own count, tests/golden/grid3d_128_mu08.json" if it else \
                "the GPU's count; the oracle's is not stored for this setting"
            it = it or inf["iterations"]
            line["cpu_baseline"], per_it = cpu_baseline(wl, it, args.cpu_seconds, whose)
            if args.cpu_all_cores:
                log("cpu baseline (oracle) on all host cores ...")
                line["cpu_baseline_all_cores"] = cpu_baseline_all_cores(
                    args.workload, args.scale, wl["mu"], it, per_it, args.cpu_seconds, whose)
        elif args.workload == "grid2d_64" and args.solver == "fgmres":
            log("cpu baseline (oracle FGMRES) ...")
            line["cpu_baseline"] = cpu_baseline_fgmres(wl, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
