"""Benchmark: spanning-tree samples/s of the full estimator path on one MI355X.

One step = one persistent launch of the estimator over a batch of tree
samples: Wilson sampling, subtree volumes and numbering, f(tau) per tree and
the exact reduction (the whole hot path).  The default workload is the
dense power-law graph: Chung-Lu, 3,000,000 vertices, expected degrees with
exponent 2.0, mean 76, cap 30,000, largest component, int64 offsets on
input; 4,096 samples per launch, so four launches make one 16,384-sample
estimate.  Inputs (graph and workspace) are resident in HBM before the timed
region; sample ids advance from step to step.

Prints ONE JSON line.  Besides the contract fields it carries `roofline`
(algorithmic HBM bytes of the persistent kernel per launch over its average
duration, against the 8 TB/s HBM peak) and `cpu_baseline` (the CPU oracle on
the host cores, on a bounded sample of the same workload).  The accuracy leg
(K-hat against exact K on the 32x32 grid), the plain one-sample-at-a-time
form and a short serving leg follow the timed region while the run stays
within its wall-clock budget (--budget).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "spanning-tree samples/s and K at ε=0.01 vs exact; served query p50/p99 ms"
HBM_PEAK_GBS = 8000.0
SECTOR = 64
LIB_SRC = os.path.join(ROOT, "paper_2511_16356_amd", "csrc")

# HBM bytes per launch of the sampling kernel, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE runs of this script (each in a run of its own), scaled by what the
# counter reads for a plain 1 GiB copy (FETCH_SIZE x 1.99992, WRITE_SIZE x 1;
# profiles/hbm_traffic_*.md).  Keyed by the SHA-256 of the library sources the
# counters were taken on (library_sha): other sources, or another workload,
# sample count or seed, report traffic = null.
MEASURED_TRAFFIC = {
    "eb3d94573d93d4b15fc1672f3ee817e16712f794e649760a8f2ab47f425636fa": [
        {"workload": "dense", "samples": 4096, "seed": 0,
         "fetch_bytes": 8.8753e12, "write_bytes": 4.2740e12, "bytes": 1.3149e13},
        {"workload": "social", "samples": 8192, "seed": 0,
         "fetch_bytes": 6.1406e12, "write_bytes": 2.8420e12, "bytes": 8.9825e12},
        {"workload": "road", "samples": 4096, "seed": 0, "direct": True,
         "fetch_bytes": 3.5018e13, "write_bytes": 6.8240e13, "bytes": 1.0326e14},
    ],
    # earlier sources, kept for the record (lean looks as a run-time switch)
    "3bc1c440df2c3d151af35ad1d81f4e825ce71d1c2097cee7f2da191f9d7aac12": [
        {"workload": "dense", "samples": 4096, "seed": 0,
         "fetch_bytes": 8.8783e12, "write_bytes": 4.2736e12, "bytes": 1.3152e13},
        {"workload": "social", "samples": 8192, "seed": 0,
         "fetch_bytes": 6.1436e12, "write_bytes": 2.8417e12, "bytes": 8.9853e12},
    ],
    "4564d6b8d6afc957cbc43894fc61214308b3a71b63e1d45e1c7d7078f7caff51": [
        {"workload": "dense", "samples": 4096, "seed": 0,
         "fetch_bytes": 1.1195e13, "write_bytes": 4.1896e12, "bytes": 1.5385e13},
    ],
    "b049347fd167b424567c63761557e6006c70dd9cfd6ef897f165fff66afc39ff": [
        {"workload": "dense", "samples": 4096, "seed": 0,
         "fetch_bytes": 1.1188e13, "write_bytes": 4.1845e12, "bytes": 1.5372e13},
        {"workload": "social", "samples": 8192, "seed": 0,
         "fetch_bytes": 7.3610e12, "write_bytes": 2.7790e12, "bytes": 1.0140e13},
        {"workload": "road", "samples": 4096, "seed": 0, "direct": True,
         "fetch_bytes": 3.5062e13, "write_bytes": 6.8268e13, "bytes": 1.0333e14},
    ],
}


# Measured ceilings of the device (bench.py --calibrate-random 128, libkc_probe.so;
# profiles/memory_ceilings_mi355x.md): the best streaming read, and independent
# random 8-byte reads by each lane to a line of its own, over a 128 GiB buffer,
# swept over reads in flight per lane and workgroups per CU.
MEASURED_CEILINGS = {"stream_read_GBps": 6362.0, "random_64B_read_GBps": 3179.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


MALL_BYTES = 256 << 20  # the last-level cache (Infinity Cache) of one MI355X


def algorithmic_bytes(draws: int, n: int, two_m: int, depth0: int, samples: int) -> int:
    """Random 64-byte sectors the method itself must touch per launch: per
    Wilson draw the drawn vertex's per-sample state, plus its CSR offset and
    neighbour when the CSR does not fit the last-level cache (they are L2/MALL
    hits when it does); per tree one sector per vertex to join it to the tree,
    and n * min(depth0, ceil(log2 n)) for the path-mapping sums."""
    csr_bytes = 8 * (n + 1) + 4 * two_m
    per_draw = 3 if csr_bytes > MALL_BYTES else 1
    per_tree_trav = n * min(depth0, math.ceil(math.log2(max(2, n))))
    return SECTOR * (per_draw * draws + samples * (n + per_tree_trav))


def host_cpu():
    """(logical CPUs, model name) of the host this runs on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count() or 1, model


def cpu_baseline(g, seed: int, first: int, threads: int, per_thread: int, what: str = "the same workload",
                 min_s: float = 10.0, target_s: float = 15.0):
    """The CPU oracle as it stands (sequential Wilson per sample, the per-edge
    f of Theorem 3.4, exact sums) on `threads` host threads, samples split
    across them, over a bounded sample of the workload: ids first ..
    first + threads * per_thread - 1, then, if those took less than min_s
    seconds, the next ids (whole rounds of `threads`, at most 64 times as
    many), sized by the rate just measured to bring the timed work to about
    target_s seconds.  Graph preparation is outside the timed region."""
    import oracle
    P = oracle.prepare_graph(g)
    count = threads * per_thread
    t0 = time.perf_counter()
    oracle.estimate_f(P, seed=seed, s0=first, count=count, threads=threads)
    dt = time.perf_counter() - t0
    if dt < min_s:
        rounds = min(64 * per_thread, max(1, math.ceil((target_s - dt) / max(dt, 1e-6) * per_thread)))
        more = threads * rounds
        t1 = time.perf_counter()
        oracle.estimate_f(P, seed=seed, s0=first + count, count=more, threads=threads)
        dt += time.perf_counter() - t1
        count += more
    nproc, model = host_cpu()
    return {"value": count / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "nproc": nproc, "cpu_model": model,
            "sample": "samples %d..%d of %s (%d on %d threads), %.1f s; the rate over this "
                      "bounded sample stands for the workload's" %
                      (first, first + count - 1, what, count, threads, dt)}


def serving_leg(seed: int, graphs: int, lo: int, hi: int, samples: int, rate: float, duration: float,
                maintenance: int = 0, one_at_a_time: bool = False, n_req: int = 0, saturate: bool = False):
    """Served query and update latency on resident graphs (continuous batching,
    paper_2511_16356_amd.serve): Poisson arrivals, 80% Kemeny queries and 20%
    update batches, half deletions (sizes log-uniform in [1, 1000], batches
    that keep the graph connected) and half insertions (sizes log-uniform in
    [1, 10]); edges drawn with probability proportional to d(u) d(v).  The
    same seed gives the same graphs and requests for either maintenance."""
    import numpy as np
    import torch
    import graphgen
    from paper_2511_16356_amd.serve import Server, Request, latency_stats
    t_gen = time.perf_counter()
    gs = graphgen.serving_graphs(graphs, lo, hi, seed)
    rng = np.random.default_rng(seed + 1)
    n_req = n_req or int(rate * duration)
    # unit-rate gaps scaled by the rate: the same requests at every rate
    times = np.cumsum(rng.exponential(1.0, size=n_req)) / rate
    if saturate:
        times = np.zeros(n_req)  # everything arrives at once: the makespan gives the capacity
    upd = rng.random(n_req) < 0.2
    gids = rng.integers(0, graphs, size=n_req)
    cur = list(gs)
    plan = []
    for t, is_upd, gid in zip(times, upd, gids):
        gid = int(gid)
        if is_upd and rng.random() < 0.5:
            size = int(round(math.exp(rng.uniform(0.0, math.log(1000.0)))))
            batch = graphgen.deletion_batch(cur[gid], size, rng)
            cur[gid] = graphgen.remove_edges(cur[gid], batch)
            plan.append((float(t), gid, "update", batch, False))
        elif is_upd:
            size = int(round(math.exp(rng.uniform(0.0, math.log(10.0)))))
            batch = graphgen.insertion_batch(cur[gid], size, rng)
            cur[gid] = graphgen.add_edges(cur[gid], batch)
            plan.append((float(t), gid, "update", batch, True))
        else:
            plan.append((float(t), gid, "query", [], False))
    log("serving: %d graphs, %d requests planned (%.1f s)" % (graphs, n_req, time.perf_counter() - t_gen))
    srv = Server(budget_bytes=32 << 30, workspace_share=4 << 30, maintenance=maintenance,
                 one_at_a_time=one_at_a_time)
    try:
        t_init = time.perf_counter()
        for gid, g in enumerate(gs):
            srv.add_graph(gid, g, seed=seed + gid, samples=samples)
        torch.cuda.synchronize()
        log("serving: %d x %d resident trees drawn (%.1f s)" % (graphs, samples, time.perf_counter() - t_init))
        reqs = []
        t0 = time.perf_counter()
        for t, gid, kind, batch, ins in plan:
            now = time.perf_counter() - t0
            if t > now:
                time.sleep(t - now)
            r = Request(gid, kind, batch, insert=ins)
            reqs.append(r)
            srv.submit(r)
        while srv.drain(timeout=20.0) < len(reqs):
            log("serving: %d of %d requests served" % (len(srv.done), len(reqs)))
        makespan = time.perf_counter() - t0
        errors = sum(1 for r in reqs if r.error)
        return {
            "workload": "%d resident graphs (cycle of grid, road-like, Chung-Lu types), %d-%d vertices "
                        "log-uniform, %d trees each; Poisson arrivals at %.0f requests/s for %.0f s, "
                        "80%% queries / 20%% update batches: half deletions (1-1000 edges), half "
                        "insertions (1-10 edges), edges with prob. ~ d(u)d(v)"
                        % (graphs, lo, hi, samples, rate, duration),
            "maintenance": "improved (Algorithm 3)" if maintenance else "basic (Algorithm 2)",
            "scheduling": "one request at a time (plain form)" if one_at_a_time else
                          "per-graph workers and streams, requests on different graphs overlap",
            "requests": len(reqs), "errors": errors, "makespan_s": makespan,
            "throughput_req_per_s": len(reqs) / makespan,
            "query": latency_stats(reqs, "query"), "update": latency_stats(reqs, "update"),
            "trees_changed": int(sum(r.result for r in reqs if r.kind == "update" and not r.error)),
        }
    finally:
        srv.close()


def exact_kemeny(offsets, indices) -> float:
    """kappa = sum over the non-unit eigenvalues of D^-1 A of 1 / (1 - lambda)
    (Eq. 1), by a dense FP64 eigensolve of the similar matrix D^-1/2 A D^-1/2."""
    import numpy as np
    n = len(offsets) - 1
    a = np.zeros((n, n))
    src = np.repeat(np.arange(n), np.diff(offsets))
    a[src, indices] = 1.0
    s = 1.0 / np.sqrt(a.sum(axis=1))
    lam = np.sort(np.linalg.eigvalsh(a * s[:, None] * s[None, :]))[:-1]
    return float(np.sum(1.0 / (1.0 - lam)))


def accuracy_leg(seed: int, samples: int, plain: int):
    """K-hat against exact K on the 32x32 grid (1,024 vertices, 1,984 edges),
    and the batched form against the plain one-sample-at-a-time GPU form
    (one kc_estimate call per sample) on the same trees."""
    import torch
    import graphgen
    import paper_2511_16356_amd as kc
    g = graphgen.grid(32, 32)
    k_exact = exact_kemeny(g.offsets, g.indices)
    with kc.Graph.from_graph(g) as G:
        G.reserve(samples)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        est = G.estimate(seed, 0, samples)
        torch.cuda.synchronize()
        t_batch = time.perf_counter() - t0
        t0 = time.perf_counter()
        est_b = G.estimate(seed, 0, plain)
        torch.cuda.synchronize()
        t_batch_plain = time.perf_counter() - t0
        s1 = 0
        t0 = time.perf_counter()
        for s in range(plain):
            s1 += G.estimate(seed, s, 1).sum_f
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
    assert s1 == est_b.sum_f  # the same trees, one at a time or batched
    rel = est.kappa / k_exact - 1.0
    ci = 1.959963984540054 * est.std_error / est.kappa
    log("accuracy: K-hat %.3f exact %.3f rel %.4f ci95 %.4f; plain %.1f vs batched %.1f samples/s" %
        (est.kappa, k_exact, rel, ci, plain / t_plain, plain / t_batch_plain))
    return {"graph": "grid 32x32 (n=1024, m=1984), Philox seed %d" % seed, "samples": samples,
            "kappa": est.kappa, "kappa_exact": k_exact, "rel_error": rel, "rel_ci95": ci,
            "within_eps_0.01": bool(abs(rel) <= 0.01 and ci <= 0.01),
            "batched_samples_per_s": samples / t_batch,
            "plain_vs_batched": {"samples": plain, "plain_samples_per_s": plain / t_plain,
                                 "batched_samples_per_s": plain / t_batch_plain,
                                 "speedup": t_plain / t_batch_plain}}


def plain_leg(G, seed: int, count: int):
    """The plain one-sample-at-a-time GPU form on the benchmark graph: one
    kc_estimate call per sample, for a bounded number of sample ids."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    draws = 0
    for s in range(count):
        draws += G.estimate(seed, s, 1).total_steps
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    log("plain: %d samples one at a time in %.1f s" % (count, dt))
    return {"samples": count, "sample_ids": "0..%d" % (count - 1), "seconds": dt, "samples_per_s": count / dt,
            "draws_per_sample": draws / count}


def plan_requests(cur: list, n_req: int, rate: float, rng, saturate: bool = False):
    """n_req requests on the graphs `cur` (updated in place as the plan's
    updates would change them): Poisson arrivals at `rate` per second (all at
    once if `saturate`), 80% Kemeny queries and 20% update batches, half
    deletions (sizes log-uniform in [1, 1000], batches that keep the graph
    connected) and half insertions (sizes log-uniform in [1, 10]); edges drawn
    with probability proportional to d(u) d(v)."""
    import numpy as np
    import graphgen
    times = np.zeros(n_req) if saturate else np.cumsum(rng.exponential(1.0, size=n_req)) / rate
    plan = []
    for t in times:
        gid = int(rng.integers(0, len(cur)))
        if rng.random() < 0.2:
            if rng.random() < 0.5:
                size = int(round(math.exp(rng.uniform(0.0, math.log(1000.0)))))
                batch = graphgen.deletion_batch(cur[gid], size, rng)
                cur[gid] = graphgen.remove_edges(cur[gid], batch)
                plan.append((float(t), gid, "update", batch, False))
            else:
                size = int(round(math.exp(rng.uniform(0.0, math.log(10.0)))))
                batch = graphgen.insertion_batch(cur[gid], size, rng)
                cur[gid] = graphgen.add_edges(cur[gid], batch)
                plan.append((float(t), gid, "update", batch, True))
        else:
            plan.append((float(t), gid, "query", [], False))
    return plan


def run_plan(srv, plan, label: str):
    """Submit the planned requests at their arrival times and wait for all of
    them; latency is arrival to completion."""
    from paper_2511_16356_amd.serve import Request, latency_stats
    reqs = []
    t0 = time.perf_counter()
    for t, gid, kind, batch, ins in plan:
        while True:
            now = time.perf_counter() - t0
            if t <= now:
                break
            time.sleep(min(t - now, 20.0))
            if t > time.perf_counter() - t0:
                log("serving %s: %d of %d requests submitted, %d served" %
                    (label, len(reqs), len(plan), sum(1 for r in reqs if r.t_done > 0.0)))
        r = Request(gid, kind, batch, insert=ins)
        reqs.append(r)
        srv.submit(r)
    while True:
        done = sum(1 for r in reqs if r.t_done > 0.0)
        if done == len(reqs):
            break
        log("serving %s: %d of %d requests served" % (label, done, len(reqs)))
        srv.drain(timeout=20.0)
    makespan = time.perf_counter() - t0
    return {"requests": len(reqs), "errors": sum(1 for r in reqs if r.error), "makespan_s": makespan,
            "throughput_req_per_s": len(reqs) / makespan,
            "query": latency_stats(reqs, "query"), "update": latency_stats(reqs, "update"),
            "trees_changed": int(sum(r.result for r in reqs if r.kind == "update" and not r.error))}


def serve_sweep(seed: int, graphs: int, lo: int, hi: int, samples: int, n_req: int,
                workspace_share: int, init_share: int, deadline_s: float = 0.0):
    """Served latency against offered load under improved maintenance, on one
    set of resident graphs: the graphs are admitted by footprint (their trees
    drawn concurrently), then the capacity is measured (n_req requests all at
    once: requests per second over the makespan), then Poisson arrivals at
    0.25, 0.5 and 0.8 of it, and at 0.5 the plain form (one request at a time)
    on the same graphs.  Every run draws fresh requests from the same mix on the
    graphs as the earlier runs left them."""
    import numpy as np
    import torch
    import graphgen
    from paper_2511_16356_amd.serve import Server
    t0 = time.perf_counter()
    gs = graphgen.serving_graphs(graphs, lo, hi, seed)
    sizes = sorted(g.n for g in gs)
    log("serving sweep: %d graphs generated, n from %d to %d, sum %d (%.1f s)" %
        (graphs, sizes[0], sizes[-1], sum(sizes), time.perf_counter() - t0))
    free = torch.cuda.mem_get_info()[0]
    budget = int(0.85 * free)
    srv = Server(budget_bytes=budget, workspace_share=workspace_share, maintenance=1, init_share=init_share)
    try:
        t0 = time.perf_counter()
        # largest first, so that the longest initial draws start first
        order = sorted(range(graphs), key=lambda i: -gs[i].n)
        def added(gid, secs, err):
            log("serving sweep: graph %d (n=%d) %s in %.1f s" % (gid, gs[gid].n, "refused" if err else "resident", secs))

        errors = srv.add_graphs([(gid, gs[gid], seed + gid, samples) for gid in order], workers=8, on_added=added)
        t_init = time.perf_counter() - t0
        resident = sum(srv.held.values())
        log("serving sweep: %d graphs resident with %d trees each (%.1f s), %.1f GB held of a %.1f GB budget; "
            "refused: %s" % (len(srv.graphs), samples, t_init, resident / 1e9, budget / 1e9, errors or "none"))
        cur = [gs[i] for i in range(graphs)]
        rng = np.random.default_rng(seed + 1)
        sat = run_plan(srv, plan_requests(cur, n_req, 1.0, rng, saturate=True), "saturated")
        cap = sat["throughput_req_per_s"]
        log("serving sweep: capacity %.2f requests/s" % cap)
        levels = []

        def time_left(frac):
            # a run at `frac` of the capacity takes about n_req / (frac * cap) seconds
            return not deadline_s or time.perf_counter() - T_START + 1.2 * n_req / (frac * cap) < deadline_s

        for frac in (0.25, 0.5, 0.8):
            if not time_left(frac):
                levels.append({"load": frac, "skipped": "deadline of %.0f s" % deadline_s})
                continue
            leg = run_plan(srv, plan_requests(cur, n_req, frac * cap, rng), "load %.2f" % frac)
            leg.update({"load": frac, "rate_req_per_s": frac * cap})
            levels.append(leg)
            q, u = leg["query"] or {}, leg["update"] or {}
            log("serving sweep: load %.2f (%.3f req/s): query p50 %s p99 %s ms, update p50 %s p99 %s ms" %
                (frac, frac * cap, q.get("p50_ms"), q.get("p99_ms"), u.get("p50_ms"), u.get("p99_ms")))
        if time_left(0.5):
            srv.set_schedule(True)
            plain = run_plan(srv, plan_requests(cur, n_req, 0.5 * cap, rng), "plain form, load 0.50")
            plain.update({"load": 0.5, "rate_req_per_s": 0.5 * cap, "scheduling": "one request at a time"})
            srv.set_schedule(False)
        else:
            plain = {"skipped": "deadline of %.0f s" % deadline_s}
        return {"sweep": "served latency vs offered load, improved maintenance (Algorithm 3)",
                "workload": "%d resident graphs (cycle of grid, road-like, Chung-Lu types), %d-%d vertices "
                            "log-uniform (sum %d), %d trees each; 80%% queries / 20%% update batches: half "
                            "deletions (1-1000 edges), half insertions (1-10 edges), edges with prob. ~ d(u)d(v); "
                            "%d requests per run" % (graphs, lo, hi, sum(sizes), samples, n_req),
                "admission": {"budget_bytes": budget, "resident_bytes": resident, "workspace_share": workspace_share,
                              "init_share": init_share, "refused": errors, "init_s": t_init},
                "capacity_req_per_s": cap, "saturated": sat, "levels": levels, "plain_at_0.5": plain}
    finally:
        srv.close()


def study_graphs(points: int):
    """The three synthetic shapes at a reduced size: the 32x32 grid (exact
    kappa known), road-like and social-like graphs of about `points` vertices."""
    import graphgen
    grid = graphgen.grid(32, 32)
    return [("grid 32x32", grid, exact_kemeny(grid.offsets, grid.indices)),
            ("road-like %d points" % points, graphgen.road_like(points, seed=0), None),
            ("social-like %d vertices" % points, graphgen.chung_lu(points, 2.2, 10.0, 5000.0, seed=0), None)]


def study_paths(points: int, samples: int, seed: int):
    """Section 5, Exp-II: the reference tree tau0 (breadth-first, depth-first,
    a uniform random spanning tree) against the spread of f/2m.  The same
    resident trees are evaluated under each tau0, so the comparison is paired;
    the traversal time is that of re-evaluating all of them."""
    import torch
    import paper_2511_16356_amd as kc
    rows = []
    for name, g, exact in study_graphs(points):
        with kc.Graph.from_graph(g) as G:
            t0 = time.perf_counter()
            G.samples_init(seed, samples)
            torch.cuda.synchronize()
            t_sample = time.perf_counter() - t0
            rand_tau0 = G.sample_trees(seed + 1, 0, 1, popcounts=False, steps=False)[0][0].cpu().numpy()
            for label, kind, par in (("bfs", kc.KC_TAU0_BFS, None), ("dfs", kc.KC_TAU0_DFS, None),
                                     ("wilson", kc.KC_TAU0_GIVEN, rand_tau0)):
                t0 = time.perf_counter()
                G.set_tau0(kind, par)
                torch.cuda.synchronize()
                t_eval = time.perf_counter() - t0
                est = G.samples_query()
                rel_sd = est.std_error * math.sqrt(samples) / est.kappa
                row = {"graph": name, "n": g.n, "m": g.two_m // 2, "tau0": label, "depth0": G.info["depth0"],
                       "samples": samples, "kappa": est.kappa, "rel_sd_per_tree": rel_sd,
                       "rel_ci95": 1.959963984540054 * est.std_error / est.kappa,
                       "sampling_s": t_sample, "reevaluate_s": t_eval}
                if exact:
                    row["rel_error_vs_exact"] = est.kappa / exact - 1.0
                rows.append(row)
                log("%s tau0=%s depth0=%d kappa=%.2f rel_sd=%.4f eval %.2f s" %
                    (name, label, row["depth0"], est.kappa, rel_sd, t_eval))
    return {"study": "reference tree tau0 (section 5, Exp-II)", "seed": seed, "rows": rows}


def study_roots(points: int, samples: int, seed: int):
    """Section 5, Exp-III: the root's degree against the sampling time.  Roots
    of degree closest to d_max/5, 2 d_max/5, ..., d_max (the smallest such
    index), each timed over the same sample ids."""
    import numpy as np
    import torch
    import paper_2511_16356_amd as kc
    rows = []
    for name, g, _ in study_graphs(points)[1:]:
        deg = np.diff(g.offsets)
        dmax = int(deg.max())
        for k in range(1, 6):
            target = k * dmax / 5.0
            root = int(np.argmin(np.abs(deg - target)))
            with kc.Graph.from_graph(g, root=root) as G:
                G.reserve(samples)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                est = G.estimate(seed, 0, samples)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                rows.append({"graph": name, "n": g.n, "root": root, "root_degree": int(deg[root]),
                             "target_degree": target, "samples": samples, "seconds": dt,
                             "samples_per_s": samples / dt, "draws_per_sample": est.total_steps / samples,
                             "kappa": est.kappa, "rel_ci95": 1.959963984540054 * est.std_error / est.kappa})
                log("%s root %d (deg %d) %.2f s draws/sample %.0f kappa %.1f" %
                    (name, root, deg[root], dt, est.total_steps / samples, est.kappa))
    return {"study": "root degree (section 5, Exp-III)", "seed": seed, "rows": rows}


def library_sha() -> str:
    """SHA-256 over the estimator library's sources (name, then contents, in
    name order; the memory-ceiling probe is not part of it)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(LIB_SRC)):
        if name.endswith((".hip", ".cpp", ".h")) and name != "kc_probe.hip":
            h.update(name.encode())
            with open(os.path.join(LIB_SRC, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def calibrate_copy(mib: int):
    """A plain device-to-device copy of known size, for scaling HBM counters."""
    import torch
    nbytes = mib << 20
    a = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes}), flush=True)


def calibrate_random(gib: int):
    """Measured ceilings for the roofline (libkc_probe.so), swept over the
    launch settings, best kept: a streaming read of a `gib` GiB buffer (loads
    in flight per thread x blocks per CU), and random reads of 64-byte lines
    from it in the estimator's shapes (8 or 16 bytes per lane from its own
    line, or four lanes on one line) x reads in flight per thread x blocks
    per CU.  Prints one JSON line with every point and the best of each."""
    import ctypes
    import torch
    from paper_2511_16356_amd import build_lib
    lib = ctypes.CDLL(build_lib.PROBE_LIB)
    lib.kc_probe_stream_sweep.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    lib.kc_probe_random_sweep.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]
    nbytes = gib << 30
    buf = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    out = {"buffer_GiB": gib, "stream": [], "random": []}
    val = ctypes.c_double(0.0)
    for inflight in (1, 2, 4, 8):
        for bpc in (4, 8, 16, 32):
            rc = lib.kc_probe_stream_sweep(ctypes.c_void_p(buf.data_ptr()), nbytes, inflight, bpc,
                                           ctypes.c_void_p(sink.data_ptr()), ctypes.byref(val))
            if rc != 0:
                raise RuntimeError("stream probe failed (%d)" % rc)
            out["stream"].append({"inflight": inflight, "blocks_per_cu": bpc, "GBps": val.value})
    shapes = {0: "8 B per lane, own line", 1: "16 B per lane, own line", 2: "4 lanes x 16 B on one line"}
    for shape in (0, 1, 2):
        for inflight in (1, 4, 8, 16, 32):
            for bpc in (4, 8, 16):
                rc = lib.kc_probe_random_sweep(ctypes.c_void_p(buf.data_ptr()), nbytes, shape, inflight, bpc,
                                               ctypes.c_void_p(sink.data_ptr()), ctypes.byref(val))
                if rc != 0:
                    raise RuntimeError("random probe failed (%d)" % rc)
                out["random"].append({"shape": shapes[shape], "inflight": inflight, "blocks_per_cu": bpc,
                                      "lines_per_s": val.value, "GBps_64B": val.value * 64 / 1e9})
        log("random shape %d done" % shape)
    out["best_stream"] = max(out["stream"], key=lambda r: r["GBps"])
    out["best_random"] = max(out["random"], key=lambda r: r["lines_per_s"])
    print(json.dumps(out), flush=True)


WORKLOADS = {
    "dense": ("dense power-law: Chung-Lu, 3,000,000 vertices, expected degrees with exponent 2.0, "
              "mean 76, cap 30,000, largest component (n=%d, m=%d, depth0=%d), int64 offsets on input"),
    "road": ("road-like: thinned random geometric graph, 1,000,000 uniform points, radius for mean "
             "degree 12, edges kept w.p. 0.2055, largest component (n=%d, m=%d, depth0=%d), int32 CSR"),
    "social": ("social-like: Chung-Lu, 1,000,000 vertices, expected degrees with exponent 2.2, mean 10, "
               "cap 5,000, largest component (n=%d, m=%d, depth0=%d), int32 CSR"),
}
DEFAULT_SAMPLES = {"dense": 4096, "road": 4096, "social": 8192}


T_START = time.perf_counter()  # reset when main() starts; the wall-clock budgets count from it


def main():
    global T_START
    T_START = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="dense",
                    help="dense: the headline workload (default); road / social: the other shapes")
    ap.add_argument("--samples", type=int, default=0, help="tree samples per step (launch)")
    ap.add_argument("--autotune", choices=["auto", "on", "off"], default="auto",
                    help="choose the launch options with kc_autotune before timing (auto: for the "
                         "social-like workload, whose configuration asks for it)")
    ap.add_argument("--tune-cache", default="", help="kc_autotune cache file (default: in the temp directory)")
    ap.add_argument("--direct", action="store_true",
                    help="time kc_estimate calls instead of replays of the captured launch")
    ap.add_argument("--chains", type=int, default=0, choices=[0, 1024, 2048],
                    help="chain-table size per sample (KC_OPT_CHAINS; 0: the library's default)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget", type=float, default=480.0,
                    help="wall-clock seconds after which the optional legs are skipped")
    ap.add_argument("--cpu-per-thread", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-latency leg")
    ap.add_argument("--serve-graphs", type=int, default=8)
    ap.add_argument("--serve-rate", type=float, default=5.0, help="requests per second")
    ap.add_argument("--serve-seconds", type=float, default=8.0)
    ap.add_argument("--serve-lo", type=int, default=10_000, help="--serve-sweep: smallest graph (vertices)")
    ap.add_argument("--serve-hi", type=int, default=2_000_000, help="--serve-sweep: largest graph (vertices)")
    ap.add_argument("--serve-samples", type=int, default=1024, help="--serve-sweep: resident trees per graph")
    ap.add_argument("--serve-requests", type=int, default=60, help="--serve-sweep: requests per run")
    ap.add_argument("--serve-workspace", type=int, default=1024, metavar="MIB",
                    help="--serve-sweep: workspace one graph keeps")
    ap.add_argument("--serve-init-workspace", type=int, default=16384, metavar="MIB",
                    help="--serve-sweep: workspace one graph may use while its trees are first drawn")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the exact-K leg on the 32x32 grid")
    ap.add_argument("--plain-samples", type=int, default=2,
                    help="sample ids run one launch each on the benchmark graph (plain form)")
    ap.add_argument("--study", choices=["tau0", "root"], default=None,
                    help="instead of the benchmark, run the reference-tree (Exp-II) or root-degree "
                         "(Exp-III) study on reduced graphs and print its JSON line")
    ap.add_argument("--serve-sweep", action="store_true",
                    help="instead of the benchmark, measure served latency against offered load")
    ap.add_argument("--study-points", type=int, default=100_000)
    ap.add_argument("--study-samples", type=int, default=512)
    ap.add_argument("--calibrate-random", type=int, default=0, metavar="GIB",
                    help="only measure streaming and random 64-byte reads over a GIB GiB buffer and exit")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain copy of MIB MiB (HBM counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (samples would "
              "shard by index range, with one 32-byte all-reduce of the sums at the end)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_random:
        calibrate_random(args.calibrate_random)
        return
    if args.calibrate_copy:
        calibrate_copy(args.calibrate_copy)
        return
    if args.serve_sweep:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(serve_sweep(args.seed + 7, args.serve_graphs, args.serve_lo, args.serve_hi,
                                     args.serve_samples, args.serve_requests, args.serve_workspace << 20,
                                     args.serve_init_workspace << 20, args.budget)), flush=True)
        return
    if args.study:
        import torch
        torch.cuda.set_device(0)
        fn = study_paths if args.study == "tau0" else study_roots
        print(json.dumps(fn(args.study_points, args.study_samples, args.seed)), flush=True)
        return

    import torch
    import graphgen
    import paper_2511_16356_amd as kc

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    g = graphgen.workload(args.workload)
    log("graph %s: n=%d 2m=%d (%.1f s)" % (args.workload, g.n, g.two_m, time.perf_counter() - t0))
    t0 = time.perf_counter()
    G = kc.Graph.from_graph(g)
    info = G.info
    log("prepared on the device (%.1f s): %s" % (time.perf_counter() - t0, info))
    stream = torch.cuda.current_stream()
    B = args.samples or DEFAULT_SAMPLES[args.workload]
    # set-up (not a step): the launch over B samples, captured once as a HIP graph
    # (kc_batch) with its workspace; launch L estimates samples L*B .. (L+1)*B - 1,
    # so the warm-up launches take the first ids and the timed ones the next
    if args.chains:
        G.set_option(kc.KC_OPT_CHAINS, args.chains)
    tuned = None
    if args.autotune == "on" or (args.autotune == "auto" and args.workload == "social"):
        # set-up: choose the launch options for batches of B samples (trial estimates
        # on sample ids from 2^40, far from the ones timed), then free the trials' workspace
        import tempfile
        t0 = time.perf_counter()
        cache = args.tune_cache or os.path.join(tempfile.gettempdir(), "kc_autotune.jsonl")
        tuned = G.autotune(B, cache_path=cache, stream=stream)
        tuned["seconds"] = time.perf_counter() - t0
        tuned["cache"] = cache
        G.trim(stream)
        log("autotune (%.1f s): %s" % (tuned["seconds"], tuned))
    batch = None
    if not args.direct:
        batch = kc.Batch([G], [args.seed], [0], [B], stream=stream)
    else:
        G.reserve(B)
    torch.cuda.synchronize()

    import threading
    watch_stop = threading.Event()
    if batch is None:
        # a direct launch can run for minutes (road-like graphs): report the samples
        # it has finished every 30 s, read from the counters the kernel publishes
        def watch():
            while not watch_stop.wait(30.0):
                log("  %d of %d samples of the running launch done" % (G.progress(), B))

        threading.Thread(target=watch, daemon=True).start()

    def step(k):
        if batch is None:
            return G.estimate(args.seed, k * B, B)
        batch.launch(stream)
        (est,), launches = batch.results(stream)
        assert launches == k + 1
        return est

    for w in range(args.warmup):
        step(w)
        log("warmup step %d done" % w)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ests = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        starts[k].record(stream)
        est = step(args.warmup + k)
        ends[k].record(stream)
        ests.append(est)
        log("step %d: kappa=%.1f +- %.1f draws/sample=%.0f" % (k, est.kappa, est.std_error, est.total_steps / B))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    watch_stop.set()
    launch_ms = [starts[k].elapsed_time(ends[k]) for k in range(args.steps)]
    if batch is not None:
        batch.close()

    total = B * args.steps
    pooled = G.combine(ests)
    draws = pooled.total_steps
    alg = algorithmic_bytes(draws, g.n, g.two_m, info["depth0"], total)
    avg_launch_s = sum(launch_ms) / len(launch_ms) / 1e3
    achieved = alg / args.steps / avg_launch_s / 1e9  # GB/s: algorithmic bytes per launch over its duration
    meas = None
    for m in MEASURED_TRAFFIC.get(library_sha(), []):
        if (m["workload"], m["samples"], m["seed"], m.get("direct", False)) == \
                (args.workload, B, args.seed, bool(args.direct)):
            meas = m
    traffic = None  # HBM bytes per launch, when counters exist for this kernel and workload
    if meas:
        traffic = meas["bytes"]
    value = total / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {
            "workload": (WORKLOADS[args.workload] % (g.n, g.two_m // 2, info["depth0"])) +
                        "; %d tree samples per step (one persistent launch%s), Philox seed %d" %
                        (B, "" if args.direct else ", replayed from a captured HIP graph", args.seed),
            "samples_per_step": B,
            "parallelism": "1 GPU, one wavefront per sample in flight",
            "chains_per_sample": G.info["chains"],
        },
        "kappa": pooled.kappa,
        "kappa_std_error": pooled.std_error,
        "kappa_rel_ci95": 1.959963984540054 * pooled.std_error / pooled.kappa if pooled.kappa else None,
        "draws_per_sample": draws / total,
        "draws_per_sampler_round": draws / max(1, pooled.sampler_iterations),
        "launch_ms": launch_ms,
        "autotune": tuned,
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "algorithmic_bytes_per_launch": alg / args.steps,
            "measured_ceilings": dict(MEASURED_CEILINGS),
            "frac_of_random_64B_ceiling": achieved / MEASURED_CEILINGS["random_64B_read_GBps"],
        },
    }
    if traffic:
        # the counted bytes against the algorithmic ones, and the HBM rate they imply
        out["roofline"]["traffic_over_algorithmic"] = traffic / (alg / args.steps)
        out["roofline"]["traffic_GBps"] = traffic / avg_launch_s / 1e9
    log("timed: %.1f samples/s, %.1f ms per launch, %.0f GB/s algorithmic" % (value, avg_launch_s * 1e3, achieved))

    def budget_left(need_s: float) -> bool:
        return time.perf_counter() - T_START + need_s < args.budget

    skipped = {"skipped": "wall-clock budget of %.0f s reached" % args.budget}
    if not args.no_cpu:
        # the oracle is test infrastructure: a failure is reported, never a fallback
        threads = min(16, os.cpu_count() or 1)
        try:
            out["cpu_baseline"] = cpu_baseline(g, args.seed, 0, threads, args.cpu_per_thread) \
                if budget_left(60) else skipped
        except Exception as exc:
            out["cpu_baseline"] = {"error": str(exc)}
    if args.plain_samples > 0:
        out["plain_one_at_a_time"] = plain_leg(G, args.seed, args.plain_samples) if budget_left(30) else skipped
        if "samples_per_s" in out["plain_one_at_a_time"]:
            out["plain_one_at_a_time"]["batched_samples_per_s"] = value
    G.close()
    del G
    if not args.no_accuracy:
        out["accuracy"] = accuracy_leg(args.seed, 8192, 2000) if budget_left(30) else skipped
    if not args.no_serve:
        out["served"] = serving_leg(args.seed + 7, args.serve_graphs, 10_000, 30_000, 1024, args.serve_rate,
                                    args.serve_seconds, maintenance=1) if budget_left(60) else skipped
    out["wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
