#!/usr/bin/env python3
"""Benchmark of the IMIN estimator on one MI355X.

Workload (default ``large``): directed Chung-Lu power-law graph with 1,000,000
nodes and 10,000,000 edges (degree exponent 2.1), trivalency probabilities
{0.1, 0.01, 0.001}, |S| = 200 uniform seeds, theta = 200,000 worlds (k = 500
for the greedy solves).  Inputs (graph handle, seeds, output buffers) are
resident in HBM before the timed region.

One step is one from-scratch pass of the estimator over all theta worlds
(``imin_evaluate``): sample every live-edge world, BFS from the seeds,
dominators and subtree sizes, and the per-node gain reduction.  ``value`` is
theta divided by the pass time (worlds/s).  The ``roofline`` object is that of
the world kernel of the tier that evaluates most of the pass's worlds (tier 0
on the trivalency graph, the HBM tier on the weighted-cascade medium
workload), timed with HIP events recorded by its own launch; the Philox and
copy probes give the measured ALU and HBM ceilings.  After the timed passes, full greedy solves (k rounds, with
incremental rounds) give the query latency percentiles; the CPU oracle's
from-scratch rate on the same query is the ``cpu_baseline``.

With ``--many N`` it measures instead a batch of N mixed queries on the same
graph (|S| uniform in 10..500, k uniform in 10..200, theta 10^4 or 10^5, each
with its own coin key): solved one after another on one stream, then side by
side on ``--streams`` streams (``imin_solve_many``), with the results of the
two runs checked to be identical; one JSON line with both rates.

With ``--serve N`` it replays N queries arriving at ``--rate`` per second
(exponential gaps; |S| uniform in 10..1000, k uniform in 10..500, theta
5*10^4) against a server on ``--streams`` streams (``imin_server_*``), and
reports the latency percentiles from arrival to result next to those of a
single queue served one query at a time (each query's time measured alone).

The default run also times LSBM (Algorithm 4: the stopping-rule estimate of
the spread, OPT^L, Max-Coverage on doubling pools of CP sequences with the
sigma bounds' stopping test) on the same graph and seeds with k = --lsbm-k,
eps = --lsbm-eps, beta = 0.1, delta = 1/n; ``--lsbm-only`` does that alone on
a named graph or workload, and with ``--sandwich`` also GSBM, LHGA and
SandIMIN (Algorithm 1).
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

METRIC = "live-edge worlds/sec (sample+BFS+gain) at 1M-node graph; p50/p99 IMIN query latency"
HBM_PEAK_GBS = 8000.0
TIMED_EVERY = 8
L0_KERNEL = 8  # the library's kernel id of the level-0 draw
RNG_SEED = 2024


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


KERNEL_SOURCES = ["imin_world.hip", "imin_device.hpp", "imin_internal.hpp", "imin_select.hpp"]


def measured_traffic(kernel: str, workload: str = "large"):
    """HBM bytes per launch of a world kernel from its committed FETCH_SIZE /
    WRITE_SIZE profile, or None when there is none or the kernel sources
    have changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", f"{workload}_{kernel}_traffic.md")).read()
    except OSError:
        return None
    fields = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("    "):
            k, v = line.strip().split(":", 1)
            fields[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2405_12871_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("kernel_source_sha256") != h.hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(g, seeds, theta, budget_s, gpu_gain):
    """The oracle as it stands, on a bounded sample of the same workload: its
    from-scratch pass (dominator mode, no blockers) over the first worlds of
    the same query, sized to about ``budget_s`` seconds of CPU work (all theta
    worlds when that fits).  When the sample is the whole workload its gains
    are compared with the GPU's."""
    import numpy as np

    from oracle import oracle
    q = oracle.Query(g, seeds)
    threads = oracle.default_threads()
    nw = max(64, min(theta, 2000))
    t0 = time.perf_counter()
    q.eval(RNG_SEED, 0, nw, threads=threads)
    per_world = (time.perf_counter() - t0) / nw
    nw2 = int(min(theta, max(nw, budget_s / max(per_world, 1e-12))))
    t0 = time.perf_counter()
    gain, total = q.eval(RNG_SEED, 0, nw2, threads=threads)
    dt = time.perf_counter() - t0
    out = {"value": nw2 / dt, "unit": "worlds/s", "cores": threads, "kind": "oracle",
           "sample": f"from-scratch pass (dominator mode, no blockers) over worlds [0, {nw2}) of the same "
                     f"query ({'all' if nw2 == theta else 'a prefix'} of theta={theta}); {dt:.1f} s on "
                     f"{threads} threads", "seconds": dt}
    if nw2 == theta:
        out["oracle_gains_equal_gpu"] = bool(np.array_equal(gain, gpu_gain))
    return out


def _same_result(a, b):
    import numpy as np
    return (not isinstance(a, Exception) and not isinstance(b, Exception) and a.n_selected == b.n_selected and
            np.array_equal(a.blockers, b.blockers) and np.array_equal(a.gains, b.gains) and
            np.array_equal(a.spread_totals, b.spread_totals))


def _solve_alone(binding, Gs, queries, label):
    """Each query solved alone, one after another (imin_solve with the block
    cache): its service time and its result."""
    import torch
    service, alone = [], []
    t_all = time.perf_counter()
    for i, (gi, seeds, k, theta, rng) in enumerate(queries):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alone.append(binding.solve(Gs[gi], seeds, k, theta, rng))
        service.append(time.perf_counter() - t0)
        log(f"{label} {i + 1}/{len(queries)}: graph {gi} |S|={len(seeds)} k={k} theta={theta} "
            f"{service[-1] * 1e3:.1f} ms (elapsed {time.perf_counter() - t_all:.1f} s)")
    return service, alone


def run_many(args, binding, dev):
    """A batch of mixed queries on the weighted-cascade twin of the
    1M-node graph, solved one after another and then all submitted at once
    to the serving runtime (pool admission, several streams)."""
    import numpy as np
    import torch

    from paper_2405_12871_amd import synth
    t0 = time.perf_counter()
    g = synth.named_graph(args.graph)
    log(f"graph {args.graph}: n={g.n} m={g.m} ({time.perf_counter() - t0:.1f} s)")
    G = binding.Graph.from_synth(g, device=dev)
    queries = synth.query_mix(args.many, [g.n], 0xB0, (10, 500), (10, 200), (10_000, 100_000))
    # one query of each size class first, so that the graph's record sizes
    # later workspaces (both runs start from it)
    binding.solve(G, queries[0][1], queries[0][2], queries[0][3], queries[0][4])
    service, alone = _solve_alone(binding, [G], queries, "alone")
    t_seq = sum(service)
    srv = binding.Server(G, n_streams=args.streams, hbm_budget=int(args.pool_gib * (1 << 30)))
    got, done_at = {}, {}
    torch.cuda.synchronize()
    start = time.perf_counter()
    owner = {srv.submit(s, k, th, r): i for i, (_, s, k, th, r) in enumerate(queries)}
    for j in range(len(queries)):
        t, r = srv.next()
        i = owner[t]
        got[i], done_at[i] = r, time.perf_counter() - start
        log(f"batch {j + 1}/{len(queries)}: query {i} done at {done_at[i]:.2f} s")
    t_par = time.perf_counter() - start
    srv.close()
    same = all(_same_result(got[i], alone[i]) for i in range(len(queries)))
    lat = [done_at[i] for i in range(len(queries))]
    print(json.dumps({
        "metric": "IMIN queries/s, batch of mixed queries on one resident graph",
        "value": len(queries) / t_par,
        "unit": "queries/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "dtype": "u32+int64",
        "config": {"workload": f"batched queries: {args.graph} weighted cascade (n={g.n}, m={g.m}), {len(queries)} queries: "
                               f"|S|~U{{10..500}}, k~U{{10..200}}, theta in {{1e4, 1e5}}, all submitted at once",
                   "streams": args.streams, "pool_GiB": args.pool_gib},
        "batch_seconds": t_par,
        "sequential_seconds": t_seq,
        "sequential_queries_per_s": len(queries) / t_seq,
        "speedup_over_sequential": t_seq / t_par,
        "batch_completion_p50_s": percentile(lat, 50),
        "batch_completion_p99_s": percentile(lat, 99),
        "service_ms_p50": percentile(service, 50) * 1e3,
        "service_ms_p99": percentile(service, 99) * 1e3,
        "identical_to_alone": bool(same),
        "blockers_selected": int(sum(r.n_selected for r in alone)),
    }), flush=True)


def run_packed(args, binding, dev):
    """A batch of from-scratch passes on the 1M-node workload's graph: each
    query its own 200 uniform seeds, world range and rng seed, and
    --packed-worlds worlds.  Timed one after another (imin_evaluate per
    query) and as one batch (imin_evaluate_batch, tier-0 launches packed);
    every query's gains and total must be identical both ways."""
    import numpy as np
    import torch

    from paper_2405_12871_amd import synth
    g, seeds0, _, _ = synth.workload("large")
    G = binding.Graph.from_synth(g, device=dev)
    rng = np.random.default_rng(0xBA7C)
    nq, nw = args.packed, args.packed_worlds
    entries_a, entries_b = [], []
    for j in range(nq):
        sd = torch.from_numpy(rng.choice(g.n, 200, replace=False).astype(np.int32)).to(dev)
        entries_a.append((sd, nw * j, nw, 100 + j, torch.empty(g.n, dtype=torch.int64, device=dev),
                          torch.empty(1, dtype=torch.int64, device=dev)))
        entries_b.append((sd, nw * j, nw, 100 + j, torch.empty(g.n, dtype=torch.int64, device=dev),
                          torch.empty(1, dtype=torch.int64, device=dev)))

    def one_by_one():
        for sd, wb, wc, seed, gain, total in entries_a:
            binding.evaluate_device(G, sd, wb, wc, seed, gain, total)

    def batched():
        binding.evaluate_batch_device(G, entries_b)

    times = {"one_by_one": [], "batched": []}
    for rep in range(args.packed_reps + 1):  # the first of each is a warm-up
        for name, fn in (("one_by_one", one_by_one), ("batched", batched)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            if rep:
                times[name].append(time.perf_counter() - t0)
        log(f"rep {rep}: " + " ".join(f"{k} {v[-1] * 1e3:.1f} ms" for k, v in times.items() if v))
    same = all(torch.equal(a[4], b[4]) and torch.equal(a[5], b[5]) for a, b in zip(entries_a, entries_b))
    t_a, t_b = float(np.median(times["one_by_one"])), float(np.median(times["batched"]))
    worlds = nq * nw
    print(json.dumps({
        "metric": "worlds/s, a batch of from-scratch passes (sample + BFS + dominators + gain sums)",
        "value": worlds / t_b,
        "unit": "worlds/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "dtype": "u32+int64",
        "config": {"workload": f"batched passes: large graph (n={g.n}, m={g.m}, trivalency), {nq} queries of "
                               f"{nw} worlds, |S| = 200 uniform each", "pack_queries": os.environ.get(
                                   "IMIN_PACK_QUERIES", "64")},
        "batched_ms": t_b * 1e3,
        "one_by_one_ms": t_a * 1e3,
        "one_by_one_worlds_per_s": worlds / t_a,
        "speedup_over_one_by_one": t_a / t_b,
        "reps": args.packed_reps,
        "identical_to_one_by_one": bool(same),
    }), flush=True)


def run_serve(args, binding, dev):
    """Poisson arrivals over resident weighted-cascade graphs (default: the
    100K-, 1M- and 4M-node ones) against the serving runtime, next to one
    queue served one query at a time (each query's service time measured
    alone)."""
    import threading

    import numpy as np
    import torch

    from paper_2405_12871_amd import synth
    names = args.graphs.split(",")
    gs = []
    for nm in names:
        t0 = time.perf_counter()
        gs.append(synth.named_graph(nm))
        log(f"graph {nm}: n={gs[-1].n} m={gs[-1].m} ({time.perf_counter() - t0:.1f} s)")
    Gs = [binding.Graph.from_synth(g, device=dev) for g in gs]
    queries = synth.query_mix(args.serve, [g.n for g in gs], 0x5E, (10, 1000), (10, 500), (50_000,),
                              n_graphs=len(gs))
    rs = np.random.default_rng(0x5E5E)
    arrivals = np.cumsum(rs.exponential(1.0 / args.rate, size=len(queries)))
    for gi, G in enumerate(Gs):  # a first query on each graph records its scratch needs
        q = next(q for q in queries if q[0] == gi) if any(q[0] == gi for q in queries) else None
        if q is not None:
            binding.solve(G, q[1], q[2], q[3], q[4])
    service, alone = _solve_alone(binding, Gs, queries, "alone")
    free, seq_lat = 0.0, []
    for a, sv in zip(arrivals, service):
        free = max(free, a) + sv
        seq_lat.append(free - a)
    log(f"serving at {args.rate}/s on {args.streams} streams")
    srv = binding.Server(Gs[0], n_streams=args.streams, hbm_budget=int(args.pool_gib * (1 << 30)))
    finish, results, tickets = {}, {}, {}
    lock = threading.Lock()
    submitted = threading.Semaphore(0)  # next() only while a query is outstanding

    def collect():
        for j in range(len(queries)):
            submitted.acquire()
            t, r = srv.next()
            now = time.perf_counter()
            with lock:
                i = tickets.pop(t)
            finish[i] = now
            results[i] = r
            log(f"served {j + 1}/{len(queries)}: query {i} latency {(now - start - arrivals[i]) * 1e3:.0f} ms")

    waiter = threading.Thread(target=collect)
    start = time.perf_counter()
    for i, ((gi, s, k, th, r), a) in enumerate(zip(queries, arrivals)):
        delay = start + a - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        with lock:
            tickets[srv.submit(s, k, th, r, graph=Gs[gi])] = i
        submitted.release()
        if i == 0:
            waiter.start()
    waiter.join()
    srv.close()
    lat = [finish[i] - (start + arrivals[i]) for i in range(len(queries))]
    same = all(_same_result(results[i], alone[i]) for i in range(len(queries)))
    span = max(finish.values()) - start
    print(json.dumps({
        "metric": "IMIN query latency under Poisson arrivals, p50/p99",
        "value": percentile(lat, 50) * 1e3,
        "unit": "ms (p50)",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic",
        "dtype": "u32+int64",
        "config": {"workload": f"served queries: graphs {names} (weighted cascade), {len(queries)} queries at {args.rate}/s "
                               f"(graph uniform, |S|~U{{10..1000}}, k~U{{10..500}}, theta=5e4)",
                   "streams": args.streams, "pool_GiB": args.pool_gib},
        "p50_ms": percentile(lat, 50) * 1e3,
        "p99_ms": percentile(lat, 99) * 1e3,
        "throughput_queries_per_s": len(queries) / span,
        "one_at_a_time": {"p50_ms": percentile(seq_lat, 50) * 1e3, "p99_ms": percentile(seq_lat, 99) * 1e3,
                          "mean_service_ms": float(np.mean(service)) * 1e3,
                          "throughput_queries_per_s": len(queries) / max(free, 1e-9)},
        "identical_to_alone": bool(same),
    }), flush=True)


def probe_ceilings(binding, dev, theta, ebar, cus):
    """Measured ceilings: Philox coins/s with the world kernels' coin layout
    (theta worlds of about Ebar/4 slot groups), and device copy GB/s (1 GiB)."""
    import torch
    groups = max(1, int(round(ebar / 4)))
    grid = cus * 8
    binding.probe_philox(theta, groups, RNG_SEED, grid, dev)  # warm
    ms = min(binding.probe_philox(theta, groups, RNG_SEED, grid, dev) for _ in range(3))
    coins = 4.0 * theta * groups / (ms / 1e3)
    src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    binding.probe_copy(dst, src, cus * 16)
    cms = min(binding.probe_copy(dst, src, cus * 16) for _ in range(3))
    nbytes = src.numel() * 4
    del src, dst
    torch.cuda.synchronize()
    return {"philox_coins_per_s": coins, "philox_probe_ms": ms, "philox_blocks": theta * groups,
            "copy_GBps": 2.0 * nbytes / (cms / 1e3) / 1e9, "copy_bytes": nbytes, "copy_probe_ms": cms}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--solves", type=int, default=5, help="full greedy solves for the latency figures (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--many", type=int, default=0, help="measure a batch of this many mixed queries instead")
    ap.add_argument("--graph", default="wc1m", help="graph of --many (a name of synth.GRAPHS)")
    ap.add_argument("--streams", type=int, default=4, help="streams for --many and --serve")
    ap.add_argument("--pool-gib", type=float, default=0.0, help="workspace pool of --many/--serve (0: default)")
    ap.add_argument("--serve", type=int, default=0, help="measure latency of this many arriving queries instead")
    ap.add_argument("--graphs", default="wc100k,wc1m,wc4m", help="graphs of --serve")
    ap.add_argument("--rate", type=float, default=200.0, help="arrivals per second for --serve")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--theta", type=int, default=0, help="worlds per pass instead of the workload's")
    ap.add_argument("--k", type=int, default=-1, help="budget of the solves instead of the workload's")
    ap.add_argument("--packed", type=int, default=0, help="measure a batch of this many from-scratch passes instead")
    ap.add_argument("--packed-worlds", type=int, default=2000, help="worlds per query of --packed")
    ap.add_argument("--packed-reps", type=int, default=5, help="timed repetitions of --packed")
    ap.add_argument("--lsbm-k", type=int, default=100, help="budget of the LSBM measurement")
    ap.add_argument("--lsbm-eps", type=float, default=0.2, help="eps of the LSBM measurement")
    ap.add_argument("--no-lsbm", action="store_true", help="skip the LSBM measurement")
    ap.add_argument("--lsbm-only", action="store_true", help="measure LSBM alone on --graph")
    ap.add_argument("--lsbm-seeds", type=int, default=10, help="seeds of --lsbm-only on a named graph")
    ap.add_argument("--lsbm-top", action="store_true", help="--lsbm-only seeds: the highest out-degrees")
    ap.add_argument("--sandwich", action="store_true", help="--lsbm-only also times GSBM, LHGA and SandIMIN")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the estimator would shard "
              f"by world range, one range per GPU, and this benchmark drives a single device",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2405_12871_amd import binding, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.many > 0:
        run_many(args, binding, dev)
        return
    if args.serve > 0:
        run_serve(args, binding, dev)
        return
    if args.packed > 0:
        run_packed(args, binding, dev)
        return
    if args.lsbm_only:
        run_lsbm(args, binding, dev)
        return
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    log(f"generating workload {args.workload}")
    t0 = time.perf_counter()
    g, seeds, k, theta = synth.workload(args.workload)
    if args.theta > 0:
        theta = args.theta  # the workload's graph and seeds with another world count
    if args.k >= 0:
        k = args.k
    log(f"  n={g.n} m={g.m} |S|={len(seeds)} k={k} theta={theta} ({time.perf_counter() - t0:.1f} s)")

    # inputs resident in HBM
    row_ptr = torch.as_tensor(g.row_ptr).to(dev)
    col = torch.as_tensor(g.col).to(dev)
    p = torch.as_tensor(g.p).to(dev)
    seeds_dev = torch.as_tensor(seeds).to(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    G = binding.Graph(g.n, row_ptr, col, p, device=dev)
    torch.cuda.synchronize()
    ingest_ms = (time.perf_counter() - t0) * 1e3
    log(f"graph ingest {ingest_ms:.2f} ms")

    # per-world sizes of the workload (an untimed pass): R and E per world
    _, T0, wsize, _, wedges = binding.evaluate(G, seeds_dev, 0, theta, RNG_SEED, per_world=True, edges=True)
    R = wsize.astype(np.int64)
    E = wedges.astype(np.int64)
    ns = len(seeds)
    log(f"workload: T0={T0} Rbar={R.mean():.1f} Ebar={E.mean():.1f}")
    ceil = probe_ceilings(binding, dev, theta, float(E.mean()), cus)
    log(f"ceilings: Philox {ceil['philox_coins_per_s'] / 1e12:.3f} T coins/s, copy {ceil['copy_GBps']:.0f} GB/s")

    tuned = None
    if not args.no_autotune:
        # launch-shape tuning on this query (results unchanged by any shape),
        # before the warm-up and outside the timed region
        pct, tms = binding.autotune(G, seeds_dev, theta, RNG_SEED)
        tuned = {"grid0_pct_of_residency": pct, "best_pass_ms_while_tuning": tms}
        log(f"autotune: tier-0 grid {pct}% of its LDS residency ({tms:.2f} ms per pass while tuning)")
    gain = torch.empty(g.n, dtype=torch.int64, device=dev)
    total = torch.empty(1, dtype=torch.int64, device=dev)
    # the work tallies, per tier, of one untimed pass: every later pass of this
    # query evaluates the same worlds in the same tiers (the first pass on a
    # handle may take other tiers and redo a tile whose scratch it outgrew, so
    # a pass whose tiers did not finish each world exactly once is repeated)
    for attempt in range(3):
        binding.timing_enable(True)
        binding.timing_mask([])
        binding.timing_reset()
        binding.evaluate_device(G, seeds_dev, 0, theta, RNG_SEED, gain, total)
        torch.cuda.synchronize()
        work = [binding.timing_work(t) for t in range(3)]
        binding.timing_enable(False)
        binding.timing_mask(None)
        if sum(w[0] for w in work) == theta:
            break
    assert sum(w[0] for w in work) == theta, "the tally pass did not finish every world exactly once"
    for i in range(args.warmup):
        binding.evaluate_device(G, seeds_dev, 0, theta, RNG_SEED, gain, total)
    torch.cuda.synchronize()
    # the roofline is that of the world tier that evaluates most of the
    # workload's worlds: tier 0 on the trivalency graph, the HBM tier on the
    # weighted-cascade ones (their worlds hold tens of thousands of nodes).
    # Every launch of that tier's kernel in the timed passes records its own
    # start and stop events (hipExtLaunchKernel on the library's stream); no
    # other kernel is bracketed, and no work tallies are taken (they cost each
    # pass a clear, a copy to the host and a sum)
    dom = max(range(3), key=lambda t: work[t][0])
    dom_kernel = {0: 0, 1: 4, 2: 1}[dom]  # the library's kernel ids of tiers 0, 1, 2
    binding.timing_enable(True)
    binding.timing_tallies(False)
    binding.timing_mask([dom_kernel, L0_KERNEL])
    binding.timing_sample(1)
    binding.timing_reset()
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        binding.evaluate_device(G, seeds_dev, 0, theta, RNG_SEED, gain, total)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    log("passes: " + " ".join(f"{x:.2f}" for x in lat) + " ms")
    n0, ms0 = binding.timing_read(dom_kernel)
    nl0, msl0 = binding.timing_read(L0_KERNEL)
    binding.timing_enable(False)
    binding.timing_tallies(True)
    binding.timing_mask(None)
    assert int(total.cpu()[0]) == T0, "passes must reproduce the characterisation pass"
    gpu_gain = gain.cpu().numpy()
    ms_per_step = total_s * 1e3 / args.steps
    value = theta / (ms_per_step / 1e3)

    # roofline of that world kernel: bytes per world as the from-scratch
    # unit of work counts them, restricted to what the world kernel itself
    # moves (sampling, BFS, dominators, subtree sizes, pair output):
    #   8 E (column + threshold per scanned slot) + 8 R (row offsets)
    #   + 4 L (visited touches per live edge) + 12 R (reached list and live
    #   subgraph) + 8 R (its (node, count) pair written)
    # with E, R, L tallied over the worlds the kernel finished; the pair's
    # bucketing and accumulation (16 R more) belong to the reduction kernels.
    # The seeds' level 0 of every world is drawn by its own kernel ahead of
    # the world kernels (from-scratch passes), so the same bytes are taken
    # over both kernels' time: one launch of each per pass.
    w0, e0, b0, r0, l0 = work[dom]
    k14 = 8 * e0 + 28 * r0 + 4 * l0
    avg_world = ms0 / max(n0, 1)
    avg_l0 = msl0 / max(nl0, 1)
    avg0 = avg_world + avg_l0
    achieved = k14 / (avg0 / 1e3) / 1e9
    allw = [sum(wk[i] for wk in work) for i in range(5)]
    pass_bytes = 8 * allw[1] + 44 * allw[3] + 4 * allw[4]
    coins0 = e0  # coins that tier's worlds needed (slots of reached rows)

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "worlds/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32+int64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: directed Chung-Lu n={g.n} m={g.m} gamma=2.1 "
                        f"{'trivalency' if args.workload == 'large' else 'weighted-cascade'}, "
                        f"|S|={ns}, theta={theta}; one step = one from-scratch pass over all theta worlds "
                        f"(sample + BFS + dominators + gain reduction)",
            "n": g.n, "m": g.m, "seeds": ns, "k": k, "theta": theta, "rng_seed": RNG_SEED,
            "graph_sha256": g.sha256()[:16],
        },
        "value_definition": "theta / wall time of one from-scratch pass over theta live-edge worlds (coins, BFS "
                            "from S, dominator-subtree sizes, per-node gain sums), inputs resident in HBM",
        "pass_ms_p50": percentile(lat, 50),
        "pass_ms_min": min(lat),
        "Rbar": float(R.mean()),
        "Ebar": float(E.mean()),
        "Lbar": allw[4] / max(allw[0], 1),
        "T0": int(T0),
        "roofline": {
            "bound": "hbm",
            "kernel": {0: "k_world_lds tier 0 (one wave per world)", 1: "k_world_lds tier 1 (four waves per world)",
                       2: "k_world_hbm tier 2 (per-world arrays in HBM)"}[dom] +
                      " (the world tier of most of the pass's worlds) with k_level0_bits (the seeds' level 0 of "
                      "every world, drawn ahead), every launch of the timed passes, durations from events recorded "
                      "by the launches themselves",
            "world_kernel_ms": avg_world,
            "level0_kernel_ms": avg_l0,
            "tier": dom,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(f"world_tier{dom}", args.workload),
            "traffic_unit": "HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE, committed profile)",
            "bytes_per_world": "8E + 28R + 4L (see value_definition of the pass roofline)",
            "algorithmic_bytes_per_launch": k14,
            "worlds_per_launch": w0,
            "avg_launch_ms": avg0,
            "launches": n0,
            "level0_launches": nl0,
            "hbm_only_algorithmic_bytes_per_launch": b0,
            "coins_per_s": coins0 / (avg0 / 1e3),
            "coins_frac_of_philox_probe": coins0 / (avg0 / 1e3) / ceil["philox_coins_per_s"],
            "frac_of_copy_probe": achieved / ceil["copy_GBps"],
        },
        "pass_roofline": {
            "achieved": pass_bytes / (ms_per_step / 1e3) / 1e9, "unit": "GB/s",
            "bytes_per_pass": pass_bytes,
            "bytes_per_world": "8E + 8R + 4L + 12R + 24R over every world of the pass",
        },
        "ceilings": ceil,
        "graph_ingest_ms": ingest_ms,
        "autotune": tuned,
    }
    if args.solves > 0:
        res.update(solve_latency(args, binding, G, seeds_dev, k, theta, dev))
    if not args.no_lsbm:
        log(f"lsbm: k={args.lsbm_k} eps={args.lsbm_eps}")
        res["lsbm"] = lsbm_measure(binding, G, seeds_dev, args.lsbm_k, args.lsbm_eps, 0.1, 1.0 / g.n, RNG_SEED)
        log(f"  {res['lsbm']}")
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(g, seeds, theta, args.cpu_seconds, gpu_gain)
    print(json.dumps(res), flush=True)


def lsbm_measure(binding, G, seeds_dev, k, eps, beta, delta, rng_seed, repeats=2):
    """LSBM (Algorithm 4) wall time: the fastest of `repeats` calls; the
    worlds it uses (the stopping rule's N, then both pools at every
    iteration) per second.  The stopping rule's doubling batches also draw
    the worlds past N in the batch where its sum crosses the threshold."""
    import torch
    best, res = None, None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = binding.lsbm(G, seeds_dev, k, eps=eps, beta=beta, delta=delta, rng_seed=rng_seed)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    info = res["info"]
    out = {"k": k, "eps": eps, "beta": beta, "delta": delta, "seconds": best, "n_selected": res["n_selected"],
           "returned_on": bool(info["returned_on"]), "on_size": info["on_size"]}
    if not info["returned_on"]:
        theta0 = int(math.ceil(info["theta_0"]))
        pools = 2 * theta0 * ((1 << info["iterations"]) - 1)
        worlds = info["sra_worlds"] + pools
        out.update({"iterations": info["iterations"], "i_max": info["i_max"], "theta": info["theta"],
                    "sra_worlds": info["sra_worlds"], "i_hat": info["i_hat"], "opt_l": info["opt_l"],
                    "theta_0": info["theta_0"], "theta_max": info["theta_max"],
                    "cov1": info["cov1"], "cov2": info["cov2"], "cov_upper": info["cov_upper"],
                    "sigma_ratio": info["sigma_l"] / info["sigma_u"], "target_ratio": 1 - 1 / math.e - eps,
                    "est_lower_bound_DL": info["cov2"] / info["theta"],
                    "worlds_used": worlds, "worlds_per_s": worlds / best})
    return out


def timed_call(fn, repeats=2):
    """(fastest wall time in s, last result) of `repeats` calls."""
    import torch
    best, res = None, None
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        best = dt if best is None else min(best, dt)
    return best, res


def run_lsbm(args, binding, dev):
    """One JSON line: LSBM (and with --sandwich also GSBM, LHGA and SandIMIN)
    on a named graph or workload, |S| = --lsbm-seeds seeds (uniform, or the
    highest out-degrees with --lsbm-top)."""
    import torch
    from paper_2405_12871_amd import synth
    if args.graph in ("small", "medium", "large"):
        g, seeds, _, _ = synth.workload(args.graph)
    else:
        g = synth.named_graph(args.graph)
        seeds = synth.seeds_top_out(g, args.lsbm_seeds) if args.lsbm_top else \
            synth.seeds_uniform(g.n, args.lsbm_seeds, 7)
    G = binding.Graph.from_synth(g, device=dev)
    seeds_dev = torch.as_tensor(seeds).to(dev)
    k, eps, delta = args.lsbm_k, args.lsbm_eps, 1.0 / g.n
    log(f"lsbm on {args.graph}: n={g.n} m={g.m} |S|={len(seeds)} k={k}")
    res = {"lsbm": lsbm_measure(binding, G, seeds_dev, k, eps, 0.1, delta, RNG_SEED)}
    log(f"  {res['lsbm']}")
    if args.sandwich:
        sec, out = timed_call(lambda: binding.gsbm(G, seeds_dev, k, eps=eps, beta=0.1, delta=delta,
                                                   rng_seed=RNG_SEED))
        res["gsbm"] = {"seconds": sec, "n_selected": out["n_selected"], **out["info"]}
        log(f"  gsbm {res['gsbm']}")
        sec, out = timed_call(lambda: binding.lhga(G, seeds_dev, k, beta=0.1, delta=delta, rng_seed=RNG_SEED))
        res["lhga"] = {"seconds": sec, "n_selected": int(len(out))}
        sec, out = timed_call(lambda: binding.sandimin(G, seeds_dev, k, eps=eps, beta=0.1, gamma=0.1, delta=delta,
                                                       rng_seed=RNG_SEED))
        res["sandimin"] = {"seconds": sec, "choice": out["choice"], "estimates": out["info"]["estimate"],
                           "eval_worlds": out["info"]["eval_worlds"], "n_blockers": out["info"]["n_blockers"]}
        log(f"  sandimin {res['sandimin']}")
    seed_rule = "top out-degree" if args.lsbm_top else "uniform"
    print(json.dumps({"metric": "LSBM (Algorithm 4) time to solution", "value": res["lsbm"]["seconds"],
                      "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
                      "dtype": "u32+int64",
                      "config": {"workload": f"{args.graph}: n={g.n} m={g.m}, |S|={len(seeds)} ({seed_rule}), "
                                             f"k={k}, eps={eps}, beta=0.1, gamma=0.1, delta=1/n"},
                      **res}), flush=True)


def solve_latency(args, binding, G, seeds_dev, k, theta, dev):
    """Full greedy solves (k rounds: round 0 from scratch, then incremental
    rounds): latency percentiles, the evaluations of each kind, and the
    roofline of the incremental-round kernel."""
    import torch
    out = (torch.zeros(max(k, 1), dtype=torch.int32, device=dev),
           torch.zeros(max(k, 1), dtype=torch.int64, device=dev),
           torch.zeros(k + 1, dtype=torch.int64, device=dev),
           torch.zeros(1, dtype=torch.int32, device=dev))
    # the warm-up solve takes the work tallies (every solve of this query does
    # the same work) and counts the round-update launches; no events
    binding.timing_enable(True)
    binding.timing_mask([6])
    binding.timing_sample(1 << 30)
    binding.timing_reset()
    binding.solve_device(G, seeds_dev, k, theta, RNG_SEED, out=out)
    torch.cuda.synchronize()
    work = [binding.timing_work(t) for t in range(6)]
    all6 = binding.timing_launches(6)
    # the timed solves: one launch in TIMED_EVERY of the round-update kernel is
    # bracketed, and no tallies are taken
    binding.timing_tallies(False)
    binding.timing_sample(TIMED_EVERY)
    binding.timing_reset()
    lat = []
    for i in range(args.solves):
        t1 = time.perf_counter()
        binding.solve_device(G, seeds_dev, k, theta, RNG_SEED, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
    log("solves: " + " ".join(f"{x:.1f}" for x in lat) + " ms")
    n6, ms6 = binding.timing_read(6)
    timed6 = binding.timing_launches(6)
    binding.timing_enable(False)
    binding.timing_tallies(True)
    binding.timing_mask(None)
    binding.timing_sample(1)
    n_sel = int(out[3].cpu()[0])
    spread = out[2].cpu().numpy()
    b6 = sum(work[t][2] for t in (3, 4, 5)) / max(all6, 1)
    avg6 = ms6 / max(n6, 1)
    return {
        "solve": {
            "k": k, "n_selected": n_sel, "solves": args.solves,
            "incremental_rounds": binding.last_solve_incremental() == 1,
            "p50_ms": percentile(lat, 50), "p99_ms": percentile(lat, 99),
            "spread_T0_over_theta": float(spread[0]) / theta,
            "spread_final_over_theta": float(spread[n_sel]) / theta,
            "world_evaluations_by_kind_per_solve": {
                nm: work[t][0] for nm, t in (
                    ("sampled_tier0", 0), ("sampled_tier1", 1), ("sampled_tier2", 2), ("replayed", 3),
                    ("label_updated", 4), ("label_updated_by_replay_workgroups", 5))},
            "round_update_roofline": {
                "achieved": b6 / (avg6 / 1e3) / 1e9 if ms6 > 0 else 0.0, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "algorithmic_bytes_per_launch": b6, "avg_launch_ms": avg6, "launches_per_solve": all6,
                "launches_in_timed_solves": timed6, "timed_launches": n6,
                "traffic": measured_traffic("round_update"),
            },
        },
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
    }


if __name__ == "__main__":
    main()
