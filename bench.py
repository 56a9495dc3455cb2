#!/usr/bin/env python3
"""Benchmark of the IMIN estimator on one MI355X.

Workload (default ``large``): directed Chung-Lu power-law graph with 1,000,000
nodes and 10,000,000 edges (degree exponent 2.1), trivalency probabilities
{0.1, 0.01, 0.001}, |S| = 200 uniform seeds, k = 500 blockers, theta = 200,000
worlds.  One step is one full greedy solve (``imin_solve``): seed set-up,
k rounds of world sampling + BFS + dominator counts + gain reduction +
selection.  Inputs (graph handle, seeds, output buffers) are resident in HBM
before the timed region.

Printed: one JSON line.  ``value`` is live-edge world evaluations actually
performed per second over whole solves (round 0 evaluates theta worlds from
scratch; each later round re-evaluates the worlds the new blocker changes).
The line also carries the from-scratch round-0 rate, the solve latency
percentiles, the roofline of the world-evaluation kernel (HIP events on the
library's stream, over every launch of the run) and the CPU oracle's rate on
a bounded sample.

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
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "live-edge worlds/sec (sample+BFS+gain) at 1M-node graph; p50/p99 IMIN query latency"
HBM_PEAK_GBS = 8000.0
TIMED_EVERY = 8
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


def measured_traffic(kernel: str):
    """HBM bytes per launch of a world kernel from its committed FETCH_SIZE /
    WRITE_SIZE profile, or None when there is none or the kernel sources
    have changed since the counters were taken."""
    import hashlib
    try:
        text = open(os.path.join(ROOT, "profiles", f"large_{kernel}_traffic.md")).read()
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


def cpu_baseline(g, seeds, k, theta, budget_s):
    """The oracle as it stands, on a bounded sample of the same query: its own
    greedy solve (every round re-evaluates all theta worlds) cut to the first
    rounds, sized to about ``budget_s`` seconds of CPU work."""
    from oracle import oracle
    q = oracle.Query(g, seeds)
    threads = oracle.default_threads()
    # one round-0 pass to size the sample
    nw = max(64, min(theta, 2000))
    t0 = time.perf_counter()
    q.eval(RNG_SEED, 0, nw, threads=threads)
    per_world = (time.perf_counter() - t0) / nw
    per_round = per_world * theta
    if per_round * 2 > budget_s:
        # even one full round is too long: a round-0 pass over a prefix of the worlds
        nw2 = int(max(nw, min(theta, budget_s / max(per_world, 1e-9))))
        t0 = time.perf_counter()
        q.eval(RNG_SEED, 0, nw2, threads=threads)
        dt = time.perf_counter() - t0
        return {"value": nw2 / dt, "unit": "worlds/s", "cores": threads, "kind": "oracle",
                "sample": f"round-0 pass (no blockers) over worlds [0, {nw2}) of the same query; "
                          f"{dt:.1f} s on {threads} threads", "seconds": dt}, None
    k_cpu = int(max(1, min(k, budget_s / per_round - 1)))
    t0 = time.perf_counter()
    res = q.solve(k_cpu, theta, RNG_SEED, threads=threads)
    dt = time.perf_counter() - t0
    # plain rounds: every round evaluates theta worlds, plus a final reachability pass
    evals = theta * (res["n_selected"] + 1)
    return {"value": evals / dt, "unit": "worlds/s", "cores": threads, "kind": "oracle",
            "sample": f"greedy solve of the same query cut to k={k_cpu} of {k} rounds (theta={theta} worlds "
                      f"per round, dominator mode, {res['n_selected'] + 1} passes); {dt:.1f} s on {threads} threads",
            "seconds": dt}, res["blockers"]


def run_many(args, binding, G, n):
    """Batch throughput: the same mixed queries sequentially and side by side."""
    import numpy as np
    import torch

    rs = np.random.default_rng(0xB0)
    queries = []
    for _ in range(args.many):
        seeds = rs.choice(n, size=int(rs.integers(10, 501)), replace=False).astype(np.int32)
        queries.append((seeds, int(rs.integers(10, 201)), int(rs.choice([10_000, 100_000])),
                        int(rs.integers(0, 1 << 62))))
    log(f"{len(queries)} queries; warm-up")
    binding.solve_many(G, queries[:min(len(queries), 2 * args.streams)], n_streams=args.streams)
    torch.cuda.synchronize()
    runs = {}
    for label, streams in (("sequential", 1), ("side_by_side", args.streams)):
        t0 = time.perf_counter()
        res = binding.solve_many(G, queries, n_streams=streams)
        torch.cuda.synchronize()
        runs[label] = (time.perf_counter() - t0, res)
        log(f"{label}: {runs[label][0] * 1e3:.1f} ms on {streams} stream(s)")
    (t_seq, seq), (t_par, par) = runs["sequential"], runs["side_by_side"]
    same = all(np.array_equal(a.blockers, b.blockers) and np.array_equal(a.gains, b.gains) and
               np.array_equal(a.spread_totals, b.spread_totals) for a, b in zip(seq, par))
    print(json.dumps({
        "metric": "greedy IMIN queries/s, mixed batch on one graph",
        "value": len(queries) / t_par,
        "unit": "queries/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "dtype": "u32+int64",
        "config": {"workload": f"{args.workload} graph, {len(queries)} queries: |S|~U{{10..500}}, "
                               f"k~U{{10..200}}, theta in {{1e4, 1e5}}", "streams": args.streams},
        "sequential_queries_per_s": len(queries) / t_seq,
        "speedup_over_sequential": t_seq / t_par,
        "identical_to_sequential": bool(same),
        "blockers_selected": int(sum(r.n_selected for r in par)),
    }))


def run_serve(args, binding, G, n):
    """Latency under arrivals: the server against one-at-a-time service."""
    import threading

    import numpy as np
    import torch

    rs = np.random.default_rng(0x5E)
    queries = []
    for _ in range(args.serve):
        seeds = rs.choice(n, size=int(rs.integers(10, 1001)), replace=False).astype(np.int32)
        queries.append((seeds, int(rs.integers(10, 501)), 50_000, int(rs.integers(0, 1 << 62))))
    arrivals = np.cumsum(rs.exponential(1.0 / args.rate, size=len(queries)))
    # each query alone: its service time and its result
    log(f"{len(queries)} queries at {args.rate}/s; solving each alone")
    binding.solve_many(G, queries[:2], n_streams=1)
    alone, service = [], []
    for q in queries:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        alone.append(binding.solve_many(G, [q], n_streams=1)[0])
        service.append(time.perf_counter() - t0)
    # one queue, one query at a time
    free, seq_lat = 0.0, []
    for a, sv in zip(arrivals, service):
        free = max(free, a) + sv
        seq_lat.append(free - a)
    # the server, queries submitted at their arrival times
    log(f"serving on {args.streams} streams")
    srv = binding.Server(G, n_streams=args.streams)
    finish, results = {}, {}
    tickets = {}
    lock = threading.Lock()
    submitted = threading.Semaphore(0)  # next() only while a query is outstanding

    def collect():
        for _ in range(len(queries)):
            submitted.acquire()
            t, r = srv.next()
            now = time.perf_counter()
            with lock:
                i = tickets.pop(t)
            finish[i] = now
            results[i] = r

    waiter = threading.Thread(target=collect)
    start = time.perf_counter()
    for i, (q, a) in enumerate(zip(queries, arrivals)):
        delay = start + a - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        with lock:
            tickets[srv.submit(*q)] = i
        submitted.release()
        if i == 0:
            waiter.start()
    waiter.join()
    srv.close()
    lat = [finish[i] - (start + arrivals[i]) for i in range(len(queries))]
    same = all(not isinstance(results[i], Exception) and
               np.array_equal(results[i].blockers, alone[i].blockers) and
               np.array_equal(results[i].spread_totals, alone[i].spread_totals) for i in range(len(queries)))
    span = max(finish.values()) - start
    print(json.dumps({
        "metric": "greedy IMIN query latency under Poisson arrivals, p50/p99",
        "value": percentile(lat, 50) * 1e3,
        "unit": "ms (p50)",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic",
        "dtype": "u32+int64",
        "config": {"workload": f"{args.workload} graph, {len(queries)} queries at {args.rate}/s: "
                               f"|S|~U{{10..1000}}, k~U{{10..500}}, theta=5e4", "streams": args.streams},
        "p50_ms": percentile(lat, 50) * 1e3,
        "p99_ms": percentile(lat, 99) * 1e3,
        "throughput_queries_per_s": len(queries) / span,
        "one_at_a_time": {"p50_ms": percentile(seq_lat, 50) * 1e3, "p99_ms": percentile(seq_lat, 99) * 1e3,
                          "mean_service_ms": float(np.mean(service)) * 1e3},
        "identical_to_alone": bool(same),
    }))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="run a 256 MiB copy first (counter scaling)")
    ap.add_argument("--many", type=int, default=0, help="measure a batch of this many mixed queries instead")
    ap.add_argument("--streams", type=int, default=4, help="streams for --many and --serve")
    ap.add_argument("--serve", type=int, default=0, help="measure latency of this many arriving queries instead")
    ap.add_argument("--rate", type=float, default=200.0, help="arrivals per second for --serve")
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
    log(f"generating workload {args.workload}")
    t0 = time.perf_counter()
    g, seeds, k, theta = synth.workload(args.workload)
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

    if args.many > 0:
        run_many(args, binding, G, g.n)
        return
    if args.serve > 0:
        run_serve(args, binding, G, g.n)
        return

    if args.copy_probe:
        # a plain copy of known size, for scaling HBM byte counters
        a = torch.empty(64 << 20, dtype=torch.int32, device=dev).fill_(1)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # every library kernel launch of this process is timed with HIP events
    binding.timing_enable(True)
    binding.timing_reset()

    # from-scratch round-0 pass: exact R and E per world
    t0 = time.perf_counter()
    gain0, T0, wsize, wsum, wedges = binding.evaluate(G, seeds_dev, 0, theta, RNG_SEED, per_world=True,
                                                      edges=True)
    r0_wall = time.perf_counter() - t0
    r0 = {kid: binding.timing_read(kid) for kid in (0, 1, 2, 4)}
    r0_work = [binding.timing_work(t) for t in range(3)]
    R = wsize.astype(np.int64)
    E = wedges.astype(np.int64)
    ns = len(seeds)
    r0_world_ms = r0[0][1] + r0[4][1] + r0[1][1]
    r0_bytes = sum(w[2] for w in r0_work)
    log(f"round 0: T0={T0} Rbar={R.mean():.1f} Ebar={E.mean():.1f} world kernels {r0_world_ms:.3f} ms "
        f"(tier0 {r0[0][1]:.3f}, tier1 {r0[4][1]:.3f}, tier2 {r0[1][1]:.3f}), reduce {r0[2][1]:.3f} ms, "
        f"wall {r0_wall * 1e3:.1f} ms, {r0_bytes / r0_world_ms / 1e6:.0f} GB/s algorithmic")

    # solves: the warm-up solves time every kernel (per-kernel breakdown);
    # the timed solves bracket only the dominant world kernel with events
    out = (torch.zeros(max(k, 1), dtype=torch.int32, device=dev),
           torch.zeros(max(k, 1), dtype=torch.int64, device=dev),
           torch.zeros(k + 1, dtype=torch.int64, device=dev),
           torch.zeros(1, dtype=torch.int32, device=dev))
    kernels = (("world_tier0", 0), ("world_tier1", 4), ("world_tier2", 1), ("round_update", 6),
               ("reduce", 2), ("select", 3), ("search_without_replay", 5))
    kern = {}
    for i in range(max(args.warmup, 1)):
        binding.timing_reset()
        binding.solve_device(G, seeds_dev, k, theta, RNG_SEED, out=out)
        torch.cuda.synchronize()
        kern = {name: binding.timing_read(kid)[1] for name, kid in kernels}
        log(f"warmup {i} done")
    # the world kernel with the most time per solve
    # kernel -> (timer id, work tiers it reports)
    world_ids = {"world_tier0": (0, (0,)), "world_tier1": (4, (1,)), "world_tier2": (1, (2,)),
                 "round_update": (6, (3, 4, 5))}
    dom = max(world_ids, key=lambda nm: kern.get(nm, 0.0))
    dom_kid, dom_tiers = world_ids[dom]
    # events take time on the stream: one launch in TIMED_EVERY of the dominant
    # kernel is bracketed, spread evenly over every solve's rounds
    binding.timing_mask([dom_kid])
    binding.timing_sample(TIMED_EVERY)
    binding.timing_reset()
    lat = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        t1 = time.perf_counter()
        binding.solve_device(G, seeds_dev, k, theta, RNG_SEED, out=out)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t1) * 1e3)
        log(f"step {i}: {lat[-1]:.1f} ms")
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t_start
    work = [binding.timing_work(t) for t in range(6)]
    n_dom, ms_dom = binding.timing_read(dom_kid)
    all_dom = binding.timing_launches(dom_kid)
    binding.timing_enable(False)
    binding.timing_mask(None)
    binding.timing_sample(1)
    n_sel = int(out[3].cpu()[0])
    rounds = min(n_sel + 1, k) if k > 0 else 1
    ms_per_step = total_s * 1e3 / args.steps
    evals = sum(w[0] for w in work) / args.steps
    value = evals / (ms_per_step / 1e3)
    # roofline of the dominant world kernel over the timed solves: algorithmic
    # bytes per launch (all its launches) over its average timed duration
    bytes_dom = sum(work[t][2] for t in dom_tiers)
    bytes_per_launch = bytes_dom / max(all_dom, 1)
    avg_ms = ms_dom / max(n_dom, 1)
    achieved = bytes_per_launch / (avg_ms / 1e3) / 1e9 if ms_dom > 0 else 0.0

    spread = out[2].cpu().numpy()
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
                        f"|S|={ns}, k={k}, theta={theta}, one full greedy solve per step",
            "n": g.n, "m": g.m, "seeds": ns, "k": k, "theta": theta, "rng_seed": RNG_SEED,
            "graph_sha256": g.sha256()[:16],
        },
        "value_definition": "live-edge world evaluations (sample + BFS + dominator counts + gain) actually "
                            "performed per second over whole greedy solves: theta from-scratch worlds in "
                            "round 0 plus the worlds each later round re-evaluates",
        "world_evaluations_per_step": evals,
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "n_selected": n_sel,
        "ag_equivalent_worlds_per_s": theta * rounds / (ms_per_step / 1e3),
        "spread_T0_over_theta": float(spread[0]) / theta,
        "spread_final_over_theta": float(spread[n_sel]) / theta,
        "round0_worlds_per_s": theta / r0_wall,
        "round0_world_kernel_ms": r0_world_ms,
        "round0_algorithmic_GBps": r0_bytes / r0_world_ms / 1e6,
        "round0_tier0": {"launches": r0[0][0], "ms": r0[0][1], "algorithmic_bytes": r0_work[0][2],
                         "worlds": r0_work[0][0]},
        "graph_ingest_ms": ingest_ms,
        "Rbar": float(R.mean()),
        "Ebar": float(E.mean()),
        "kernel_ms_per_step": kern,
        "world_evaluations_by_kind_per_step": {
            nm: work[t][0] / args.steps for nm, t in (("sampled_tier0", 0), ("sampled_tier1", 1), ("sampled_tier2", 2),
                                                       ("replayed", 3), ("label_updated", 4),
                                                       ("label_updated_by_replay_workgroups", 5))},
        "roofline": {
            "bound": "hbm",
            "kernel": f"{dom} (the world kernel with the most time per solve), its launches in the timed solves "
                      f"(one in {TIMED_EVERY} bracketed with HIP events)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(dom) if args.workload == "large" else None,
            "traffic_unit": "HBM bytes per launch (scaled FETCH_SIZE + WRITE_SIZE, committed profile)",
            "launches": all_dom,
            "timed_launches": n_dom,
            "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": bytes_per_launch,
        },
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        cb, cpu_blockers = cpu_baseline(g, seeds, k, theta, args.cpu_seconds)
        if cpu_blockers is not None:
            # the oracle's blockers must be the first blockers of the GPU solve
            gpu_b = out[0].cpu().numpy()[:len(cpu_blockers)]
            cb["oracle_blockers_equal_gpu_prefix"] = bool(np.array_equal(gpu_b, cpu_blockers))
        res["cpu_baseline"] = cb
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
