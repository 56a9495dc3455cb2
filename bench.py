#!/usr/bin/env python3
"""Benchmark of the IMIN estimator on one MI355X.

Workload (default ``large``): directed Chung-Lu power-law graph with 1,000,000
nodes and 10,000,000 edges (degree exponent 2.1), trivalency probabilities
{0.1, 0.01, 0.001}, |S| = 200 uniform seeds, k = 500 blockers, theta = 200,000
worlds.  One step is one full greedy solve (``imin_solve``): seed set-up,
k rounds of world sampling + BFS + dominator counts + gain reduction +
selection.  Inputs (graph handle, seeds, output buffers) are resident in HBM
before the timed region.

Printed: one JSON line.  ``value`` is live-edge world evaluations per second
over the whole solve (theta worlds per greedy round).  The line also carries
the from-scratch round-0 rate, the solve latency percentiles, the roofline of
the world-evaluation kernel and the CPU oracle's rate on a bounded sample.
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
RNG_SEED = 2024


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    i = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[i]


def cpu_baseline(g, seeds, theta, budget_s):
    """The oracle as it stands, on a bounded sample of the round-0 pass."""
    from oracle import oracle
    q = oracle.Query(g, seeds)
    threads = oracle.default_threads()
    nw = max(64, min(theta, 2000))
    t0 = time.perf_counter()
    q.eval(RNG_SEED, 0, nw, threads=threads)
    dt = time.perf_counter() - t0
    if dt < budget_s / 4 and nw < theta:
        nw2 = int(min(theta, max(nw, nw * budget_s / max(dt, 1e-3))))
        t0 = time.perf_counter()
        q.eval(RNG_SEED, 0, nw2, threads=threads)
        dt = time.perf_counter() - t0
        nw = nw2
    return {"value": nw / dt, "unit": "worlds/s", "cores": threads, "kind": "oracle",
            "sample": f"round-0 pass (no blockers) over worlds [0, {nw}) of the same query, "
                      f"{dt:.1f} s on {threads} threads",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["small", "medium", "large"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the estimator shards "
              f"by world range, see the design notes; no multi-GPU run is part of this build)",
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

    # from-scratch round-0 pass: roofline of the world kernel, exact R and E
    binding.timing_enable(True)
    binding.timing_reset()
    t0 = time.perf_counter()
    gain0, T0, wsize, wsum, wedges = binding.evaluate(G, seeds_dev, 0, theta, RNG_SEED, per_world=True,
                                                      edges=True)
    r0_wall = time.perf_counter() - t0
    n_small, ms_small = binding.timing_read(0)
    n_big, ms_big = binding.timing_read(1)
    n_red, ms_red = binding.timing_read(2)
    R = wsize.astype(np.int64)
    E = wedges.astype(np.int64)
    ns = len(seeds)
    bytes_total = int((8 * E + 8 * R + 8 * (R - ns) + 12).sum())
    world_ms = ms_small + ms_big
    log(f"round 0: T0={T0} Rbar={R.mean():.1f} Ebar={E.mean():.1f} world kernels {world_ms:.3f} ms "
        f"(small {ms_small:.3f} x{n_small}, big {ms_big:.3f} x{n_big}), reduce {ms_red:.3f} ms, wall {r0_wall*1e3:.1f} ms")

    # timed solves
    out = (torch.zeros(max(k, 1), dtype=torch.int32, device=dev),
           torch.zeros(max(k, 1), dtype=torch.int64, device=dev),
           torch.zeros(k + 1, dtype=torch.int64, device=dev),
           torch.zeros(1, dtype=torch.int32, device=dev))
    for i in range(args.warmup):
        binding.solve_device(G, seeds_dev, k, theta, RNG_SEED, out=out)
        torch.cuda.synchronize()
        log(f"warmup {i} done")
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
    n_sel = int(out[3].cpu()[0])
    rounds = min(n_sel + 1, k) if k > 0 else 1
    ms_per_step = total_s * 1e3 / args.steps
    value = theta * rounds / (ms_per_step / 1e3)
    ts_launch, ts_ms = binding.timing_read(0)
    tb_launch, tb_ms = binding.timing_read(1)
    tr_launch, tr_ms = binding.timing_read(2)
    tsel_launch, tsel_ms = binding.timing_read(3)
    binding.timing_enable(False)

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
        "p50_ms": percentile(lat, 50),
        "p99_ms": percentile(lat, 99),
        "n_selected": n_sel,
        "spread_T0_over_theta": float(spread[0]) / theta,
        "spread_final_over_theta": float(spread[n_sel]) / theta,
        "round0_worlds_per_s": theta / (r0_wall),
        "round0_world_kernel_ms": world_ms,
        "graph_ingest_ms": ingest_ms,
        "Rbar": float(R.mean()),
        "Ebar": float(E.mean()),
        "kernel_ms_per_step": {
            "world_small": ts_ms / args.steps, "world_big": tb_ms / args.steps,
            "reduce": tr_ms / args.steps, "select": tsel_ms / args.steps,
            "launches_world_small": ts_launch / args.steps,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_world_small (round-0 pass, one launch over theta worlds)",
            "achieved": bytes_total / (world_ms / 1e3) / 1e9,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": bytes_total / (world_ms / 1e3) / 1e9 / HBM_PEAK_GBS,
            "traffic": None,
            "algorithmic_bytes": bytes_total,
        },
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        res["cpu_baseline"] = cpu_baseline(g, seeds, theta, args.cpu_seconds)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
