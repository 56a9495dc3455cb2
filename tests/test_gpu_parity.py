"""Parity of the HIP path with the CPU oracle, through the C ABI.

Integer results must be identical: per-world reached-set sizes and node-id
sums, per-node gains summed over worlds, totals, blocker sequences, gains and
spread totals of the greedy rounds.
"""
import os
import sys

import numpy as np
import pytest

from paper_2405_12871_amd import synth

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2405_12871_amd import binding
    binding.load()
    return binding


def _eval_both(B, oracle_mod, g, seeds, w0, nw, rng_seed, blocked=()):
    _log(f"evaluate {g.name} n={g.n} m={g.m} seeds={len(seeds)} worlds=[{w0},{w0 + nw}) blocked={len(blocked)}")
    G = B.Graph.from_synth(g)
    gain, total, ws, wsum = B.evaluate(G, seeds, w0, nw, rng_seed, blocked=blocked, per_world=True)
    q = oracle_mod.Query(g, seeds)
    ogain, ototal, ows, owsum = q.eval(rng_seed, w0, nw, blocked=blocked, per_world=True)
    return (gain, total, ws, wsum), (ogain, ototal, ows, owsum)


def _assert_same(got, want):
    gain, total, ws, wsum = got
    ogain, ototal, ows, owsum = want
    np.testing.assert_array_equal(ws, ows)
    np.testing.assert_array_equal(wsum, owsum)
    np.testing.assert_array_equal(gain, ogain)
    assert total == ototal


@pytest.mark.parametrize("case", range(10))
def test_evaluate_random_graphs(B, oracle_mod, case):
    rng = np.random.default_rng(case)
    n = int(rng.integers(3, 300))
    m = int(rng.integers(1, 8 * n))
    g = synth.random_small_graph(n, m, seed=3000 + case, prob=["mixed", "uniform", "wc"][case % 3],
                                 allow_multi=bool(case % 2))
    ns = int(rng.integers(1, max(2, n // 5)))
    seeds = rng.choice(n, ns, replace=False).astype(np.int32)
    others = np.setdiff1d(np.arange(n), seeds)
    blocked = rng.choice(others, min(len(others), int(rng.integers(0, 5))), replace=False).tolist()
    got, want = _eval_both(B, oracle_mod, g, seeds, int(rng.integers(0, 1000)), 777, 40 + case, blocked)
    _assert_same(got, want)


@pytest.mark.parametrize("case", range(6))
def test_level0_drawn_ahead_equals_inline(B, oracle_mod, monkeypatch, case):
    """Level 0 drawn ahead as bits (the default) and drawn inline by the world
    kernels give the oracle's worlds: rows that start and end inside a slot
    group, p = 1 and p = 0 slots, seeds next to seeds, self-loops and
    multi-edges, blocked nodes, and seeds whose rows span many groups."""
    rng = np.random.default_rng(700 + case)
    n = int(rng.integers(20, 400))
    m = int(rng.integers(n, 10 * n))
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    # a few hub seeds with long rows, and edges between seeds
    seeds = rng.choice(n, int(rng.integers(1, max(2, n // 6))), replace=False).astype(np.int32)
    hub = int(seeds[0])
    extra = rng.integers(0, n, 3 * n)
    src = np.concatenate([src, np.full(extra.size, hub), seeds[:-1], [hub]])
    dst = np.concatenate([dst, extra, seeds[1:], [hub]])
    p = rng.choice([0.0, 1.0, 0.5, 0.05, 0.3], src.size).astype(np.float32)
    g = synth.from_edges(n, src, dst, p, name=f"level0-{case}")
    others = np.setdiff1d(np.arange(n), seeds)
    blocked = rng.choice(others, min(len(others), int(rng.integers(0, 4))), replace=False).tolist()
    w0, nw, key = int(rng.integers(0, 10000)), int(rng.integers(100, 3000)), 900 + case
    want = oracle_mod.Query(g, seeds).eval(key, w0, nw, blocked=blocked, per_world=True)
    G = B.Graph.from_synth(g)
    for mode in ("1", "0"):
        monkeypatch.setenv("IMIN_LEVEL0_BITS", mode)
        _log(f"level 0 case {case} mode {mode}: n={n} m={g.m} seeds={len(seeds)} worlds={nw}")
        got = B.evaluate(G, seeds, w0, nw, key, blocked=blocked, per_world=True)
        _assert_same(got, want)


@pytest.mark.parametrize("case", range(3))
def test_query_thresholds_with_exclusions_in_lds_or_global(B, oracle_mod, monkeypatch, case):
    """The query's thresholds with its seeds and blockers folded in, built
    with the exclusion bits staged in LDS (the default where they fit) and
    read from global memory (the path of larger graphs): both give the
    oracle's worlds, with blocked heads next to seeds and rows ending inside a
    slot group."""
    rng = np.random.default_rng(720 + case)
    n = int(rng.integers(50, 3000))
    m = int(rng.integers(n, 8 * n))
    src = rng.integers(0, n, m)
    dst = rng.integers(0, n, m)
    p = rng.choice([1.0, 0.5, 0.2, 0.05], m).astype(np.float32)
    g = synth.from_edges(n, src, dst, p, name=f"qthr-{case}")
    seeds = rng.choice(n, int(rng.integers(1, max(2, n // 20))), replace=False).astype(np.int32)
    others = np.setdiff1d(np.arange(n), seeds)
    blocked = rng.choice(others, min(len(others), int(rng.integers(1, 30))), replace=False).tolist()
    w0, nw, key = int(rng.integers(0, 5000)), int(rng.integers(200, 2000)), 950 + case
    want = oracle_mod.Query(g, seeds).eval(key, w0, nw, blocked=blocked, per_world=True)
    G = B.Graph.from_synth(g)
    for mode in ("1", "0"):
        monkeypatch.setenv("IMIN_QUERY_THR_LDS", mode)
        _log(f"query thresholds case {case} lds={mode}: n={n} m={g.m} seeds={len(seeds)} worlds={nw}")
        got = B.evaluate(G, seeds, w0, nw, key, blocked=blocked, per_world=True)
        _assert_same(got, want)


def test_evaluate_small_workload(B, oracle_mod):
    g, seeds, k, theta = synth.workload("small")
    got, want = _eval_both(B, oracle_mod, g, seeds, 0, theta, 1)
    _assert_same(got, want)


def test_evaluate_medium_sample(B, oracle_mod):
    """Big worlds (about 24K reached nodes each): the workgroup-per-world path."""
    g, seeds, k, theta = synth.workload("medium")
    got, want = _eval_both(B, oracle_mod, g, seeds, 5000, 300, 7)
    _assert_same(got, want)


def test_evaluate_large_sample(B, oracle_mod):
    g, seeds, k, theta = synth.workload("large")
    got, want = _eval_both(B, oracle_mod, g, seeds, 123456, 4000, 11)
    _assert_same(got, want)


def test_world_range_shards_add_up(B):
    """Gains over [0, 1000) equal the sum over three disjoint sub-ranges."""
    g, seeds, _, _ = synth.workload("small")
    G = B.Graph.from_synth(g)
    full = B.evaluate(G, seeds, 0, 1000, 5)
    parts = [B.evaluate(G, seeds, a, b - a, 5) for a, b in ((0, 313), (313, 640), (640, 1000))]
    np.testing.assert_array_equal(full[0], sum(p[0] for p in parts))
    assert full[1] == sum(p[1] for p in parts)


def test_tile_beyond_2pow31_pairs(B):
    """The medium workload's from-scratch pass puts all 100,000 worlds in one
    tile: 2.35e9 (node, count) pairs, more than a 32-bit position can address.
    Its gains and total equal the sums over two half ranges (each below 2^31
    pairs)."""
    g, seeds, _, theta = synth.workload("medium")
    G = B.Graph.from_synth(g)
    _log("medium: one tile of all worlds")
    full_gain, full_total, ws, _ = B.evaluate(G, seeds, 0, theta, 11, per_world=True)
    assert int(ws.astype(np.int64).sum()) - theta * len(seeds) > 2 ** 31
    _log("medium: two half ranges")
    h = theta // 2
    a = B.evaluate(G, seeds, 0, h, 11)
    b = B.evaluate(G, seeds, h, theta - h, 11)
    np.testing.assert_array_equal(full_gain, a[0] + b[0])
    assert full_total == a[1] + b[1] == int(ws.astype(np.int64).sum())


def test_tiles(B, oracle_mod, monkeypatch):
    """Tiny tiles force the tile loop (a ragged last tile included); the
    retry of a tile whose scratch overflows is covered by the regrowth
    tests below."""
    g, seeds, _, _ = synth.workload("small")
    monkeypatch.setenv("IMIN_TILE_WORLDS", "97")
    got, want = _eval_both(B, oracle_mod, g, seeds, 10, 1001, 2)
    _assert_same(got, want)


def test_scratch_regrowth(B, oracle_mod, monkeypatch):
    """A bump region far too small for the worlds that outgrow the fixed
    slots is grown and the tile redone; the integers do not change."""
    monkeypatch.setenv("IMIN_BIG_SCRATCH", "64")
    monkeypatch.setenv("IMIN_START_TIER", "1")
    g, seeds, _, _ = synth.workload("small")
    got, want = _eval_both(B, oracle_mod, g, seeds, 0, 1500, 8)
    _assert_same(got, want)


def test_scratch_hint_from_earlier_calls(B, oracle_mod, monkeypatch):
    """The first solve on a graph grows a far too small bump region and
    redoes its tile; the second sizes it from what the first needed.  Both
    give the oracle's selection."""
    monkeypatch.setenv("IMIN_BIG_SCRATCH", "64")
    monkeypatch.setenv("IMIN_START_TIER", "1")
    g = synth.random_small_graph(1200, 3000, seed=92, prob="uniform")
    seeds = np.array([5, 17, 400, 999], np.int32)
    G = B.Graph.from_synth(g)
    want = oracle_mod.Query(g, seeds).solve(6, 500, 31)
    for call in range(2):
        _log(f"solve {call} on one graph with a tiny initial bump region")
        res = B.solve(G, seeds, 6, 500, 31)
        np.testing.assert_array_equal(res.blockers, want["blockers"])
        np.testing.assert_array_equal(res.gains, want["gains"])
        np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


@pytest.mark.parametrize("tier", ["0", "1", "2"])
def test_every_start_tier_gives_the_same_integers(B, oracle_mod, monkeypatch, tier):
    """Worlds first tried on the LDS tiers or directly on the HBM tier."""
    monkeypatch.setenv("IMIN_START_TIER", tier)
    g, seeds, _, _ = synth.workload("small")
    got, want = _eval_both(B, oracle_mod, g, seeds, 0, 2000, 3)
    _assert_same(got, want)
    g2 = synth.random_small_graph(200, 900, seed=12, prob="mixed", allow_multi=True)
    got, want = _eval_both(B, oracle_mod, g2, np.array([1, 7, 9], np.int32), 0, 500, 4, blocked=[3, 4])
    _assert_same(got, want)


@pytest.mark.parametrize("shape", ["path", "star", "grid", "star1000", "path100", "star70k", "dense", "mixed70k"])
def test_evaluate_deterministic_shapes(B, oracle_mod, shape):
    """p = 1 shapes that outgrow the LDS tiers: 1500- and 100-level paths,
    3000- and 1000-leaf stars, a 50x50 grid (many equal-level predecessors).
    Beyond the bounded HBM-tier slots (2^16 nodes, 2^16 extra edges): a
    70,000-leaf star, a 1,200-node graph with 100,000 live edges, and a
    graph whose worlds mix both sizes (seed 0 reaches a 70,000-leaf star
    through an edge of p = 0.5)."""
    if shape == "dense":
        rng = np.random.default_rng(9)
        n = 1200
        pairs = np.unique(rng.integers(0, n, size=(130_000, 2)), axis=0)
        pairs = pairs[pairs[:, 0] != pairs[:, 1]][:100_000]
        g = synth.from_edges(n, pairs[:, 0], pairs[:, 1], np.ones(len(pairs), np.float32), name=shape)
        got, want = _eval_both(B, oracle_mod, g, np.array([0], np.int32), 0, 3, 1)
        _assert_same(got, want)
        return
    if shape == "mixed70k":
        n = 70_002
        src = np.concatenate([[0], np.ones(n - 2, int)])
        dst = np.arange(1, n)
        p = np.concatenate([[0.5], np.ones(n - 2)]).astype(np.float32)
        g = synth.from_edges(n, src, dst, p, name=shape)
        got, want = _eval_both(B, oracle_mod, g, np.array([0], np.int32), 0, 40, 5)
        assert 0 < int((got[2] > 2).sum()) < 40  # both small and huge worlds
        _assert_same(got, want)
        return
    if shape in ("path", "path100"):
        n = 1500 if shape == "path" else 100
        src, dst = np.arange(n - 1), np.arange(1, n)
    elif shape in ("star", "star1000", "star70k"):
        n = {"star": 3001, "star1000": 1001, "star70k": 70_001}[shape]
        src, dst = np.zeros(n - 1, int), np.arange(1, n)
    else:
        s = 50
        n = s * s
        idx = np.arange(n).reshape(s, s)
        src = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
        dst = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    g = synth.from_edges(n, src, dst, np.ones(len(src), np.float32), name=shape)
    seeds = np.array([0], dtype=np.int32)
    got, want = _eval_both(B, oracle_mod, g, seeds, 0, 3, 1)
    _assert_same(got, want)


@pytest.mark.parametrize("case", range(6))
def test_solve_random_graphs(B, oracle_mod, case):
    rng = np.random.default_rng(100 + case)
    n = int(rng.integers(5, 400))
    g = synth.random_small_graph(n, int(rng.integers(n, 6 * n)), seed=4000 + case,
                                 prob=["mixed", "wc", "uniform"][case % 3])
    seeds = rng.choice(n, int(rng.integers(1, 6)), replace=False).astype(np.int32)
    k, theta = int(rng.integers(0, 12)), int(rng.integers(1, 900))
    _log(f"solve random case={case} n={n} k={k} theta={theta}")
    G = B.Graph.from_synth(g)
    res = B.solve(G, seeds, k, theta, 77 + case)
    want = oracle_mod.Query(g, seeds).solve(k, theta, 77 + case)
    assert res.n_selected == want["n_selected"]
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


@pytest.mark.parametrize("variant", ["plain", "store_overflow", "tier1", "tier2", "batch1", "batch7", "noreplay",
                                     "nolabelrule", "xscratch", "tiles", "lanes32", "lanes64"])
def test_solve_round_variants(B, oracle_mod, monkeypatch, variant):
    """Incremental rounds (default: worlds where no live edge leaves the new
    blocker's dominator subtree updated from their labels, other changed
    worlds replayed from their stored live edges), replay without the label
    rule, plain rounds, a resident store too small to
    hold round 0 (falls back to plain rounds), re-evaluation by sampling on
    every tier, regrowth of the extra-edge scratch, several tiles, other
    round batch sizes and other lane counts per world in the label rule all
    give the oracle's selection."""
    if variant == "plain":
        monkeypatch.setenv("IMIN_INCREMENTAL", "0")
    elif variant == "store_overflow":
        monkeypatch.setenv("IMIN_STORE_CAP", "5000")
    elif variant == "noreplay":
        monkeypatch.setenv("IMIN_REPLAY", "0")
    elif variant == "nolabelrule":
        monkeypatch.setenv("IMIN_LABEL_RULE", "0")
    elif variant.startswith("lanes"):
        monkeypatch.setenv("IMIN_RULE_LANES", variant[5:])
    elif variant == "xscratch":
        monkeypatch.setenv("IMIN_XBIG_SCRATCH", "16")
        monkeypatch.setenv("IMIN_BIG_SCRATCH", "64")
        monkeypatch.setenv("IMIN_START_TIER", "1")
    elif variant == "tiles":
        monkeypatch.setenv("IMIN_TILE_WORLDS", "97")
    elif variant.startswith("batch"):
        monkeypatch.setenv("IMIN_ROUND_BATCH", variant[5:])
    else:
        monkeypatch.setenv("IMIN_START_TIER", variant[-1])
    g = synth.random_small_graph(300, 1500, seed=77, prob="wc")
    seeds = np.array([3, 30, 111], np.int32)
    _log(f"solve variant {variant}")
    res = B.solve(B.Graph.from_synth(g), seeds, 15, 700, 5)
    want = oracle_mod.Query(g, seeds).solve(15, 700, 5)
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


@pytest.mark.parametrize("tiles", [False, True])
@pytest.mark.parametrize("bucket_log", ["1", "13"])
def test_index_bucket_widths(B, oracle_mod, monkeypatch, bucket_log, tiles):
    """The node index (and, with one tile, the round-0 gains computed with
    it) built with buckets of 2 node ids (2500 buckets) or of 8192 ids (one
    bucket counted in three slices of at most 2048 nodes), from one tile of
    worlds or from several, gives the oracle's selection."""
    monkeypatch.setenv("IMIN_INDEX_BUCKET_LOG", bucket_log)
    if tiles:
        monkeypatch.setenv("IMIN_TILE_WORLDS", "211")
    g = synth.random_small_graph(5000, 20000, seed=123, prob="wc")
    seeds = np.array([7, 1234, 4999], np.int32)
    _log(f"solve with index buckets of 2^{bucket_log} ids, tiles={tiles}")
    res = B.solve(B.Graph.from_synth(g), seeds, 10, 600, 9)
    want = oracle_mod.Query(g, seeds).solve(10, 600, 9)
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


@pytest.mark.parametrize("case", ["uniform", "multi", "binary"])
def test_solve_replay_mixed_world_sizes(B, oracle_mod, case):
    """Worlds from a few nodes to over a thousand: changed worlds are either
    replayed or, when too large for the replay store, sampled again; parallel
    edges and self-loops are kept in the multi case."""
    n = 1200
    if case == "multi":
        g = synth.random_small_graph(n, 3600, seed=91, prob="uniform", allow_multi=True)
    else:
        g = synth.random_small_graph(n, 3000, seed=92, prob=case)
    seeds = np.array([5, 17, 400, 999], np.int32)
    _log(f"solve mixed world sizes {case}")
    res = B.solve(B.Graph.from_synth(g), seeds, 12, 600, 31)
    want = oracle_mod.Query(g, seeds).solve(12, 600, 31)
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


def test_solve_worlds_beyond_the_replays(B, oracle_mod):
    """Worlds of 3 to about 2,400 reached nodes: changed worlds are replayed
    by the round-update workgroups (up to 512 entries) or by the wide replay
    (up to 2,048), and sampled again beyond that; the selection is the
    oracle's."""
    g = synth.random_small_graph(5000, 13000, seed=93, prob="uniform")
    seeds = np.random.default_rng(1).choice(5000, size=6, replace=False).astype(np.int32)
    G = B.Graph.from_synth(g)
    _log("solve with worlds beyond both replays")
    B.timing_reset()
    B.timing_enable(True)
    try:
        res = B.solve(G, seeds, 8, 240, 3)
        wide_launches = B.timing_launches(7)
    finally:
        B.timing_enable(False)
    assert wide_launches > 0
    want = oracle_mod.Query(g, seeds).solve(8, 240, 3)
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


def test_solve_small_workload(B, oracle_mod):
    g, seeds, k, theta = synth.workload("small")
    _log("solve small workload")
    res = B.solve(B.Graph.from_synth(g), seeds, k, theta, 1)
    want = oracle_mod.Query(g, seeds).solve(k, theta, 1)
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


@pytest.mark.parametrize("n_streams", [1, 3])
def test_solve_many_equals_each_query_alone(B, oracle_mod, n_streams):
    """Queries with different seed sets, budgets, world counts and coin keys
    solved side by side on several streams give each query's own oracle
    selection."""
    g = synth.random_small_graph(2000, 8000, seed=55, prob="wc")
    G = B.Graph.from_synth(g)
    rs = np.random.default_rng(7)
    queries = []
    for _ in range(5):
        seeds = rs.choice(2000, size=int(rs.integers(1, 20)), replace=False).astype(np.int32)
        queries.append((seeds, int(rs.integers(1, 12)), int(rs.choice([300, 700, 1500])), int(rs.integers(0, 1 << 40))))
    _log(f"solve_many, {len(queries)} queries on {n_streams} streams")
    res = B.solve_many(G, queries, n_streams=n_streams)
    for (seeds, k, theta, rng), r in zip(queries, res):
        want = oracle_mod.Query(g, seeds).solve(k, theta, rng)
        np.testing.assert_array_equal(r.blockers, want["blockers"])
        np.testing.assert_array_equal(r.gains, want["gains"])
        np.testing.assert_array_equal(r.spread_totals, want["spread_totals"])


def test_solve_many_reports_each_query(B, oracle_mod):
    """A query with a repeated seed fails with a data error of its own; the
    others are solved."""
    g = synth.random_small_graph(300, 1500, seed=77, prob="wc")
    G = B.Graph.from_synth(g)
    good = (np.array([3, 30, 111], np.int32), 6, 400, 5)
    bad = (np.array([3, 3], np.int32), 6, 400, 5)
    _log("solve_many with a failing query")
    res = B.solve_many(G, [good, bad, good], n_streams=2, raise_on_error=False)
    assert isinstance(res[1], B.IminError) and res[1].status == 2 and "query 1" in str(res[1])
    want = oracle_mod.Query(g, good[0]).solve(6, 400, 5)
    for r in (res[0], res[2]):
        np.testing.assert_array_equal(r.blockers, want["blockers"])
        np.testing.assert_array_equal(r.spread_totals, want["spread_totals"])
    with pytest.raises(B.IminError) as ei:
        B.solve_many(G, [good, bad], n_streams=2)
    assert ei.value.status == 2


def test_server_solves_queries_as_they_arrive(B, oracle_mod):
    """Queries submitted to a server on three streams, some while others
    run, each come back once with the oracle's selection; a failing query
    returns its own error; next() with nothing outstanding is refused."""
    g = synth.random_small_graph(2000, 8000, seed=56, prob="wc")
    G = B.Graph.from_synth(g)
    rs = np.random.default_rng(11)
    queries = []
    for _ in range(6):
        seeds = rs.choice(2000, size=int(rs.integers(1, 15)), replace=False).astype(np.int32)
        queries.append((seeds, int(rs.integers(1, 10)), int(rs.choice([300, 900])), int(rs.integers(0, 1 << 40))))
    _log("server: 6 queries on 3 streams")
    srv = B.Server(G, n_streams=3)
    try:
        tickets = {srv.submit(*q): i for i, q in enumerate(queries[:3])}
        got = {}
        t, r = srv.next()
        got[tickets.pop(t)] = r
        tickets.update({srv.submit(*q): i for i, q in enumerate(queries[3:], start=3)})
        bad = srv.submit(np.array([5, 5], np.int32), 3, 300, 1)
        while tickets or bad is not None:
            t, r = srv.next()
            if t == bad:
                assert isinstance(r, B.IminError) and r.status == 2
                bad = None
            else:
                got[tickets.pop(t)] = r
        with pytest.raises(B.IminError):
            srv.next()
    finally:
        srv.close()
    assert sorted(got) == list(range(6))
    for i, (seeds, k, theta, rng) in enumerate(queries):
        want = oracle_mod.Query(g, seeds).solve(k, theta, rng)
        np.testing.assert_array_equal(got[i].blockers, want["blockers"])
        np.testing.assert_array_equal(got[i].gains, want["gains"])
        np.testing.assert_array_equal(got[i].spread_totals, want["spread_totals"])


def test_batch_and_server_without_queries(B):
    """An empty batch returns no results; a server closed before any
    query was submitted stops its workers and returns; next() on it with
    nothing outstanding is refused."""
    g = synth.random_small_graph(200, 800, seed=58, prob="wc")
    G = B.Graph.from_synth(g)
    assert B.solve_many(G, [], n_streams=3) == []
    srv = B.Server(G, n_streams=2)
    with pytest.raises(B.IminError):
        srv.next()
    srv.close()


def test_server_with_concurrent_submitters(B):
    """Two threads submit while a third collects: every query comes back
    once, each equal to the same query solved alone."""
    import threading

    g = synth.random_small_graph(1500, 6000, seed=57, prob="wc")
    G = B.Graph.from_synth(g)
    rs = np.random.default_rng(13)
    queries = []
    for _ in range(16):
        seeds = rs.choice(1500, size=int(rs.integers(1, 12)), replace=False).astype(np.int32)
        queries.append((seeds, int(rs.integers(1, 8)), int(rs.choice([200, 500])), int(rs.integers(0, 1 << 40))))
    alone = [B.solve(G, *q) for q in queries]
    _log("server: 16 queries from two submitting threads")
    srv = B.Server(G, n_streams=4)
    owner, lock, sem, got, errors = {}, threading.Lock(), threading.Semaphore(0), {}, []

    def submit(part):
        try:
            for i in range(part, len(queries), 2):
                with lock:
                    owner[srv.submit(*queries[i])] = i
                sem.release()
        except Exception as e:  # reported below
            errors.append(e)
            sem.release()

    def collect():
        for _ in range(len(queries)):
            sem.acquire()
            if errors:
                return
            t, r = srv.next()
            with lock:
                got[owner.pop(t)] = r

    threads = [threading.Thread(target=submit, args=(0,)), threading.Thread(target=submit, args=(1,)),
               threading.Thread(target=collect)]
    try:
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=60)
    finally:
        srv.close()
    assert not errors
    assert sorted(got) == list(range(len(queries)))
    for i, r in got.items():
        np.testing.assert_array_equal(r.blockers, alone[i].blockers)
        np.testing.assert_array_equal(r.spread_totals, alone[i].spread_totals)


def test_block_cache_reuse(B, oracle_mod):
    """Scratch blocks handed back to the cache and reused by later calls
    (holding a previous call's contents), then freed and allocated afresh,
    give the same selections every time."""
    g1 = synth.random_small_graph(1500, 4500, seed=17, prob="wc")
    g2 = synth.random_small_graph(300, 900, seed=18, prob="uniform")
    s1 = np.array([3, 700], np.int32)
    s2 = np.array([9], np.int32)
    want1 = oracle_mod.Query(g1, s1).solve(8, 500, 5)
    want2 = oracle_mod.Query(g2, s2).solve(5, 200, 6)
    G1, G2 = B.Graph.from_synth(g1), B.Graph.from_synth(g2)
    for step, (G, s, k, th, rs, want) in enumerate([(G1, s1, 8, 500, 5, want1), (G2, s2, 5, 200, 6, want2),
                                                    (G1, s1, 8, 500, 5, want1), (None, None, 0, 0, 0, None),
                                                    (G1, s1, 8, 500, 5, want1)]):
        _log(f"block cache step {step}")
        if G is None:
            B.cache_release()
            continue
        res = B.solve(G, s, k, th, rs)
        np.testing.assert_array_equal(res.blockers, want["blockers"])
        np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


@pytest.mark.parametrize("prob", [1.0, 0.6])
@pytest.mark.parametrize("case", ["back_edge", "escape", "both"])
def test_label_rule_exit_cases(B, oracle_mod, case, prob):
    """Worlds built so that a blocker's dominator subtree has an edge back to
    one of its dominators (the label rule still holds), an edge out to a
    node it does not dominate (it must not: that node's dominator changes),
    or both; every round matches the oracle."""
    if case == "back_edge":
        src, dst = [0, 1, 2, 3, 1, 4, 5], [1, 2, 3, 1, 4, 5, 4]
        n = 6
    elif case == "escape":
        src, dst = [0, 0, 1, 3, 2, 4, 1, 5], [1, 2, 3, 4, 4, 6, 5, 6]
        n = 7
    else:
        src = [0, 0, 1, 2, 3, 3, 4, 5, 5, 6, 7, 2, 8]
        dst = [1, 2, 3, 4, 1, 5, 5, 6, 7, 4, 8, 8, 3]
        n = 9
    g = synth.from_edges(n, src, dst, [prob] * len(src))
    seeds = np.array([0], np.int32)
    _log(f"label rule exits {case} p={prob}")
    res = B.solve(B.Graph.from_synth(g), seeds, n - 1, 300, 13)
    want = oracle_mod.Query(g, seeds).solve(n - 1, 300, 13)
    assert res.n_selected == want["n_selected"]
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


def test_example1_and_submodularity_graph(B):
    """The paper's worked example and the submodularity-ratio construction."""
    g = synth.from_edges(7, [0, 0, 1, 2, 3, 3, 5], [1, 2, 3, 3, 5, 6, 6], [1.0] * 7)
    res = B.solve(B.Graph.from_synth(g), np.array([0], np.int32), 2, 13, 0)
    assert res.blockers.tolist() == [3, 1]
    assert res.spread_totals.tolist() == [6 * 13, 3 * 13, 2 * 13]
    n = 30
    g2 = synth.from_edges(n, [0, 0, 1, 2] + [3] * (n - 4), [1, 2, 3, 3] + list(range(4, n)), [1.0] * (n - 0))
    res2 = B.solve(B.Graph.from_synth(g2), np.array([0], np.int32), 10, 5, 0)
    assert res2.n_selected == 3
    assert res2.blockers.tolist() == [3, 1, 2]
    assert res2.spread_totals.tolist() == [n * 5, 15, 10, 5]


def test_edge_cases(B):
    import torch
    g = synth.random_small_graph(50, 200, seed=1, prob="uniform")
    G = B.Graph.from_synth(g)
    # every node a seed: no candidate, nothing selected
    res = B.solve(G, np.arange(50, dtype=np.int32), 5, 20, 0)
    assert res.n_selected == 0 and res.spread_totals.tolist() == [50 * 20]
    # k = 0 still reports T_0
    res0 = B.solve(G, np.array([3], np.int32), 0, 20, 0)
    assert res0.n_selected == 0 and len(res0.spread_totals) == 1
    # theta = 1
    B.solve(G, np.array([3], np.int32), 3, 1, 0)
    # a graph without edges
    e = synth.from_edges(4, [], [], [])
    r = B.solve(B.Graph.from_synth(e), np.array([1], np.int32), 2, 7, 0)
    assert r.n_selected == 0 and r.spread_totals.tolist() == [7]
    # data errors are reported, not crashed on
    with pytest.raises(B.IminError) as ei:
        B.solve(G, np.array([3, 3], np.int32), 2, 5, 0)
    assert ei.value.status == 2
    with pytest.raises(B.IminError):
        B.solve(G, np.array([60], np.int32), 2, 5, 0)
    with pytest.raises(B.IminError) as ei:
        B.evaluate(G, np.array([3], np.int32), 0, 5, 0, blocked=[3])
    assert ei.value.status == 2
    bad = synth.from_edges(3, [0, 1], [1, 2], [0.5, 1.5])
    with pytest.raises(B.IminError) as ei:
        B.Graph.from_synth(bad)
    assert ei.value.status == 2
    badc = synth.Graph(n=3, row_ptr=np.array([0, 1, 2, 2]), col=np.array([1, 7], np.int32),
                       p=np.array([0.5, 0.5], np.float32))
    with pytest.raises(B.IminError):
        B.Graph.from_synth(badc)
    torch.cuda.synchronize()


def _argmax_candidates(gain, seeds, blocked):
    """argmax of the oracle's gains over V minus (S + B), ties to the smaller id."""
    key = gain.astype(np.int64).copy()
    key[np.asarray(seeds, dtype=np.int64)] = -1
    if len(blocked):
        key[np.asarray(blocked, dtype=np.int64)] = -1
    u = int(np.argmax(key))  # first maximum: the smallest id
    return u, int(gain[u])


def _check_rounds_against_oracle(oracle_mod, g, seeds, theta, rng_seed, res, rounds):
    """At each round r: the oracle's from-scratch pass under B_r (the GPU's
    first r blockers) gives T_r, and, while r < n_selected, an argmax and a
    gain that must be the GPU's blockers[r] and gains[r]."""
    q = oracle_mod.Query(g, seeds)
    chunk = 10000
    for r in rounds:
        if r > res.n_selected:
            continue
        blocked = res.blockers[:r].tolist()
        # world ranges add up (an oracle pin); one progress line per range
        gain, total = np.zeros(g.n, np.int64), 0
        for w0 in range(0, theta, chunk):
            gi, ti = q.eval(rng_seed, w0, min(chunk, theta - w0), blocked=blocked)
            gain += gi
            total += ti
            _log(f"  oracle pass under the first {r} blockers: worlds {w0}..{min(theta, w0 + chunk)}")
        assert total == int(res.spread_totals[r]), (r, total, int(res.spread_totals[r]))
        if r < res.n_selected:
            u, gu = _argmax_candidates(gain, seeds, blocked)
            assert u == int(res.blockers[r]), (r, u, int(res.blockers[r]))
            assert gu == int(res.gains[r]), (r, gu, int(res.gains[r]))


def test_coin_threshold_boundary(B, oracle_mod):
    """A coin equal to the edge's threshold leaves the edge dead (the edge is
    kept with probability exactly p when p * 2^32 is an integer); one step of
    256 above it makes it live.  The coins and thresholds come from the
    oracle; the GPU draws its own."""
    from conftest import boundary_coins, dyadic_p
    seeds = np.array([0], np.int32)
    for rng_seed in (7, 0x0123456789ABCDEF):
        for w, c in boundary_coins(oracle_mod, rng_seed, 3):
            for cc, live in ((c, False), (c + 256, True), (c - 256, False)):
                g = synth.from_edges(2, [0], [1], [dyadic_p(cc)])
                _log(f"coin boundary seed={rng_seed:#x} world={w} coin={c:#x} thr={cc:#x}")
                G = B.Graph.from_synth(g)
                _, total, ws, _ = B.evaluate(G, seeds, w, 1, rng_seed, per_world=True)
                assert int(ws[0]) == (2 if live else 1) and total == int(ws[0]), (rng_seed, w, c, cc)
                G.destroy()


def test_large_workload_rounds(B, oracle_mod):
    """Full-size 1M-node workload (k = 500, theta = 2e5): the first rounds
    equal the oracle's greedy; at rounds spread over the whole solve the
    oracle's from-scratch pass under the GPU's blockers so far gives the same
    T_r, argmax and gain; every round satisfies the exact invariants."""
    g, seeds, k, theta = synth.workload("large")
    _log("solve large workload (full k, theta)")
    G = B.Graph.from_synth(g)
    res = B.solve(G, seeds, k, theta, 2024)
    T = res.spread_totals
    assert res.n_selected == k
    assert len(set(res.blockers.tolist())) == k
    assert not set(res.blockers.tolist()) & set(seeds.tolist())
    assert np.all(res.gains > 0)
    np.testing.assert_array_equal(T[1:], T[:-1] - res.gains)
    kpar = int(os.environ.get("IMIN_TEST_KPAR", "2"))
    _log(f"oracle solve large workload k={kpar}")
    want = oracle_mod.Query(g, seeds).solve(kpar, theta, 2024)
    np.testing.assert_array_equal(res.blockers[:kpar], want["blockers"])
    np.testing.assert_array_equal(res.gains[:kpar], want["gains"])
    np.testing.assert_array_equal(T[:kpar + 1], want["spread_totals"])
    _check_rounds_against_oracle(oracle_mod, g, seeds, theta, 2024, res, (2, 10, 50, 100, 250, 499, 500))


def test_medium_workload_every_round_reduced_theta(B, oracle_mod):
    """The medium workload's graph and seeds (worlds of about 24K nodes) with
    k = 100 at theta = 300: every round of the GPU's solve equals the
    oracle's greedy."""
    g, seeds, k, _ = synth.workload("medium")
    theta = 300
    _log(f"solve medium graph k={k} theta={theta}")
    res = B.solve(B.Graph.from_synth(g), seeds, k, theta, 31)
    _log("oracle solve")
    want = oracle_mod.Query(g, seeds).solve(k, theta, 31)
    assert res.n_selected == want["n_selected"]
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


@pytest.mark.timeout(1200)
def test_medium_workload_full_solve(B, oracle_mod, monkeypatch):
    """The full medium workload (k = 100, theta = 1e5).  Its round 0 stores
    about 2.35e9 entries, so the incremental rounds index store positions
    beyond 2^31: every round equals the solve with plain rounds (every world
    re-evaluated each round, no store), and at rounds 1 and 99
    (IMIN_TEST_MEDIUM_ROUNDS adds others) the oracle's from-scratch pass under
    the GPU's blockers so far gives the same T_r, argmax and gain."""
    g, seeds, k, theta = synth.workload("medium")
    G = B.Graph.from_synth(g)
    _log("solve medium workload (full k, theta), incremental rounds")
    res = B.solve(G, seeds, k, theta, 2024)
    assert B.last_solve_incremental() == 1
    T = res.spread_totals
    assert T[0] > 2**31  # entries of round 0's store, one per reached non-seed
    np.testing.assert_array_equal(T[1:res.n_selected + 1], T[:res.n_selected] - res.gains[:res.n_selected])
    _log("solve medium workload (full k, theta), plain rounds")
    monkeypatch.setenv("IMIN_INCREMENTAL", "0")
    plain = B.solve(G, seeds, k, theta, 2024)
    assert B.last_solve_incremental() == 0
    monkeypatch.delenv("IMIN_INCREMENTAL")
    assert plain.n_selected == res.n_selected
    np.testing.assert_array_equal(plain.blockers, res.blockers)
    np.testing.assert_array_equal(plain.gains, res.gains)
    np.testing.assert_array_equal(plain.spread_totals, res.spread_totals)
    rounds = [int(x) for x in os.environ.get("IMIN_TEST_MEDIUM_ROUNDS", "1,99").split(",")]
    _check_rounds_against_oracle(oracle_mod, g, seeds, theta, 2024, res, rounds)


def test_solve_worlds_beyond_the_hbm_tier_bounds(B, oracle_mod):
    """Worlds of 70,000 nodes (beyond the bounded HBM-tier slots) beside
    one-node worlds, in a full solve: with the block cache and with a
    workspace, every round equals the oracle's."""
    h = 35_000  # leaves per hub: a world reaching both hubs has 70,003 nodes
    n = 3 + 2 * h
    src = np.concatenate([[0, 0, 1], np.full(h, 1), np.full(h, 2)])
    dst = np.concatenate([[1, 2, 2], np.arange(3, 3 + h), np.arange(3 + h, n)])
    p = np.concatenate([[0.5, 0.5, 1.0], np.full(2 * h, 0.95)]).astype(np.float32)
    g = synth.from_edges(n, src, dst, p, name="hub70k")
    seeds = np.array([0], np.int32)
    want = oracle_mod.Query(g, seeds).solve(4, 30, 6)
    G = B.Graph.from_synth(g)
    for label, res in (("cache", B.solve(G, seeds, 4, 30, 6)), ("workspace", B.solve_ws(G, seeds, 4, 30, 6))):
        _log(f"hub70k solve ({label})")
        assert res.n_selected == want["n_selected"]
        np.testing.assert_array_equal(res.blockers, want["blockers"])
        np.testing.assert_array_equal(res.gains, want["gains"])
        np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


def test_solve_with_worlds_labelled_by_replays(B, oracle_mod, monkeypatch):
    """Every world starts in the HBM tier, which keeps no dominator-tree
    labels, so the small ones get their labels from replays during the
    rounds; a replay that labels a world must not let the label rule take
    the same world in the same round.  Weighted-cascade 1M-node graph, 207
    seeds, theta = 1e5, k = 37 (worlds of a few to thousands of nodes): the
    solve equals the one whose worlds start in the LDS tiers, and the
    oracle's from-scratch passes at rounds 0, 1 and 36."""
    g = synth.named_graph("wc1m")
    q = synth.query_mix(5, [g.n], 0xB0, (10, 500), (10, 200), (10_000, 100_000))
    _, seeds, k, theta, rng = q[4]
    G = B.Graph.from_synth(g)
    _log("solve with worlds starting in the LDS tiers")
    base = B.solve(G, seeds, k, theta, rng)
    monkeypatch.setenv("IMIN_START_TIER", "2")
    _log("solve with every world starting in the HBM tier")
    res = B.solve(G, seeds, k, theta, rng)
    assert res.n_selected == base.n_selected == k
    np.testing.assert_array_equal(res.blockers, base.blockers)
    np.testing.assert_array_equal(res.gains, base.gains)
    np.testing.assert_array_equal(res.spread_totals, base.spread_totals)
    _check_rounds_against_oracle(oracle_mod, g, seeds, theta, rng, res, (0, 1, 36))


def test_autotune_keeps_every_result(B, oracle_mod):
    """The launch-shape tuner times several tier-0 grid sizes (checking on the
    device that each gives the same gains) and keeps the fastest; passes and
    solves after it still equal the oracle."""
    g = synth.random_small_graph(3000, 15000, seed=404, prob="mixed")
    seeds = np.array([7, 700, 2900], np.int32)
    G = B.Graph.from_synth(g)
    pct, ms = B.autotune(G, seeds, 4000, 5)
    _log(f"autotune: grid0 {pct}% of residency, {ms:.3f} ms per pass")
    assert pct in (50, 75, 100, 150, 200, 300) and ms > 0
    q = oracle_mod.Query(g, seeds)
    gain, total = B.evaluate(G, seeds, 0, 4000, 5)
    want_gain, want_total = q.eval(5, 0, 4000)
    assert total == want_total
    np.testing.assert_array_equal(gain, want_gain)
    res = B.solve(G, seeds, 6, 4000, 5)
    want = q.solve(6, 4000, 5)
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])
    B.set_launch_shape(G, 0)
