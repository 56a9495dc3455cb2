"""Batches and the serving loop over a pool of device memory: several
resident graphs, admission by workspace size, re-admission after a
workspace shortfall found on the device.  Every result must equal the same
query solved alone (worlds are keyed by each query's own coin key)."""
import sys

import numpy as np
import pytest

from paper_2405_12871_amd import synth

pytestmark = pytest.mark.gpu

IMIN_ERR_WORKSPACE = 6


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


def _same(a, b):
    assert a.n_selected == b.n_selected
    np.testing.assert_array_equal(a.blockers, b.blockers)
    np.testing.assert_array_equal(a.gains, b.gains)
    np.testing.assert_array_equal(a.spread_totals, b.spread_totals)


def _graphs(B):
    gs = [synth.random_small_graph(800, 3200, seed=301, prob="wc"),
          synth.random_small_graph(2500, 9000, seed=302, prob="mixed"),
          synth.random_small_graph(400, 2400, seed=303, prob="uniform")]
    return gs, [B.Graph.from_synth(g) for g in gs]


def _queries(gs, Gs, count, seed):
    rs = np.random.default_rng(seed)
    qs = []
    for _ in range(count):
        j = int(rs.integers(0, len(gs)))
        seeds = rs.choice(gs[j].n, size=int(rs.integers(1, 12)), replace=False).astype(np.int32)
        qs.append((j, seeds, int(rs.integers(1, 9)), int(rs.choice([200, 600, 1200])), int(rs.integers(0, 1 << 40))))
    return qs


def test_batch_over_three_graphs(B, oracle_mod):
    gs, Gs = _graphs(B)
    qs = _queries(gs, Gs, 9, 5)
    _log("batch of 9 queries over 3 graphs")
    res = B.solve_many(Gs[0], [(Gs[j], s, k, th, r) for j, s, k, th, r in qs], n_streams=3)
    for (j, s, k, th, r), got in zip(qs, res):
        want = oracle_mod.Query(gs[j], s).solve(k, th, r)
        assert got.n_selected == want["n_selected"]
        np.testing.assert_array_equal(got.blockers, want["blockers"])
        np.testing.assert_array_equal(got.spread_totals, want["spread_totals"])


def test_server_over_three_graphs_under_memory_pressure(B):
    """A pool barely larger than the largest query's workspace holds one
    query at a time: the rest wait for memory, and every result still equals
    the query solved alone.  A query larger than the whole pool is refused."""
    gs, Gs = _graphs(B)
    qs = _queries(gs, Gs, 10, 6)
    alone = [B.solve(Gs[j], s, k, th, r) for j, s, k, th, r in qs]
    need = max(B.workspace_size(Gs[j], len(s), k, th) for j, s, k, th, r in qs)
    _log(f"server with a {need * 3 // 2} byte pool")
    srv = B.Server(Gs[0], n_streams=3, hbm_budget=need * 3 // 2)
    try:
        owner = {srv.submit(s, k, th, r, graph=Gs[j]): i for i, (j, s, k, th, r) in enumerate(qs)}
        big = srv.submit(np.array([1, 2], np.int32), 3, 1 << 22, 0, graph=Gs[1])
        got = {}
        for _ in range(len(qs) + 1):
            t, res = srv.next()
            if t == big:
                assert isinstance(res, B.IminError) and res.status == IMIN_ERR_WORKSPACE
            else:
                got[owner[t]] = res
    finally:
        srv.close()
    assert sorted(got) == list(range(len(qs)))
    for i, a in enumerate(alone):
        _same(got[i], a)


def test_server_readmits_after_a_device_side_shortfall(B, oracle_mod, monkeypatch):
    """Worlds that all start in the large LDS tier overflow the bump region
    of a workspace sized before any record: the server sees
    IMIN_ERR_WORKSPACE in the query's device status, admits it again with
    the size the graph now records, and returns the oracle's selection."""
    monkeypatch.setenv("IMIN_START_TIER", "1")
    g = synth.random_small_graph(3000, 12000, seed=78, prob="uniform")
    G = B.Graph.from_synth(g)
    seeds = np.array([5, 17, 400, 999, 2100], np.int32)
    srv = B.Server(G, n_streams=2)
    try:
        srv.submit(seeds, 3, 5000, 4)
        _, res = srv.next()
    finally:
        srv.close()
    want = oracle_mod.Query(g, seeds).solve(3, 5000, 4)
    assert res.n_selected == want["n_selected"]
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])


def test_server_pool_too_small_for_incremental_rounds(B, oracle_mod, monkeypatch):
    """A pool that holds the query's plain-rounds workspace but not its
    incremental one: the server sizes the query with the plain layout
    instead of refusing it, and returns the oracle's selection."""
    g = synth.random_small_graph(3000, 12000, seed=79, prob="uniform")
    G = B.Graph.from_synth(g)
    seeds = np.array([3, 41, 700, 1500], np.int32)
    k, theta = 4, 4000
    # the same query alone first: the graph then records what its worlds
    # need beyond tier 0, and both layouts are sized for it
    alone = B.solve(G, seeds, k, theta, 8)
    inc = B.workspace_size(G, len(seeds), k, theta)
    monkeypatch.setenv("IMIN_INCREMENTAL", "0")
    plain = B.workspace_size(G, len(seeds), k, theta)
    monkeypatch.delenv("IMIN_INCREMENTAL")
    _log(f"workspace: incremental {inc} bytes, plain {plain} bytes")
    assert plain + 4096 < inc
    srv = B.Server(G, n_streams=1, hbm_budget=(plain + 256 + inc) // 2)
    try:
        srv.submit(seeds, k, theta, 8)
        _, res = srv.next()
    finally:
        srv.close()
    assert not isinstance(res, B.IminError), res
    _same(res, alone)
    want = oracle_mod.Query(g, seeds).solve(k, theta, 8)
    assert res.n_selected == want["n_selected"]
    np.testing.assert_array_equal(res.blockers, want["blockers"])
    np.testing.assert_array_equal(res.gains, want["gains"])
    np.testing.assert_array_equal(res.spread_totals, want["spread_totals"])
