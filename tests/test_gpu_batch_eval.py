"""Batched from-scratch passes (imin_evaluate_batch) through the C ABI.

Every query of a batch must get exactly the integers of the same pass run
alone (imin_evaluate) and of the oracle on the same worlds: the packed
tier-0 launch only changes which workgroup evaluates a world, never the world
or where its results go.  The batches mix queries that are packed with ones
that are not (larger than a tile), queries whose worlds overflow tier 0 into
the larger tiers, blocked sets, world ranges that start past 0, and batches
larger than one packed group.
"""
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


def _queries(g, rng, nq, max_w):
    qs = []
    for j in range(nq):
        ns = int(rng.integers(1, max(2, g.n // 20)))
        seeds = rng.choice(g.n, ns, replace=False).astype(np.int32)
        others = np.setdiff1d(np.arange(g.n), seeds)
        nb = int(rng.integers(0, 4))
        blocked = rng.choice(others, min(nb, len(others)), replace=False).astype(np.int32).tolist()
        qs.append({"seeds": seeds, "blocked": blocked, "w_begin": int(rng.integers(0, 5000)),
                   "w_count": int(rng.integers(1, max_w)), "rng_seed": int(rng.integers(0, 1 << 62))})
    return qs


def _check(B, oracle_mod, G, g, qs, with_oracle=True):
    got = B.evaluate_batch(G, qs, per_world=True)
    assert len(got) == len(qs)
    for j, (qd, r) in enumerate(zip(qs, got)):
        alone = B.evaluate(G, qd["seeds"], qd["w_begin"], qd["w_count"], qd["rng_seed"], blocked=qd["blocked"],
                           per_world=True)
        np.testing.assert_array_equal(r[0], alone[0], err_msg=f"query {j} gain")
        assert r[1] == alone[1], j
        np.testing.assert_array_equal(r[2], alone[2], err_msg=f"query {j} sizes")
        if with_oracle:
            og, ot, osz, _ = oracle_mod.Query(g, qd["seeds"]).eval(qd["rng_seed"], qd["w_begin"], qd["w_count"],
                                                                   blocked=qd["blocked"], per_world=True)
            np.testing.assert_array_equal(r[0], og, err_msg=f"query {j} gain vs oracle")
            assert r[1] == ot, j
            np.testing.assert_array_equal(r[2], osz, err_msg=f"query {j} sizes vs oracle")


@pytest.mark.parametrize("case", range(4))
def test_batch_equals_alone_and_oracle(B, oracle_mod, case):
    rng = np.random.default_rng(500 + case)
    n = int(rng.integers(50, 2000))
    g = synth.random_small_graph(n, int(rng.integers(2 * n, 8 * n)), seed=510 + case,
                                 prob=["mixed", "wc", "uniform", "mixed"][case], allow_multi=bool(case % 2))
    G = B.Graph.from_synth(g)
    qs = _queries(g, rng, int(rng.integers(2, 12)), 3000)
    _log(f"batch case {case}: n={g.n} m={g.m} queries={len(qs)}")
    _check(B, oracle_mod, G, g, qs)


def test_batch_with_unpacked_queries_and_groups(B, oracle_mod, monkeypatch):
    """Tiles of 700 worlds (queries above it are not packed) and groups of
    three queries per packed launch."""
    monkeypatch.setenv("IMIN_TILE_WORLDS", "700")
    monkeypatch.setenv("IMIN_PACK_QUERIES", "3")
    rng = np.random.default_rng(77)
    g = synth.random_small_graph(1500, 9000, seed=78, prob="mixed")
    G = B.Graph.from_synth(g)
    qs = _queries(g, rng, 8, 1500)
    _log("batch with unpacked queries, groups of 3: " + " ".join(str(q["w_count"]) for q in qs))
    assert any(q["w_count"] > 700 for q in qs) and any(q["w_count"] <= 700 for q in qs)
    _check(B, oracle_mod, G, g, qs)


def test_batch_worlds_overflowing_tier0(B, oracle_mod):
    """Dense probabilities: many worlds reach more nodes than tier 0 holds and
    go on to the larger tiers from the packed launch's lists."""
    g = synth.random_small_graph(4000, 24000, seed=91, prob="uniform")
    G = B.Graph.from_synth(g)
    rng = np.random.default_rng(92)
    qs = [{"seeds": rng.choice(4000, 3, replace=False).astype(np.int32), "blocked": [],
           "w_begin": 100 * j, "w_count": 300 + 50 * j, "rng_seed": 1000 + j} for j in range(5)]
    _log("batch with tier-0 overflow")
    # the handle is fresh (no hints from earlier passes), so every query starts
    # at tier 0 and is packed; the oracle shows that worlds overflow it
    sizes = oracle_mod.Query(g, qs[0]["seeds"]).eval(qs[0]["rng_seed"], qs[0]["w_begin"], qs[0]["w_count"],
                                                     per_world=True)[2]
    assert (sizes > 256).any(), "the case must overflow tier 0"
    _check(B, oracle_mod, G, g, qs)
    # the handle now knows its worlds need the HBM tier: a second batch starts
    # its queries there (unpacked, slots taken at set-up, the group sharing
    # the tier's budget)
    _log("second batch on the same handle")
    _check(B, oracle_mod, G, g, [dict(q, rng_seed=q["rng_seed"] + 50) for q in qs])


def test_batch_large_workload(B, oracle_mod):
    """Twenty queries on the 1M-node workload, 2,000 worlds each, with seed
    sets drawn like the workload's; four are checked against the oracle, all
    against their solo passes."""
    g, seeds0, _, _ = synth.workload("large")
    G = B.Graph.from_synth(g)
    rng = np.random.default_rng(13)
    qs = []
    for j in range(20):
        seeds = rng.choice(g.n, 200, replace=False).astype(np.int32) if j else seeds0
        qs.append({"seeds": seeds, "blocked": [], "w_begin": 2000 * j, "w_count": 2000, "rng_seed": 31 + j})
    _log("batch on the large workload")
    got = B.evaluate_batch(G, qs, per_world=True)
    for j in range(20):
        alone = B.evaluate(G, qs[j]["seeds"], qs[j]["w_begin"], 2000, qs[j]["rng_seed"], per_world=True)
        np.testing.assert_array_equal(got[j][0], alone[0])
        assert got[j][1] == alone[1]
        np.testing.assert_array_equal(got[j][2], alone[2])
    for j in (0, 7, 13, 19):
        og, ot = oracle_mod.Query(g, qs[j]["seeds"]).eval(qs[j]["rng_seed"], qs[j]["w_begin"], 2000)
        np.testing.assert_array_equal(got[j][0], og)
        assert got[j][1] == ot


def test_empty_batch(B):
    g = synth.random_small_graph(30, 60, seed=1, prob="wc")
    G = B.Graph.from_synth(g)
    assert B.evaluate_batch(G, []) == []


def test_batch_rejects_bad_data(B):
    """A query with a repeated seed or a seed out of range fails the batch with
    the data error, as imin_evaluate fails; a valid batch on the same handle
    still gives the solo results afterwards."""
    g = synth.random_small_graph(200, 800, seed=5, prob="wc")
    G = B.Graph.from_synth(g)
    good = {"seeds": np.array([1, 2], np.int32), "blocked": [], "w_begin": 0, "w_count": 300, "rng_seed": 9}
    for bad_seeds in ([3, 3], [4, 200]):
        bad = dict(good, seeds=np.array(bad_seeds, np.int32))
        _log(f"batch with bad seeds {bad_seeds}")
        with pytest.raises(B.IminError) as ei:
            B.evaluate_batch(G, [good, bad])
        assert ei.value.status == 2  # IMIN_ERR_DATA
    got = B.evaluate_batch(G, [good])
    alone = B.evaluate(G, good["seeds"], 0, 300, 9)
    np.testing.assert_array_equal(got[0][0], alone[0])
    assert got[0][1] == alone[1]
