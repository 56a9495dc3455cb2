"""Lower-bound coverage and LSBM through the C ABI against the oracle.

Max-Coverage (blockers, marginal coverages, Cov of every prefix and the
upper-bound terms), the coverage of a given set, reach counts and the whole of
Algorithm 4 must give the oracle's integers on the same worlds; the sigma
bounds, computed from those integers by the same formulas, agree to rounding.
"""
import math
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


def _case(i):
    rng = np.random.default_rng(900 + i)
    n = int(rng.integers(30, 600))
    g = synth.random_small_graph(n, int(rng.integers(2 * n, 6 * n)), seed=910 + i,
                                 prob=["mixed", "uniform", "wc", "wc", "mixed", "uniform"][i % 6],
                                 allow_multi=bool(i % 2))
    seeds = rng.choice(n, int(rng.integers(1, max(2, n // 10))), replace=False).astype(np.int32)
    k, theta = int(rng.integers(1, 15)), int(rng.integers(20, 3000))
    return g, seeds, k, theta


def _same_mc(got, want):
    assert got["n_selected"] == want["n_selected"]
    np.testing.assert_array_equal(got["blockers"], want["blockers"])
    np.testing.assert_array_equal(got["gains"], want["gains"])
    np.testing.assert_array_equal(got["cov"], want["cov"])
    np.testing.assert_array_equal(got["cov_upper"], want["cov_upper"])


def test_graph_export(B, oracle_mod):
    g = synth.random_small_graph(300, 1500, seed=4, prob="mixed")
    G = B.Graph.from_synth(g)
    row_ptr, col, thr = B.graph_export(G)
    np.testing.assert_array_equal(row_ptr, g.row_ptr)
    np.testing.assert_array_equal(col, g.col)
    np.testing.assert_array_equal(thr, oracle_mod.thresholds(g.p))


@pytest.mark.parametrize("case", range(8))
def test_max_coverage_equals_oracle(B, oracle_mod, case):
    g, seeds, k, theta = _case(case)
    _log(f"max coverage case {case}: n={g.n} m={g.m} |S|={len(seeds)} k={k} theta={theta}")
    G = B.Graph.from_synth(g)
    got = B.max_coverage(G, seeds, k, theta, 40 + case)
    _same_mc(got, oracle_mod.Query(g, seeds).max_coverage(k, theta, 40 + case))


@pytest.mark.parametrize("tier", ["1", "2"])
@pytest.mark.parametrize("tile", [None, "700"])
def test_max_coverage_tiers_and_tiles(B, oracle_mod, monkeypatch, tier, tile):
    """Every world starting in the large LDS tier or the HBM tier, and worlds
    split into tiles (compacted into the store) give the same integers."""
    monkeypatch.setenv("IMIN_START_TIER", tier)
    if tile:
        monkeypatch.setenv("IMIN_TILE_WORLDS", tile)
    g = synth.random_small_graph(2500, 10000, seed=31, prob="wc")
    seeds = np.array([3, 400, 1200, 2222], np.int32)
    k, theta = 12, 2000
    _log(f"max coverage tier {tier} tile {tile}")
    G = B.Graph.from_synth(g)
    got = B.max_coverage(G, seeds, k, theta, 9)
    _same_mc(got, oracle_mod.Query(g, seeds).max_coverage(k, theta, 9))


def test_max_coverage_worlds_beyond_the_lds_tiers(B, oracle_mod):
    """Worlds of thousands of nodes (dense weighted cascade) go to the HBM
    tiers by themselves; their stored dominator trees cover exactly."""
    g = synth.random_small_graph(6000, 60000, seed=8, prob="uniform")
    seeds = np.array([1, 2, 3], np.int32)
    k, theta = 8, 200
    _log("max coverage with large worlds")
    G = B.Graph.from_synth(g)
    got = B.max_coverage(G, seeds, k, theta, 5)
    _same_mc(got, oracle_mod.Query(g, seeds).max_coverage(k, theta, 5))


def test_max_coverage_edge_cases(B, oracle_mod):
    # Example 4's realization: v3 (3 per world), then v1 over v2 by id
    g = synth.from_edges(7, [0, 0, 1, 2, 3, 3, 5], [1, 2, 3, 3, 5, 6, 6], [1.0] * 7)
    G = B.Graph.from_synth(g)
    got = B.max_coverage(G, np.array([0], np.int32), 2, 9, 1)
    assert got["blockers"].tolist() == [3, 1]
    assert got["cov"].tolist() == [0, 27, 36] and got["cov_upper"].tolist() == [36, 45, 45]
    # k larger than the candidates that cover anything: stops at gain 0
    got = B.max_coverage(G, np.array([0], np.int32), 6, 5, 1)
    want = oracle_mod.Query(g, np.array([0], np.int32)).max_coverage(6, 5, 1)
    _same_mc(got, want)
    assert got["n_selected"] == 3  # v3, v1, v2; then v5 and v6 are covered and v4 is never reached
    # k = 0: the empty prefix only
    got = B.max_coverage(G, np.array([0], np.int32), 0, 5, 1)
    assert got["n_selected"] == 0 and got["cov"].tolist() == [0] and got["cov_upper"].tolist() == [0]
    # a seed whose worlds reach nothing
    h = synth.from_edges(4, [1, 2], [2, 3], [0.5, 0.5])
    H = B.Graph.from_synth(h)
    got = B.max_coverage(H, np.array([0], np.int32), 3, 50, 2)
    assert got["n_selected"] == 0 and got["cov_upper"].tolist() == [0]


@pytest.mark.parametrize("case", range(4))
def test_coverage_equals_oracle(B, oracle_mod, case):
    g, seeds, _, theta = _case(10 + case)
    rng = np.random.default_rng(case)
    cands = np.setdiff1d(np.arange(g.n), seeds)
    G = B.Graph.from_synth(g)
    q = oracle_mod.Query(g, seeds)
    for size in (0, 1, 5, 40):
        blk = rng.choice(cands, min(size, cands.size), replace=False).astype(np.int32)
        assert B.coverage(G, seeds, blk, theta, 70 + case) == q.coverage(blk, theta, 70 + case), size


def test_coverage_rejects_seeds(B):
    g = synth.random_small_graph(50, 200, seed=2, prob="uniform")
    G = B.Graph.from_synth(g)
    with pytest.raises(B.IminError) as ei:
        B.coverage(G, np.array([1, 2], np.int32), np.array([2], np.int32), 10, 0)
    assert ei.value.status == 2


@pytest.mark.parametrize("case", range(3))
def test_reach_counts_equal_oracle(B, oracle_mod, case):
    g, seeds, _, _ = _case(20 + case)
    G = B.Graph.from_synth(g)
    q = oracle_mod.Query(g, seeds)
    counts, sizes = B.reach_counts(G, seeds, 100 * case, 1500, 11, per_world=True)
    want = q.reach_counts(11, 100 * case, 1500)
    want[seeds] = 0
    np.testing.assert_array_equal(counts, want)
    np.testing.assert_array_equal(sizes, q.world_sizes(11, 100 * case, 1500))


def _same_lsbm(got, want):
    info = got["info"]
    assert bool(info["returned_on"]) == bool(want["returned_on"])
    assert info["on_size"] == want["on_size"]
    np.testing.assert_array_equal(got["blockers"], want["blockers"])
    if want["returned_on"]:
        return
    assert info["reach_bound"] == want["reach_bound"]
    assert info["sra_worlds"] == want["sra_worlds"]
    assert info["i_hat"] == want["i_hat"]
    assert info["opt_l"] == want["opt_l"]
    assert math.isclose(info["theta_max"], want["theta_max"], rel_tol=1e-12)
    assert math.isclose(info["theta_0"], want["theta_0"], rel_tol=1e-12)
    assert info["i_max"] == want["i_max"]
    last = want["iterations"][-1]
    assert info["iterations"] == len(want["iterations"])
    assert info["theta"] == last["theta"]
    assert (info["cov1"], info["cov2"], info["cov_upper"]) == (last["cov1"], last["cov2"], last["cov_upper"])
    assert math.isclose(info["sigma_l"], last["sigma_l"], rel_tol=1e-12, abs_tol=1e-300)
    assert math.isclose(info["sigma_u"], last["sigma_u"], rel_tol=1e-12)


@pytest.mark.parametrize("case", range(3))
def test_lsbm_equals_oracle(B, oracle_mod, case):
    from oracle import lsbm
    g = synth.random_small_graph(400 + 200 * case, 3000 + 1500 * case, seed=50 + case,
                                 prob=["wc", "mixed", "uniform"][case])
    seeds = np.array([5, 60, 222][: case + 1], np.int32)
    k, eps = 3 + case, [0.3, 0.2, 0.25][case]
    _log(f"lsbm case {case}: n={g.n} m={g.m} k={k} eps={eps}")
    G = B.Graph.from_synth(g)
    got = B.lsbm(G, seeds, k, eps=eps, beta=0.1, rng_seed=13 + case)
    want = lsbm.lsbm(g, seeds, k, eps=eps, beta=0.1, rng_seed=13 + case, sra_batch=1 << 14)
    _log(f"  gpu info {got['info']}")
    assert not want["returned_on"]  # the case exercises the sampling path
    _same_lsbm(got, want)


def test_lsbm_returns_on(B, oracle_mod):
    from oracle import lsbm
    g = synth.from_edges(8, [0, 0, 0, 1, 2], [1, 2, 3, 4, 5], [0.5, 0.5, 0.0, 0.5, 0.5])
    G = B.Graph.from_synth(g)
    got = B.lsbm(G, np.array([0], np.int32), 2, rng_seed=1)
    _same_lsbm(got, lsbm.lsbm(g, np.array([0], np.int32), 2, rng_seed=1))
    assert got["blockers"].tolist() == [1, 2]  # the edge to 3 can never be live


@pytest.mark.parametrize("workload,theta,k,rounds", [("large", 200000, 100, (0, 1, 37, 99, 100)),
                                                      ("medium", 2000, 30, (0, 1, 15, 29, 30))])
def test_max_coverage_at_full_graph_size(B, oracle_mod, workload, theta, k, rounds):
    """On the 1M-node trivalency graph (200 seeds) and the 100K-node weighted
    cascade graph (50 seeds): for sampled prefixes B_r of the GPU's selection,
    the oracle's marginal coverages given B_r reproduce Cov(B_r), the next pick
    (argmax, ties to the smaller id) and its gain, and the upper-bound term."""
    g, seeds, _, _ = synth.workload(workload)
    _log(f"max coverage at {workload}: n={g.n} theta={theta} k={k}")
    G = B.Graph.from_synth(g)
    got = B.max_coverage(G, seeds, k, theta, 3)
    assert got["n_selected"] == k
    q = oracle_mod.Query(g, seeds)
    for r in rounds:
        marg, cov = q.cover_marginals(got["blockers"][:r], theta, 3)
        _log(f"  prefix {r}: Cov {cov}")
        assert cov == got["cov"][r]
        assert cov + int(np.sort(marg)[::-1][:k].sum()) == got["cov_upper"][r]
        if r < k:
            assert int(np.argmax(marg)) == got["blockers"][r]
            assert int(marg.max()) == got["gains"][r]
