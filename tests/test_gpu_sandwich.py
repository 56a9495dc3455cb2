"""Global Sampling, GSBM, LHGA and SandIMIN through the C ABI against the oracle.

Per-world sizes under blockers, V'_s, Max-Coverage and coverage over LRR sets,
and the three solvers and their best-of-three choice must give the oracle's
integers on the same samples; the bounds and spread estimates, computed from
those integers by the same formulas, agree to rounding.
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
    rng = np.random.default_rng(1900 + i)
    n = int(rng.integers(30, 700))
    g = synth.random_small_graph(n, int(rng.integers(2 * n, 6 * n)), seed=1910 + i,
                                 prob=["wc", "mixed", "uniform", "wc", "mixed", "wc"][i % 6], allow_multi=bool(i % 2))
    seeds = rng.choice(n, int(rng.integers(1, max(2, n // 12))), replace=False).astype(np.int32)
    k, theta = int(rng.integers(1, 12)), int(rng.integers(20, 5000))
    return g, seeds, k, theta


def _same_mc(got, want):
    assert got["n_selected"] == want["n_selected"]
    np.testing.assert_array_equal(got["blockers"], want["blockers"])
    np.testing.assert_array_equal(got["gains"], want["gains"])
    np.testing.assert_array_equal(got["cov"], want["cov"])
    np.testing.assert_array_equal(got["cov_upper"], want["cov_upper"])


@pytest.mark.parametrize("case", range(3))
def test_world_sizes_equal_oracle(B, oracle_mod, case):
    g, seeds, _, _ = _case(case)
    G = B.Graph.from_synth(g)
    q = oracle_mod.Query(g, seeds)
    cands = np.setdiff1d(np.arange(g.n), seeds)[:5]
    for blocked in ([], cands.tolist()):
        np.testing.assert_array_equal(B.world_sizes(G, seeds, 50, 3000, 8, blocked),
                                      q.world_sizes(8, 50, 3000, blocked=blocked))


@pytest.mark.parametrize("case", range(3))
def test_vprime_equals_oracle(B, case):
    from oracle import sandwich
    g, seeds, _, _ = _case(case)
    G = B.Graph.from_synth(g)
    np.testing.assert_array_equal(B.vprime(G, seeds), sandwich.vprime(g, seeds))


@pytest.mark.parametrize("case", range(6))
def test_lrr_max_coverage_equals_oracle(B, oracle_mod, case):
    from oracle import sandwich
    g, seeds, k, theta = _case(case)
    _log(f"lrr max coverage case {case}: n={g.n} m={g.m} |S|={len(seeds)} k={k} theta={theta}")
    G = B.Graph.from_synth(g)
    vp = sandwich.vprime(g, seeds)
    got = B.lrr_max_coverage(G, seeds, k, theta, 60 + case)
    _same_mc(got, oracle_mod.Query(g, seeds).lrr_max_coverage(vp, k, theta, 60 + case))


@pytest.mark.parametrize("tile", ["300", "4096"])
def test_lrr_max_coverage_tiles(B, oracle_mod, monkeypatch, tile):
    """Samples split into tiles (compacted into the store) and a small
    sampling budget (few slots) give the same integers."""
    from oracle import sandwich
    monkeypatch.setenv("IMIN_TILE_WORLDS", tile)
    monkeypatch.setenv("IMIN_LRR_BUDGET", str(3 * 8 * 4000))
    g = synth.random_small_graph(4000, 20000, seed=33, prob="wc")
    seeds = np.array([5, 900, 3100], np.int32)
    k, theta = 10, 6000
    _log(f"lrr max coverage tile {tile}")
    G = B.Graph.from_synth(g)
    got = B.lrr_max_coverage(G, seeds, k, theta, 17)
    _same_mc(got, oracle_mod.Query(g, seeds).lrr_max_coverage(sandwich.vprime(g, seeds), k, theta, 17))


def test_lrr_slots_kept_between_calls(B, oracle_mod, monkeypatch):
    """The handle keeps its sampling slots: later calls, other keys and other
    seed sets on it start from the stamps earlier calls left (three slots,
    so each takes thousands of samples) and still give the oracle's integers."""
    from oracle import sandwich
    monkeypatch.setenv("IMIN_LRR_BUDGET", str(3 * 8 * 3000))
    g = synth.random_small_graph(3000, 15000, seed=71, prob="wc")
    G = B.Graph.from_synth(g)
    for j, (seeds, key, theta) in enumerate([([4, 700], 3, 5000), ([4, 700], 3, 5000), ([4, 700], 9, 7000),
                                             ([11, 1200, 2500], 3, 4000)]):
        seeds = np.array(seeds, np.int32)
        _log(f"kept slots call {j}: |S|={len(seeds)} key={key} theta={theta}")
        q = oracle_mod.Query(g, seeds)
        vp = sandwich.vprime(g, seeds)
        want = q.lrr_max_coverage(vp, 8, theta, key)
        _same_mc(B.lrr_max_coverage(G, seeds, 8, theta, key), want)
        blk = want["blockers"][:3].astype(np.int32)
        assert B.lrr_coverage(G, seeds, blk, theta, key + 1) == q.lrr_coverage(vp, blk, theta, key + 1)


def test_lrr_concurrent_calls_on_one_handle(B, oracle_mod):
    """Two calls on one handle at once, each on its own stream: one borrows
    the kept slots, the other takes its own, and both give the oracle's
    integers."""
    import threading
    import torch
    from oracle import sandwich
    g = synth.random_small_graph(2500, 12000, seed=72, prob="wc")
    G = B.Graph.from_synth(g)
    seeds = np.array([3, 1000, 2000], np.int32)
    q = oracle_mod.Query(g, seeds)
    vp = sandwich.vprime(g, seeds)
    keys = (21, 22)
    want = {k: q.lrr_max_coverage(vp, 6, 20000, k) for k in keys}
    got, errs = {}, []

    def run(key):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                for _ in range(3):
                    got[key] = B.lrr_max_coverage(G, seeds, 6, 20000, key)
            s.synchronize()
        except Exception as e:  # reported below
            errs.append(e)

    _log("concurrent LRR calls on one handle")
    th = [threading.Thread(target=run, args=(k,)) for k in keys]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errs, errs
    for k in keys:
        _same_mc(got[k], want[k])


def test_lrr_large_cones(B, oracle_mod):
    """Dense uniform probabilities: cones of thousands of nodes."""
    from oracle import sandwich
    g = synth.random_small_graph(5000, 50000, seed=8, prob="uniform")
    seeds = np.array([1, 2], np.int32)
    k, theta = 6, 150
    _log("lrr max coverage with large cones")
    G = B.Graph.from_synth(g)
    got = B.lrr_max_coverage(G, seeds, k, theta, 5)
    _same_mc(got, oracle_mod.Query(g, seeds).lrr_max_coverage(sandwich.vprime(g, seeds), k, theta, 5))


@pytest.mark.parametrize("case", range(3))
def test_lrr_coverage_equals_oracle(B, oracle_mod, case):
    from oracle import sandwich
    g, seeds, _, theta = _case(10 + case)
    vp = sandwich.vprime(g, seeds)
    G = B.Graph.from_synth(g)
    q = oracle_mod.Query(g, seeds)
    rng = np.random.default_rng(case)
    for size in (0, 1, 6, 30):
        blk = rng.choice(vp, min(size, vp.size), replace=False).astype(np.int32) if vp.size else np.zeros(0, np.int32)
        assert B.lrr_coverage(G, seeds, blk, theta, 90 + case) == q.lrr_coverage(vp, blk, theta, 90 + case), size


def test_lrr_with_nothing_reachable(B):
    h = synth.from_edges(4, [1, 2], [2, 3], [0.5, 0.5])
    H = B.Graph.from_synth(h)
    got = B.lrr_max_coverage(H, np.array([0], np.int32), 3, 50, 2)
    assert got["n_selected"] == 0 and got["cov"].tolist() == [0] and got["cov_upper"].tolist() == [0]
    assert B.lrr_coverage(H, np.array([0], np.int32), np.array([1], np.int32), 50, 2) == 0


def _graph(case):
    g = synth.random_small_graph(500 + 150 * case, 3000 + 1200 * case, seed=70 + case,
                                 prob=["wc", "mixed", "wc"][case])
    seeds = np.array([3, 50, 120, 333][: case + 2], np.int32)
    return g, seeds


def _close(a, b):
    return math.isclose(a, b, rel_tol=1e-12, abs_tol=1e-300)


@pytest.mark.parametrize("case", range(3))
def test_gsbm_equals_oracle(B, case):
    from oracle import sandwich
    g, seeds = _graph(case)
    k, eps = 3 + case, 0.3
    _log(f"gsbm case {case}: n={g.n} m={g.m} k={k}")
    G = B.Graph.from_synth(g)
    got = B.gsbm(G, seeds, k, eps=eps, rng_seed=21 + case)
    want = sandwich.gsbm(g, seeds, k, eps=eps, rng_seed=21 + case, sra_batch=1 << 14)
    info = got["info"]
    _log(f"  gpu info {info}")
    assert not want["returned_on"]
    np.testing.assert_array_equal(got["blockers"], want["blockers"])
    assert info["nvp"] == want["nvp"] and info["i_max"] == want["i_max"]
    assert info["opt_l"] == want["opt_l"]
    assert _close(info["theta_0"], want["theta_0"]) and _close(info["theta_max"], want["theta_max"])
    last = want["iterations"][-1]
    assert info["iterations"] == len(want["iterations"]) and info["theta"] == last["theta"]
    assert (info["cov1"], info["cov2"], info["cov_upper"]) == (last["cov1"], last["cov2"], last["cov_upper"])
    assert _close(info["sigma_l"], last["sigma_l"]) and _close(info["sigma_u"], last["sigma_u"])


@pytest.mark.parametrize("case", range(3))
def test_lhga_equals_oracle(B, case):
    from oracle import sandwich
    g, seeds = _graph(case)
    G = B.Graph.from_synth(g)
    for k in (2, 5):
        np.testing.assert_array_equal(B.lhga(G, seeds, k, rng_seed=5 + case),
                                      sandwich.lhga(g, seeds, k, rng_seed=5 + case, sra_batch=1 << 14))


@pytest.mark.parametrize("case", range(2))
def test_sandimin_equals_oracle(B, case):
    from oracle import sandwich
    g, seeds = _graph(case)
    k = 3 + case
    _log(f"sandimin case {case}")
    G = B.Graph.from_synth(g)
    got = B.sandimin(G, seeds, k, eps=0.3, rng_seed=2 + case)
    want = sandwich.sandimin(g, seeds, k, eps=0.3, rng_seed=2 + case, sra_batch=1 << 14)
    _log(f"  gpu {got['choice']} {got['info']['estimate']}")
    for name in ("B_L", "B_U", "B_R", "blockers"):
        np.testing.assert_array_equal(got[name], want[name], err_msg=name)
    assert got["choice"] == want["choice"]
    for i in range(3):
        assert got["info"]["estimate"][i] == want["estimates"][i][0]
        assert got["info"]["eval_worlds"][i] == want["estimates"][i][1]


def test_solvers_return_on_for_a_large_budget(B):
    g = synth.from_edges(8, [0, 0, 0, 1, 2], [1, 2, 3, 4, 5], [0.5, 0.5, 0.0, 0.5, 0.5])
    G = B.Graph.from_synth(g)
    s = np.array([0], np.int32)
    assert B.gsbm(G, s, 2, rng_seed=1)["blockers"].tolist() == [1, 2]
    assert B.lhga(G, s, 3, rng_seed=1).tolist() == [1, 2]
    res = B.sandimin(G, s, 2, rng_seed=1)
    assert res["blockers"].tolist() == [1, 2] and res["choice"] == "L"
