"""Pins for the oracle's lower-bound coverage and LSBM (Sections 3.2, 4.1, 5.1).

Each test ties the oracle to something other than itself: the paper's worked
example of CP sets, the definition of a CP set as the nodes common to every
path (by blocking each node in turn), the exact lower bound over every world
(Lemma 4.2), a brute-force Max-Coverage written again in Python, an
exhaustive search for the sample optimum, the equations the bounds of
Lemma 5.3 solve, and closed forms of the stopping rule.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from paper_2405_12871_amd import synth

from conftest import GOLDEN


def _example1():
    with open(os.path.join(GOLDEN, "example1_realization.json")) as f:
        fx = json.load(f)
    src = [e[0] for e in fx["edges"]]
    dst = [e[1] for e in fx["edges"]]
    return fx, synth.from_edges(fx["n"], src, dst, [1.0] * len(src))


# ------------------------------------------------------ CP sets (Section 4.1)
def test_example4_cp_sets(oracle_mod):
    """Example 4: C(v1) = {v1}, C(v3) = {v3}, C(v6) = {v3, v6},
    C(v5) = {v3, v5}, C(v2) = {v2}; each set is built after its immediate
    dominator's (depth-first preorder)."""
    fx, g = _example1()
    q = oracle_mod.Query(g, np.array(fx["seeds"], dtype=np.int32))
    seq = q.cp_world(rng_seed=5, w=0)
    got = {v: set(c) for v, c in seq}
    want = {int(v): set(c) for v, c in fx["expected_cp_sets"].items()}
    assert got == want
    order = [v for v, _ in seq]
    for v, c in seq:
        assert c[-1] == v
        for u in c[:-1]:
            assert order.index(u) < order.index(v)


def _live_edges(g, rng_seed, w, oracle_mod):
    from oracle import exact_enum
    src, dst = g.edges()
    live = []
    for e in range(g.m):
        t = exact_enum.threshold(float(g.p[e]))
        if t == exact_enum.ALWAYS_LIVE or oracle_mod.coin(rng_seed, w, e) < t:
            live.append((int(src[e]), int(dst[e])))
    return live


def _reach(n, live, seeds, blocked):
    adj = [[] for _ in range(n)]
    for u, v in live:
        adj[u].append(v)
    seen = set(int(s) for s in seeds)
    stack = list(seen)
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if v not in blocked and v not in seen:
                seen.add(v)
                stack.append(v)
    return seen


def _cp_by_definition(n, live, seeds):
    """Definition 4.1 by brute force: v's CP set is v plus every non-seed u
    whose removal cuts every path from the seeds to v."""
    base = _reach(n, live, seeds, set())
    sset = set(int(s) for s in seeds)
    cps = {v: {v} for v in base if v not in sset}
    for u in base:
        if u in sset:
            continue
        cut = base - _reach(n, live, seeds, {u})
        for v in cut:
            if v != u:
                cps[v].add(u)
    return cps


@pytest.mark.parametrize("case", range(6))
def test_cp_sets_are_the_common_path_nodes(oracle_mod, case):
    rng = np.random.default_rng(40 + case)
    n = int(rng.integers(8, 40))
    g = synth.random_small_graph(n, int(rng.integers(n, 4 * n)), seed=60 + case,
                                 prob=["mixed", "uniform", "wc"][case % 3], allow_multi=bool(case % 2))
    seeds = rng.choice(n, int(rng.integers(1, 4)), replace=False).astype(np.int32)
    q = oracle_mod.Query(g, seeds)
    for w in range(12):
        got = {v: set(c) for v, c in q.cp_world(rng_seed=7, w=w)}
        want = _cp_by_definition(n, _live_edges(g, 7, w, oracle_mod), seeds)
        assert got == want, (case, w)


# ------------------------------------------- coverage is unbiased (Lemma 4.2)
def _tiny(idx):
    rng = np.random.default_rng(3000 + idx)
    n = int(rng.integers(5, 8))
    g = synth.random_small_graph(n, int(rng.integers(7, 11)), seed=3100 + idx, prob="uniform")
    seeds = np.array([0], dtype=np.int32) if idx % 2 else np.array([0, 1], dtype=np.int32)
    return g, seeds


@pytest.mark.parametrize("idx", range(4))
def test_coverage_estimates_the_exact_lower_bound(oracle_mod, idx):
    """Cov(B)/theta lies within 5 standard errors of D^L(B) computed exactly
    over all 2^m worlds from its definition (N_phi(v): the nodes lost when v
    alone is blocked)."""
    from oracle import exact_enum
    g, seeds = _tiny(idx)
    src, dst = g.edges()
    q = oracle_mod.Query(g, seeds)
    theta = 30000
    cands = [v for v in range(g.n) if v not in seeds.tolist()]
    for B in ([cands[0]], cands[:2], cands[-2:], cands):
        m1, m2 = exact_enum.expected_lower_bound(g.n, src, dst, g.p, seeds, B)
        var = float(m2 - m1 * m1)
        cov = q.coverage(np.array(B, np.int32), theta, rng_seed=21 + idx)
        assert abs(cov / theta - float(m1)) <= 5 * math.sqrt(max(var, 0.0) / theta) + 1e-12, B


def test_coverage_equals_the_per_world_definition(oracle_mod):
    """Per world, the number of reached non-seeds whose CP set meets B equals
    |union over v in B of N_phi(v)|, counted by blocking each v alone."""
    g = synth.random_small_graph(30, 90, seed=91, prob="mixed")
    seeds = np.array([2, 11], np.int32)
    q = oracle_mod.Query(g, seeds)
    B = [5, 17, 23, 29]
    theta = 40
    want = 0
    for w in range(theta):
        live = _live_edges(g, 13, w, oracle_mod)
        base = _reach(g.n, live, seeds, set())
        lost = set()
        for v in B:
            if v in base:
                lost |= base - _reach(g.n, live, seeds, {v})
        want += len(lost)
    assert q.coverage(np.array(B, np.int32), theta, rng_seed=13) == want


# ------------------------------------------------ Max-Coverage (Section 5.1)
def _brute_max_coverage(g, seeds, k, theta, rng_seed, oracle_mod):
    """The procedure of Algorithm 4 written out: CP sets by Definition 4.1,
    argmax of Cov(B + v) - Cov(B) over V minus S and B (ties to the smaller id),
    stop when the best marginal is 0; Cov^u terms by sorting the marginals."""
    sets = []
    for w in range(theta):
        cps = _cp_by_definition(g.n, _live_edges(g, rng_seed, w, oracle_mod), seeds)
        sets.extend(cps.values())

    def cov(B):
        return sum(1 for c in sets if c & B)

    sset = set(seeds.tolist())
    B, picks, gains, covs, cus = set(), [], [], [], []
    while True:
        base = cov(B)
        marg = {v: cov(B | {v}) - base for v in range(g.n) if v not in sset and v not in B}
        covs.append(base)
        cus.append(base + sum(sorted(marg.values(), reverse=True)[:k]))
        if len(picks) == k or not marg:
            break
        best = min(marg, key=lambda v: (-marg[v], v))
        if marg[best] == 0:
            break
        picks.append(best)
        gains.append(marg[best])
        B.add(best)
    return picks, gains, covs, cus, sets


@pytest.mark.parametrize("case", range(5))
def test_max_coverage_matches_brute_force(oracle_mod, case):
    rng = np.random.default_rng(80 + case)
    n = int(rng.integers(10, 30))
    g = synth.random_small_graph(n, int(rng.integers(2 * n, 5 * n)), seed=90 + case,
                                 prob=["mixed", "uniform", "wc"][case % 3])
    seeds = rng.choice(n, int(rng.integers(1, 3)), replace=False).astype(np.int32)
    k, theta = int(rng.integers(1, 6)), int(rng.integers(5, 40))
    q = oracle_mod.Query(g, seeds)
    res = q.max_coverage(k, theta, rng_seed=31 + case, threads=1 + case % 3)
    picks, gains, covs, cus, _ = _brute_max_coverage(g, seeds, k, theta, 31 + case, oracle_mod)
    assert res["blockers"].tolist() == picks
    assert res["gains"].tolist() == gains
    assert res["cov"].tolist() == covs
    assert res["cov_upper"].tolist() == cus


@pytest.mark.parametrize("case", range(3))
def test_upper_bound_holds_for_the_sample_optimum(oracle_mod, case):
    """min_i Cov^u_i bounds the best size-k coverage of the sample (found by
    trying every k-subset), and greedy reaches at least 1 - 1/e of it."""
    n = 12
    g = synth.random_small_graph(n, 40, seed=130 + case, prob="uniform")
    seeds = np.array([0], np.int32)
    k, theta = 3, 25
    q = oracle_mod.Query(g, seeds)
    res = q.max_coverage(k, theta, rng_seed=5)
    _, _, _, _, sets = _brute_max_coverage(g, seeds, k, theta, 5, oracle_mod)
    best = max(sum(1 for c in sets if c & set(B)) for B in itertools.combinations(range(1, n), k))
    assert best <= int(res["cov_upper"].min())
    assert res["cov"][-1] >= (1 - 1 / math.e) * best


def test_max_coverage_on_example4(oracle_mod):
    """On Example 4's realization every world is the same: v3 covers v3, v5
    and v6 (3 per world), then v1 and v2 tie at 1 and the smaller id wins."""
    fx, g = _example1()
    q = oracle_mod.Query(g, np.array(fx["seeds"], dtype=np.int32))
    theta = 9
    res = q.max_coverage(2, theta, rng_seed=1)
    assert res["blockers"].tolist() == [3, 1]
    assert res["gains"].tolist() == [3 * theta, theta]
    assert res["cov"].tolist() == [0, 3 * theta, 4 * theta]
    # top-2 marginals: {3, 1} at B_0, {1, 1} at B_1, {1} at B_2
    assert res["cov_upper"].tolist() == [4 * theta, 5 * theta, 5 * theta]


# ---------------------------------------------- bounds of Lemma 5.3 (Alg. 4)
@pytest.mark.parametrize("a", [3.0, 12.5, 40.0])
def test_sigma_lower_solves_its_tail_equation(a):
    """For x >= 5a/18, z = theta * sigma^L is the root below x of
    x - z = sqrt(2 a z + a^2/9) + a/3 (the lower tail of Lemma 5.1 set to
    exp(-a)); below 5a/18 the bound is not positive."""
    from oracle import lsbm
    theta = 1000
    for x in (5 * a / 18, a, 3 * a, 50 * a, 1e4):
        z = lsbm.sigma_lower(x, theta, 0.0, 1.0, a) * theta
        assert z <= x
        assert math.isclose(x - z, math.sqrt(2 * a * z + a * a / 9) + a / 3, rel_tol=1e-9, abs_tol=1e-9)
    for x in (0.0, a / 18, 5 * a / 18 * 0.99):
        assert lsbm.sigma_lower(x, theta, 0.0, 1.0, a) <= 1e-15  # 0 at x = 0, up to rounding


def test_sigma_lower_takes_the_worst_end_of_the_range():
    from oracle import lsbm
    a, theta, beta = 10.0, 500, 0.1
    big = 100.0  # (1 - beta) * cov / I >= 5a/18: increasing side, the low end
    assert lsbm.sigma_lower(big, theta, beta, 1.0, a) == lsbm.sigma_lower(big * (1 - beta), theta, 0.0, 1.0, a)
    small = 1.0  # (1 + beta) * cov / I <= 5a/18: decreasing side, the high end
    assert lsbm.sigma_lower(small, theta, beta, 1.0, a) == lsbm.sigma_lower(small * (1 + beta), theta, 0.0, 1.0, a)
    mid = 5 * a / 18  # the range straddles the minimum
    assert lsbm.sigma_lower(mid, theta, beta, 1.0, a) == 0.0


@pytest.mark.parametrize("a", [3.0, 40.0])
def test_sigma_upper_solves_its_tail_equation(a):
    """z = theta * sigma^U is the root above y of z - y = sqrt(2 a z)."""
    from oracle import lsbm
    theta = 700
    for y in (0.0, 1.0, a, 1e3, 1e6):
        z = lsbm.sigma_upper(y, theta, 0.0, 1.0, a) * theta
        assert z >= y
        assert math.isclose(z - y, math.sqrt(2 * a * z), rel_tol=1e-9, abs_tol=1e-9)


def test_theta_schedule_closed_forms():
    """theta_0 = theta_max (1 - beta) eps^2 OPT^L / I_hat reduces to
    2 ((1 - 1/e) sqrt(ln 12/delta) + sqrt((1 - 1/e)(ln C(n-|S|, k) + ln 12/delta)))^2,
    and ln C agrees with the gamma function."""
    from oracle import lsbm
    n, ns, k, eps, beta, delta = 100000, 10, 100, 0.2, 0.1, 1e-5
    assert math.isclose(lsbm.ln_binom(n - ns, k),
                        math.lgamma(n - ns + 1) - math.lgamma(k + 1) - math.lgamma(n - ns - k + 1), rel_tol=1e-9)
    c = 1 - 1 / math.e
    want0 = 2 * (c * math.sqrt(math.log(12 / delta)) +
                 math.sqrt(c * (lsbm.ln_binom(n - ns, k) + math.log(12 / delta)))) ** 2
    for i_hat, opt in ((350.0, 2.5), (10.0, 9.0), (1e5, 0.01)):
        tmax, t0, imax = lsbm.theta_schedule(n, ns, k, eps, beta, delta, i_hat, opt)
        assert math.isclose(t0, want0, rel_tol=1e-12)
        assert math.isclose(tmax / t0, i_hat / ((1 - beta) * eps * eps * opt), rel_tol=1e-12)
        assert imax == max(1, math.ceil(math.log2(tmax / t0)))


# -------------------------------------- stopping rule and OPT^L (Section 5.1)
def test_stopping_rule_on_a_constant_spread(oracle_mod):
    """Every probability 1: every world reaches the same b nodes, Z = 1, and the
    rule stops at N = ceil(Upsilon_1) with I_hat = b Upsilon_1 / N."""
    from oracle import lsbm
    g = synth.from_edges(6, [0, 0, 1, 2, 3], [1, 2, 3, 3, 4], [1.0] * 5)
    seeds = np.array([0], np.int32)
    b = lsbm.reach_bound(g, seeds)
    assert b == 5
    q = oracle_mod.Query(g, seeds)
    _, ups1 = lsbm.sra_constants(0.1, 1e-3)
    i_hat, N = lsbm.stopping_rule(q, 9, b, 0.1, 1e-3, batch=4096)
    assert N == math.ceil(ups1)
    assert i_hat == b * ups1 / N


@pytest.mark.parametrize("idx", range(3))
def test_stopping_rule_is_within_beta_of_the_exact_spread(oracle_mod, idx):
    from oracle import exact_enum, lsbm
    g, seeds = _tiny(idx)
    src, dst = g.edges()
    m1, _ = exact_enum.expected_spread(g.n, src, dst, g.p, seeds)
    q = oracle_mod.Query(g, seeds)
    beta = 0.05
    i_hat, _ = lsbm.stopping_rule(q, 77 + idx, lsbm.reach_bound(g, seeds), beta, 1e-4)
    assert abs(i_hat - float(m1)) <= beta * float(m1)


@pytest.mark.parametrize("idx", range(2))
def test_reach_frequencies_estimate_reach_probabilities(oracle_mod, idx):
    """counts[v]/N within 5 standard errors of Pr[s -> v], exact by enumeration."""
    from oracle import exact_enum
    g, seeds = _tiny(idx)
    src, dst = g.edges()
    q = oracle_mod.Query(g, seeds)
    N = 40000
    counts = q.reach_counts(3, 0, N)
    assert int(counts.sum()) == int(q.world_sizes(3, 0, N).sum())
    pr = [0] * g.n
    for p, edges, live in exact_enum.enumerate_worlds(g.n, src, dst, g.p):
        for v in exact_enum._reach(g.n, edges, live, seeds, set()):
            pr[v] += p
    for v in range(g.n):
        pv = float(pr[v])
        assert abs(counts[v] / N - pv) <= 5 * math.sqrt(pv * (1 - pv) / N) + 1e-12


def test_out_neighbours_and_reach_bound():
    from oracle import lsbm
    # 0 -> 1 (p 0.5), 0 -> 2 (p 0), 3 -> 0, 1 -> 4, 5 isolated; seeds {0, 3}
    g = synth.from_edges(6, [0, 0, 3, 1], [1, 2, 0, 4], [0.5, 0.0, 1.0, 0.2])
    seeds = np.array([0, 3], np.int32)
    assert lsbm.out_neighbours(g, seeds).tolist() == [1]
    assert lsbm.reach_bound(g, seeds) == 4  # 0, 3, 1, 4


def test_lsbm_returns_on_when_the_budget_covers_it(oracle_mod):
    from oracle import lsbm
    g = synth.from_edges(6, [0, 0, 1, 2], [1, 2, 3, 4], [0.5, 0.5, 0.5, 0.5])
    res = lsbm.lsbm(g, np.array([0], np.int32), k=2, rng_seed=1)
    assert res["returned_on"] and res["blockers"].tolist() == [1, 2]


def test_lsbm_end_to_end(oracle_mod):
    """Algorithm 4 on a small graph: pools double until the ratio test passes
    or i_max is reached, and the answer is Max-Coverage on the last C_1."""
    from oracle import lsbm
    g = synth.random_small_graph(300, 1500, seed=17, prob="wc")
    seeds = np.array([3, 50, 120], np.int32)
    k = 5
    res = lsbm.lsbm(g, seeds, k=k, eps=0.3, beta=0.1, rng_seed=4, sra_batch=1 << 12)
    its = res["iterations"]
    assert 1 <= len(its) <= res["i_max"]
    assert its[0]["theta"] == math.ceil(res["theta_0"])
    for a, b in zip(its, its[1:]):
        assert b["theta"] == 2 * a["theta"]
        assert a["sigma_l"] / a["sigma_u"] < 1 - 1 / math.e - 0.3
    last = its[-1]
    assert last["sigma_l"] / last["sigma_u"] >= 1 - 1 / math.e - 0.3 or len(its) == res["i_max"]
    q = oracle_mod.Query(g, seeds)
    k1, k2, _ = lsbm.pool_keys(4)
    mc = q.max_coverage(k, last["theta"], k1)
    assert res["blockers"].tolist() == mc["blockers"].tolist()
    assert last["cov2"] == q.coverage(mc["blockers"], last["theta"], k2)
    assert last["cov1"] <= last["cov_upper"]


def test_cover_marginals_match_the_greedy(oracle_mod):
    """Marginals given each greedy prefix: their argmax (ties to the smaller id)
    is the next pick, their maximum its gain, and the k largest plus Cov(B_r)
    the upper-bound term; Cov(B_r) itself matches."""
    g = synth.random_small_graph(200, 900, seed=12, prob="wc")
    seeds = np.array([1, 77], np.int32)
    q = oracle_mod.Query(g, seeds)
    k, theta = 6, 300
    res = q.max_coverage(k, theta, rng_seed=8)
    for r in range(res["n_selected"] + 1):
        marg, cov = q.cover_marginals(res["blockers"][:r], theta, rng_seed=8)
        assert cov == res["cov"][r]
        assert cov + int(np.sort(marg)[::-1][:k].sum()) == res["cov_upper"][r]
        if r < res["n_selected"]:
            assert int(np.argmax(marg)) == res["blockers"][r]
            assert int(marg.max()) == res["gains"][r]
