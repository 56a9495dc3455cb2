"""Pins for the oracle's Global Sampling, GSBM, LHGA and SandIMIN
(Sections 3.1, 3.3, 4.2, 5.2, 5.3).

LRR sets are checked against their definition written again in Python, the
upper-bound estimator against the exact D^U over every world (Lemma 4.4),
Max-Coverage over LRR sets against a brute-force greedy, the GSBM settings
against their closed forms and the equations their bounds solve, LHGA on a
graph whose scores are known, and SandIMIN's spread estimates against the
exact spread.
"""
import itertools
import math

import numpy as np
import pytest

from paper_2405_12871_amd import synth

from test_oracle_lsbm import _live_edges, _reach


def _lrr_by_definition(n, live, seeds, v):
    """Nodes that reach v in phi^s (the reached non-seeds and the live edges
    among them); empty when v is not reached."""
    base = _reach(n, live, seeds, set())
    if v not in base:
        return []
    inside = base - set(int(s) for s in seeds)
    rev = {}
    for a, b in live:
        if a in inside and b in inside:
            rev.setdefault(b, []).append(a)
    seen = {v}
    stack = [v]
    while stack:
        x = stack.pop()
        for a in rev.get(x, ()):
            if a not in seen:
                seen.add(a)
                stack.append(a)
    return sorted(seen)


@pytest.mark.parametrize("case", range(5))
def test_lrr_sets_match_their_definition(oracle_mod, case):
    from oracle import sandwich
    rng = np.random.default_rng(70 + case)
    n = int(rng.integers(10, 50))
    g = synth.random_small_graph(n, int(rng.integers(2 * n, 5 * n)), seed=80 + case,
                                 prob=["mixed", "uniform", "wc"][case % 3], allow_multi=bool(case % 2))
    seeds = rng.choice(n, int(rng.integers(1, 4)), replace=False).astype(np.int32)
    vp = sandwich.vprime(g, seeds)
    q = oracle_mod.Query(g, seeds)
    key = 1000 + case
    for i in range(15):
        v = int(vp[oracle_mod.lrr_pick(key, i, len(vp))]) if len(vp) else -1
        want = _lrr_by_definition(n, _live_edges(g, key, i, oracle_mod), seeds, v) if len(vp) else []
        assert q.lrr_set(key, i, vp) == want, (case, i)


def test_lrr_pick_is_uniform(oracle_mod):
    M, N = 12, 24000
    counts = np.bincount([oracle_mod.lrr_pick(77, i, M) for i in range(N)], minlength=M)
    chi2 = float(((counts - N / M) ** 2 / (N / M)).sum())
    assert chi2 < 40.0  # 11 degrees of freedom; p < 1e-4 beyond this


def test_vprime_excludes_seeds_and_dead_edges():
    from oracle import sandwich
    # 0 -> 1 (p 0.5), 0 -> 2 (p 0), 1 -> 3, 3 -> 0 (a seed), 4 isolated
    g = synth.from_edges(5, [0, 0, 1, 3], [1, 2, 3, 0], [0.5, 0.0, 0.3, 1.0])
    assert sandwich.vprime(g, np.array([0], np.int32)).tolist() == [1, 3]


def _tiny(idx):
    rng = np.random.default_rng(4000 + idx)
    n = int(rng.integers(5, 8))
    g = synth.random_small_graph(n, int(rng.integers(7, 11)), seed=4100 + idx, prob="uniform")
    seeds = np.array([0], dtype=np.int32) if idx % 2 else np.array([0, 1], dtype=np.int32)
    return g, seeds


@pytest.mark.parametrize("idx", range(4))
def test_lrr_coverage_estimates_the_exact_upper_bound(oracle_mod, idx):
    """|V'_s| Cov(B) / theta lies within 5 standard errors of D^U(B), exact over
    all 2^m worlds (Lemma 4.4)."""
    from oracle import exact_enum, sandwich
    g, seeds = _tiny(idx)
    src, dst = g.edges()
    vp = sandwich.vprime(g, seeds)
    if vp.size == 0:
        pytest.skip("no node is reachable")
    q = oracle_mod.Query(g, seeds)
    theta = 40000
    for B in ([int(vp[0])], [int(x) for x in vp[:2]], [int(x) for x in vp]):
        m1, _ = exact_enum.expected_upper_bound(g.n, src, dst, g.p, seeds, B)
        qb = float(m1) / len(vp)  # each sample is covered with this probability
        est = len(vp) * q.lrr_coverage(vp, np.array(B, np.int32), theta, 31 + idx) / theta
        assert abs(est - float(m1)) <= 5 * len(vp) * math.sqrt(qb * (1 - qb) / theta) + 1e-12, B


def _brute_lrr_max_coverage(g, seeds, vp, k, theta, key, oracle_mod):
    sets = []
    for i in range(theta):
        v = int(vp[oracle_mod.lrr_pick(key, i, len(vp))])
        s = set(_lrr_by_definition(g.n, _live_edges(g, key, i, oracle_mod), seeds, v))
        if s:
            sets.append(s)

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


@pytest.mark.parametrize("case", range(4))
def test_lrr_max_coverage_matches_brute_force(oracle_mod, case):
    from oracle import sandwich
    rng = np.random.default_rng(150 + case)
    n = int(rng.integers(12, 30))
    g = synth.random_small_graph(n, int(rng.integers(2 * n, 5 * n)), seed=160 + case,
                                 prob=["mixed", "uniform", "wc"][case % 3])
    seeds = rng.choice(n, 2, replace=False).astype(np.int32)
    vp = sandwich.vprime(g, seeds)
    k, theta = int(rng.integers(1, 5)), int(rng.integers(10, 60))
    q = oracle_mod.Query(g, seeds)
    res = q.lrr_max_coverage(vp, k, theta, 9 + case, threads=1 + case % 3)
    picks, gains, covs, cus, sets = _brute_lrr_max_coverage(g, seeds, vp, k, theta, 9 + case, oracle_mod)
    assert res["blockers"].tolist() == picks
    assert res["gains"].tolist() == gains
    assert res["cov"].tolist() == covs
    assert res["cov_upper"].tolist() == cus
    if k <= 3 and len(vp) <= 18:  # the upper-bound terms bound the sample optimum
        best = max((sum(1 for c in sets if c & set(B)) for B in itertools.combinations(vp.tolist(), k)),
                   default=0)
        assert best <= min(cus)


def test_gsbm_schedule_closed_forms():
    from oracle import lsbm, sandwich
    n, ns, nvp, k, eps, delta = 50000, 10, 30000, 50, 0.2, 1e-4
    c = 1 - 1 / math.e
    want0 = 2 * (c * math.sqrt(math.log(6 / delta)) + math.sqrt(c * (lsbm.ln_binom(n - ns, k) +
                                                                    math.log(6 / delta)))) ** 2
    for opt in (0.5, 3.0, 40.0):
        tmax, t0, imax = sandwich.gsbm_schedule(n, ns, nvp, k, eps, delta, opt)
        assert math.isclose(t0, want0, rel_tol=1e-12)
        assert math.isclose(tmax / t0, nvp / (eps * eps * opt), rel_tol=1e-12)
        assert imax == max(1, math.ceil(math.log2(tmax / t0)))


@pytest.mark.parametrize("a", [3.0, 30.0])
def test_gsbm_bounds_solve_their_tail_equations(a):
    from oracle import sandwich
    theta, nvp = 800, 500
    for x in (5 * a / 18, a, 10 * a, 1e4):
        z = sandwich.gsbm_sigma_lower(x, theta, nvp, a) * theta / nvp
        assert math.isclose(x - z, math.sqrt(2 * a * z + a * a / 9) + a / 3, rel_tol=1e-9, abs_tol=1e-9)
    for y in (0, 1, a, 1e5):
        z = sandwich.gsbm_sigma_upper(y, theta, nvp, a) * theta / nvp
        assert math.isclose(z - y, math.sqrt(2 * a * z), rel_tol=1e-9, abs_tol=1e-9)


def test_lhga_on_known_scores(oracle_mod):
    """Every probability 1: each node of ON is reached in every world, so the
    score orders ON by out-degree, ties to the smaller id."""
    from oracle import sandwich
    # seed 0 -> 1..6; out-degrees of 1..6: 2, 0, 3, 3, 1, 2 (edges into 7..9)
    src = [0] * 6 + [1, 1, 3, 3, 3, 4, 4, 4, 5, 6, 6]
    dst = [1, 2, 3, 4, 5, 6] + [7, 8, 7, 8, 9, 7, 8, 9, 9, 7, 9]
    g = synth.from_edges(10, src, dst, [1.0] * len(src))
    got = sandwich.lhga(g, np.array([0], np.int32), 4, rng_seed=3, sra_batch=1 << 10)
    assert got.tolist() == [3, 4, 1, 6]
    assert sandwich.lhga(g, np.array([0], np.int32), 6, rng_seed=3).tolist() == [1, 2, 3, 4, 5, 6]


@pytest.mark.parametrize("idx", range(3))
def test_spread_estimates_are_within_gamma(oracle_mod, idx):
    from oracle import exact_enum, lsbm, sandwich
    g, seeds = _tiny(idx)
    src, dst = g.edges()
    vp = sandwich.vprime(g, seeds)
    blocked = [int(vp[0])] if vp.size else []
    m1, _ = exact_enum.expected_spread(g.n, src, dst, g.p, seeds, blocked)
    q = oracle_mod.Query(g, seeds)
    est, _ = sandwich.estimate_spread(q, 5 + idx, lsbm.reach_bound(g, seeds), blocked, 0.05, 1e-4)
    assert abs(est - float(m1)) <= 0.05 * float(m1)


def test_spread_estimate_on_a_constant_spread(oracle_mod):
    """All probabilities 1: |R_w(B)| = I is the same in every world, and the
    rule stops at the first N with N I >= b Upsilon_1."""
    from oracle import lsbm, sandwich
    g = synth.from_edges(6, [0, 0, 1, 2, 3], [1, 2, 3, 3, 4], [1.0] * 5)
    seeds = np.array([0], np.int32)
    q = oracle_mod.Query(g, seeds)
    b = lsbm.reach_bound(g, seeds)
    _, ups1 = lsbm.sra_upsilon(0.1, 1e-3)
    est, N = sandwich.estimate_spread(q, 2, b, [1], 0.1, 1e-3, batch=4096)
    I = 4  # 0, 2, 3, 4 stay reached with 1 blocked
    assert N * I >= b * ups1 > (N - 1) * I
    assert est == b * ups1 / N


def test_sandimin_picks_the_smallest_estimate(oracle_mod):
    from oracle import sandwich
    g = synth.random_small_graph(500, 3000, seed=17, prob="wc")
    seeds = np.array([3, 50, 120], np.int32)
    res = sandwich.sandimin(g, seeds, 5, eps=0.3, rng_seed=4, sra_batch=1 << 12)
    ests = [e for e, _ in res["estimates"]]
    i = "LUR".index(res["choice"])
    assert ests[i] == min(ests) and all(ests[j] > ests[i] for j in range(i))
    assert res["blockers"].tolist() == [res["B_L"], res["B_U"], res["B_R"]][i].tolist()
