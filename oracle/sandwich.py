"""GSBM (Section 5.2), LHGA (Section 5.3) and SandIMIN (Algorithm 1, Section 3.1)
on the C oracle's primitives.

TEST INFRASTRUCTURE ONLY: it checks the GPU library and is loaded by the
tests and the CPU leg of the benchmark, never by the library.

* V'_s: the non-seed nodes reachable from S over edges that can be live,
  ascending.
* GSBM follows Algorithm 4 with LRR sets (Algorithm 3) in place of CP
  sequences and the settings of Section 5.2:
  theta_max = 2 |V'_s| ((1-1/e) sqrt(ln 6/delta) + sqrt((1-1/e)(ln C(n-|S|, k)
  + ln 6/delta)))^2 / (eps^2 OPT^L), theta_0 = theta_max eps^2 OPT^L / |V'_s|,
  sigma^L = ((sqrt(Cov_2 + 2a/9) - sqrt(a/2))^2 - a/18) |V'_s| / theta,
  sigma^U = (sqrt(Cov^u_1 + a/2) + sqrt(a/2))^2 |V'_s| / theta.
  Readings: ln C(n - |S|, k), as the proof in the appendix has it (the main
  text's C(|V'_s| - |S|, k) would subtract the seeds twice, V'_s having none);
  i_max, a_1 = a_2 and the doubling as in Algorithm 4; the ON shortcut and
  OPT^L exactly as LSBM computes them.
* LHGA: the k nodes of ON with the largest score Pr[s -> v] deg(v), ties to
  the smaller id, with Pr[s -> v] the reach frequency over the stopping-rule
  worlds (so the score compares as count(v) * outdeg(v), exact integers) and
  deg(v) the node's out-degree (CSR slots); ON itself when |ON| <= k.
* SandIMIN: of B_L, B_U and B_R, the one with the smallest (gamma, delta)
  estimate of E[I_{G[V \\ B]}(s)] (the Stopping Rule Algorithm on |R_w(B)| / b
  over the worlds of the evaluation key); ties keep the earlier of L, U, R.

Keys: LRR pool j uses rng_seed XOR LRR_KEY_XOR[j]; the evaluation of
Algorithm 1 uses rng_seed XOR EVAL_KEY_XOR.
"""
from __future__ import annotations

import math

import numpy as np

from . import lsbm as L
from . import oracle

LRR1_KEY_XOR = 0x2545F4914F6CDD1D
LRR2_KEY_XOR = 0x9FB21C651E98DF25
EVAL_KEY_XOR = 0xD6E8FEB86659FD93


def vprime(g, seeds) -> np.ndarray:
    """V'_s: non-seed nodes reachable from S over edges that can be live."""
    n = int(g.n)
    row_ptr = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    live = oracle.thresholds(g.p) > 0
    seen = np.zeros(n, dtype=bool)
    frontier = np.unique(np.asarray(seeds, dtype=np.int64))
    seen[frontier] = True
    while frontier.size:
        lens = row_ptr[frontier + 1] - row_ptr[frontier]
        if lens.sum() == 0:
            break
        idx = np.repeat(row_ptr[frontier] - np.concatenate(([0], np.cumsum(lens)[:-1])), lens) + np.arange(lens.sum())
        heads = col[idx][live[idx]]
        heads = np.unique(heads[~seen[heads]])
        seen[heads] = True
        frontier = heads
    seen[np.asarray(seeds, dtype=np.int64)] = False
    return np.nonzero(seen)[0].astype(np.int32)


def reach_estimates(g, seeds, beta: float, delta: float, rng_seed: int, threads=None, sra_batch: int = 1 << 16):
    """(N, reach counts int64[n]) over the stopping-rule worlds of Algorithm 4."""
    q = oracle.Query(g, np.asarray(seeds, dtype=np.int32))
    _, _, ks = L.pool_keys(rng_seed)
    _, N = L.stopping_rule(q, ks, L.reach_bound(g, seeds), beta, delta, batch=sra_batch, threads=threads)
    return N, q.reach_counts(ks, 0, N, threads=threads)


def opt_lower(on, counts, N: int, k: int) -> float:
    top = np.sort(counts[on])[::-1][:k]
    opt = float(int(top.sum())) / N
    return opt if opt > 0.0 else 1.0 / N


def gsbm_schedule(n: int, n_seeds: int, nvp: int, k: int, eps: float, delta: float, opt_l: float):
    """theta_max, theta_0 and i_max of GSBM (Section 5.2)."""
    c = 1.0 - 1.0 / L.E_CONST
    l6 = math.log(6.0 / delta)
    root = c * math.sqrt(l6) + math.sqrt(c * (L.ln_binom(n - n_seeds, k) + l6))
    theta_max = 2.0 * nvp * root * root / (eps * eps * opt_l)
    theta_0 = theta_max * eps * eps * opt_l / nvp
    i_max = max(1, math.ceil(math.log2(theta_max / theta_0)))
    return theta_max, theta_0, i_max


def gsbm_sigma_lower(cov2: int, theta: int, nvp: int, a1: float) -> float:
    d = math.sqrt(cov2 + 2.0 * a1 / 9.0) - math.sqrt(a1 / 2.0)
    return (d * d - a1 / 18.0) * nvp / theta


def gsbm_sigma_upper(cov_u: int, theta: int, nvp: int, a2: float) -> float:
    d = math.sqrt(cov_u + a2 / 2.0) + math.sqrt(a2 / 2.0)
    return d * d * nvp / theta


def gsbm(g, seeds, k: int, eps: float = 0.2, beta: float = 0.1, delta: float | None = None, rng_seed: int = 0,
         threads=None, sra_batch: int = 1 << 16, estimates=None) -> dict:
    """GSBM; estimates = (N, counts) shares the stopping-rule worlds."""
    n = int(g.n)
    seeds = np.asarray(seeds, dtype=np.int32)
    if delta is None:
        delta = 1.0 / n
    on = L.out_neighbours(g, seeds)
    res = dict(on_size=int(on.size), iterations=[])
    if on.size <= k:
        res.update(blockers=on.copy(), returned_on=True)
        return res
    vp = vprime(g, seeds)
    N, counts = estimates or reach_estimates(g, seeds, beta, delta, rng_seed, threads, sra_batch)
    opt_l = opt_lower(on, counts, N, k)
    theta_max, theta_0, i_max = gsbm_schedule(n, len(seeds), int(vp.size), k, eps, delta, opt_l)
    a1 = math.log(3.0 * i_max / delta)
    res.update(returned_on=False, nvp=int(vp.size), opt_l=opt_l, theta_max=theta_max, theta_0=theta_0,
               i_max=i_max, a1=a1)
    q = oracle.Query(g, seeds)
    k1, k2 = (rng_seed ^ LRR1_KEY_XOR) & L.MASK64, (rng_seed ^ LRR2_KEY_XOR) & L.MASK64
    theta = math.ceil(theta_0)
    target = 1.0 - 1.0 / L.E_CONST - eps
    for i in range(1, i_max + 1):
        mc = q.lrr_max_coverage(vp, k, theta, k1, threads=threads)
        bu = mc["blockers"]
        cov2 = q.lrr_coverage(vp, bu, theta, k2, threads=threads)
        cov_u = int(np.min(mc["cov_upper"]))
        sl = gsbm_sigma_lower(cov2, theta, int(vp.size), a1)
        su = gsbm_sigma_upper(cov_u, theta, int(vp.size), a1)
        res["iterations"].append(dict(theta=theta, cov1=int(mc["cov"][-1]), cov2=cov2, cov_upper=cov_u,
                                      sigma_l=sl, sigma_u=su, n_selected=mc["n_selected"]))
        if sl / su >= target or i == i_max:
            res.update(blockers=bu.copy(), theta=theta)
            return res
        theta *= 2
    raise AssertionError("unreachable: the last iteration returns")


def lhga(g, seeds, k: int, beta: float = 0.1, delta: float | None = None, rng_seed: int = 0, threads=None,
         sra_batch: int = 1 << 16, estimates=None) -> np.ndarray:
    """LHGA (Section 5.3): blockers, ascending score order broken by id."""
    seeds = np.asarray(seeds, dtype=np.int32)
    if delta is None:
        delta = 1.0 / int(g.n)
    on = L.out_neighbours(g, seeds)
    if on.size <= k:
        return on.copy()
    _, counts = estimates or reach_estimates(g, seeds, beta, delta, rng_seed, threads, sra_batch)
    outdeg = np.diff(np.asarray(g.row_ptr, dtype=np.int64))
    score = counts[on] * outdeg[on]
    order = sorted(range(on.size), key=lambda i: (-int(score[i]), int(on[i])))
    return on[order[:k]].astype(np.int32)


def estimate_spread(q: "oracle.Query", key: int, b: int, blocked, gamma: float, delta: float, batch: int = 1 << 16,
                    threads=None):
    """(gamma, delta) estimate of E[I_{G[V \\ B]}(s)] by the Stopping Rule
    Algorithm on |R_w(B)| / b; returns (estimate, N)."""
    _, ups1 = L.sra_upsilon(gamma, delta)
    need = float(b) * ups1
    total, w0 = 0, 0
    while True:
        sizes = q.world_sizes(key, w0, batch, threads=threads, blocked=blocked).astype(np.int64)
        csum = total + np.cumsum(sizes)
        hit = np.nonzero(csum.astype(np.float64) >= need)[0]
        if hit.size:
            N = w0 + int(hit[0]) + 1
            return float(b) * ups1 / N, N
        total = int(csum[-1])
        w0 += batch


def sandimin(g, seeds, k: int, eps: float = 0.2, beta: float = 0.1, gamma: float = 0.1,
             delta: float | None = None, rng_seed: int = 0, threads=None, sra_batch: int = 1 << 16) -> dict:
    """Algorithm 1: dict(blockers, choice, estimates, B_L, B_U, B_R)."""
    seeds = np.asarray(seeds, dtype=np.int32)
    if delta is None:
        delta = 1.0 / int(g.n)
    est = reach_estimates(g, seeds, beta, delta, rng_seed, threads, sra_batch)
    bl = L.lsbm(g, seeds, k, eps=eps, beta=beta, delta=delta, rng_seed=rng_seed, threads=threads,
                sra_batch=sra_batch)["blockers"]
    bu = gsbm(g, seeds, k, eps=eps, beta=beta, delta=delta, rng_seed=rng_seed, threads=threads,
              sra_batch=sra_batch, estimates=est)["blockers"]
    br = lhga(g, seeds, k, beta=beta, delta=delta, rng_seed=rng_seed, threads=threads, estimates=est)
    q = oracle.Query(g, seeds)
    b = L.reach_bound(g, seeds)
    key = (rng_seed ^ EVAL_KEY_XOR) & L.MASK64
    ests = [estimate_spread(q, key, b, cand, gamma, delta, batch=sra_batch, threads=threads)
            for cand in (bl, bu, br)]
    best = min(range(3), key=lambda i: (ests[i][0], i))
    return dict(blockers=[bl, bu, br][best].copy(), choice="LUR"[best], estimates=ests, B_L=bl, B_U=bu, B_R=br)
