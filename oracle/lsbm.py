"""Algorithm 4 (LSBM, Section 5.1) on the C oracle's coverage primitives.

TEST INFRASTRUCTURE ONLY: it checks the GPU library's LSBM and is loaded by the
tests and the CPU leg of the benchmark, never by the library.

Every step follows Section 5.1 in the paper's order and notation:

* ON, the out-neighbours of S (over edges the sampler can draw live, i.e.
  with threshold above 0; seeds left out); when |ON| <= k the answer is ON.
* I_hat, an estimate of E[I_G(s)] with (beta, delta/6) relative accuracy.  The
  paper delegates this to a generalised stopping rule it does not print; here
  it is the Stopping Rule Algorithm of Dagum, Karp, Luby and Ross ("An optimal
  algorithm for Monte Carlo estimation", SIAM J. Comput. 2000) applied to
  Z = |R_w| / b, where b (the nodes reachable from S over edges that can be
  live) bounds every world's spread so that Z lies in [0, 1].
* OPT^L, the sum of Pr[s -> v] over the k nodes of ON most likely to be
  reached, each probability estimated by its reach frequency over the N worlds
  the stopping rule drew.
* theta_max (Lemma 5.2), theta_0, i_max, a_1 = a_2 = ln(3 i_max / delta).
* For i = 1 .. i_max: Max-Coverage on the first pool C_1, its coverage on the
  second pool C_2, sigma^L from C_2 and sigma^U from Cov^u on C_1 (Lemma 5.3);
  stop when sigma^L / sigma^U >= 1 - 1/e - eps or i = i_max, else double both
  pools.

Pool j's worlds are worlds 0, 1, ... of the generator keyed by
rng_seed XOR POOL_KEY_XOR[j] (pool 1 uses rng_seed itself, so its worlds are
those of the greedy solve); the stopping rule's worlds use SRA_KEY_XOR.
Doubling a pool keeps its first half: the new CP sequences are the next worlds.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle

POOL2_KEY_XOR = 0x9E3779B97F4A7C15
SRA_KEY_XOR = 0xC2B2AE3D27D4EB4F
MASK64 = (1 << 64) - 1
E_CONST = math.e


def pool_keys(rng_seed: int):
    """(C_1 key, C_2 key, stopping-rule key)."""
    s = rng_seed & MASK64
    return s, s ^ POOL2_KEY_XOR, s ^ SRA_KEY_XOR


def _can_be_live(g) -> np.ndarray:
    """Edges the sampler can draw live: integer threshold above 0 (an edge
    with 0 < p < 2^-32 has threshold 0 and is never live)."""
    return oracle.thresholds(g.p) > 0


def out_neighbours(g, seeds) -> np.ndarray:
    """ON: nodes a seed reaches by one edge that can be live, not themselves
    seeds, ascending (Algorithm 4, first step)."""
    seeds = np.asarray(seeds, dtype=np.int64)
    live = _can_be_live(g)
    out = []
    for u in seeds:
        a, b = int(g.row_ptr[u]), int(g.row_ptr[u + 1])
        cols = np.asarray(g.col[a:b], dtype=np.int64)
        out.append(cols[live[a:b]])
    on = np.unique(np.concatenate(out)) if out else np.zeros(0, np.int64)
    return np.setdiff1d(on, seeds).astype(np.int32)


def reach_bound(g, seeds) -> int:
    """b: nodes reachable from S (seeds included) over edges that can be live,
    found level by level."""
    n = int(g.n)
    row_ptr = np.asarray(g.row_ptr, dtype=np.int64)
    col = np.asarray(g.col, dtype=np.int64)
    pos = _can_be_live(g)
    seen = np.zeros(n, dtype=bool)
    frontier = np.unique(np.asarray(seeds, dtype=np.int64))
    seen[frontier] = True
    while frontier.size:
        starts, ends = row_ptr[frontier], row_ptr[frontier + 1]
        lens = ends - starts
        if lens.sum() == 0:
            break
        idx = np.repeat(starts - np.concatenate(([0], np.cumsum(lens)[:-1])), lens) + np.arange(lens.sum())
        heads = col[idx][pos[idx]]
        heads = np.unique(heads[~seen[heads]])
        seen[heads] = True
        frontier = heads
    return int(seen.sum())


def sra_upsilon(eps: float, fail: float):
    """Upsilon = 4 (e - 2) ln(2 / fail) / eps^2 and Upsilon_1 = 1 + (1 + eps)
    Upsilon of the Stopping Rule Algorithm (relative error eps, failure
    probability fail)."""
    ups = 4.0 * (E_CONST - 2.0) * math.log(2.0 / fail) / (eps * eps)
    return ups, 1.0 + (1.0 + eps) * ups


def sra_constants(beta: float, delta: float):
    """The Stopping Rule Algorithm's constants for E[I_G(s)] in Algorithm 4:
    relative error beta, failure probability delta / 6."""
    return sra_upsilon(beta, delta / 6.0)


def stopping_rule(q: "oracle.Query", key: int, b: int, beta: float, delta: float, batch: int = 1 << 16,
                  threads=None):
    """(I_hat, N): draw worlds 0, 1, ... until the sum of |R_w| / b reaches
    Upsilon_1; I_hat = b * Upsilon_1 / N."""
    _, ups1 = sra_constants(beta, delta)
    need = float(b) * ups1
    total = 0
    w0 = 0
    while True:
        sizes = q.world_sizes(key, w0, batch, threads=threads).astype(np.int64)
        csum = total + np.cumsum(sizes)
        hit = np.nonzero(csum.astype(np.float64) >= need)[0]
        if hit.size:
            N = w0 + int(hit[0]) + 1
            return float(b) * ups1 / N, N
        total = int(csum[-1])
        w0 += batch


def ln_binom(N: int, k: int) -> float:
    """ln C(N, k) as the sum over j = 1..k of ln((N - k + j) / j)."""
    s = 0.0
    for j in range(1, k + 1):
        s += math.log((N - k + j) / j)
    return s


def theta_schedule(n: int, n_seeds: int, k: int, eps: float, beta: float, delta: float, i_hat: float,
                   opt_l: float):
    """theta_max (Lemma 5.2), theta_0 and i_max of Algorithm 4."""
    c = 1.0 - 1.0 / E_CONST
    l12 = math.log(12.0 / delta)
    root = c * math.sqrt(l12) + math.sqrt(c * (ln_binom(n - n_seeds, k) + l12))
    theta_max = 2.0 * i_hat * root * root / ((1.0 - beta) * eps * eps * opt_l)
    theta_0 = theta_max * (1.0 - beta) * eps * eps * opt_l / i_hat
    i_max = max(1, math.ceil(math.log2(theta_max / theta_0)))
    return theta_max, theta_0, i_max


def sigma_lower(cov2: int, theta2: int, beta: float, i_hat: float, a1: float) -> float:
    """sigma^L(B_L) of Algorithm 4 (Lemma 5.3): the smallest value of
    f(x) = ((sqrt(x + 2a/9) - sqrt(a/2))^2 - a/18) / |C_2| over the range of
    x = Cov / E[I] that I_hat's accuracy allows, where f is monotone; 0 where
    the range straddles f's minimum at 5a/18."""
    def f(x):
        d = math.sqrt(x + 2.0 * a1 / 9.0) - math.sqrt(a1 / 2.0)
        return (d * d - a1 / 18.0) / theta2
    lo = cov2 * (1.0 - beta) / i_hat
    hi = cov2 * (1.0 + beta) / i_hat
    if lo >= 5.0 * a1 / 18.0:
        return f(lo)
    if hi <= 5.0 * a1 / 18.0:
        return f(hi)
    return 0.0


def sigma_upper(cov_u: int, theta1: int, beta: float, i_hat: float, a2: float) -> float:
    """sigma^U(B_L^o) of Algorithm 4 (Lemma 5.3)."""
    y = cov_u * (1.0 + beta) / i_hat
    d = math.sqrt(y + a2 / 2.0) + math.sqrt(a2 / 2.0)
    return d * d / theta1


def lsbm(g, seeds, k: int, eps: float = 0.2, beta: float = 0.1, delta: float | None = None,
         rng_seed: int = 0, threads=None, sra_batch: int = 1 << 16) -> dict:
    """Algorithm 4.  Returns dict(blockers, ...) with every intermediate
    quantity (ON size, b, N, I_hat, OPT^L, the theta schedule, and per
    iteration theta, Cov_1, Cov_2, Cov^u, sigma^L, sigma^U)."""
    n = int(g.n)
    seeds = np.asarray(seeds, dtype=np.int32)
    if delta is None:
        delta = 1.0 / n
    on = out_neighbours(g, seeds)
    res = dict(on_size=int(on.size), iterations=[])
    if on.size <= k:
        res.update(blockers=on.copy(), returned_on=True)
        return res
    q = oracle.Query(g, seeds)
    k1, k2, ks = pool_keys(rng_seed)
    b = reach_bound(g, seeds)
    i_hat, N = stopping_rule(q, ks, b, beta, delta, batch=sra_batch, threads=threads)
    counts = q.reach_counts(ks, 0, N, threads=threads)
    top = np.sort(counts[on])[::-1][:k]
    opt_l = float(int(top.sum())) / N
    if opt_l <= 0.0:
        opt_l = 1.0 / N  # no node of ON was reached in the N worlds: the smallest positive estimate
    theta_max, theta_0, i_max = theta_schedule(n, len(seeds), k, eps, beta, delta, i_hat, opt_l)
    a1 = math.log(3.0 * i_max / delta)
    a2 = a1
    theta = math.ceil(theta_0)
    res.update(reach_bound=b, sra_worlds=N, i_hat=i_hat, opt_l=opt_l, theta_max=theta_max, theta_0=theta_0,
               i_max=i_max, a1=a1, returned_on=False)
    target = 1.0 - 1.0 / E_CONST - eps
    for i in range(1, i_max + 1):
        mc = q.max_coverage(k, theta, k1, threads=threads)
        bl = mc["blockers"]
        cov1 = int(mc["cov"][-1])
        cov2 = q.coverage(bl, theta, k2, threads=threads)
        cov_u = int(np.min(mc["cov_upper"]))
        sl = sigma_lower(cov2, theta, beta, i_hat, a1)
        su = sigma_upper(cov_u, theta, beta, i_hat, a2)
        res["iterations"].append(dict(theta=theta, cov1=cov1, cov2=cov2, cov_upper=cov_u, sigma_l=sl,
                                      sigma_u=su, n_selected=mc["n_selected"]))
        if sl / su >= target or i == i_max:
            res.update(blockers=bl.copy(), gains=mc["gains"].copy(), theta=theta)
            return res
        theta *= 2
    raise AssertionError("unreachable: the last iteration returns")
