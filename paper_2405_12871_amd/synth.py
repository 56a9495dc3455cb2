"""Seeded synthetic inputs: directed graphs with edge probabilities, and seed sets.

This module is the only code shared by the CPU oracle's tests and the GPU path.
It draws inputs and nothing else: it holds none of the estimator's arithmetic
(no coins, thresholds, reachability or dominators).

Graphs stand in for the social networks of the paper's experiments (Section 6,
Table 6: directed and undirected SNAP graphs from 1K to 1.6M nodes with average
degree 3.2 to 59.5), which are not available here.  They are directed Chung-Lu
power-law graphs:

* expected out-weights r_i = (i + i0)^(-1/(gamma-1)), i0 fixed by bisection so
  that the heaviest node's expected degree is ceil(sqrt(m)) (the structural
  cut-off);
* in-weights are the same sequence under a seeded permutation, so in- and
  out-rank are uncorrelated;
* endpoints are drawn by inverse CDF, self-loops and repeated pairs dropped,
  until exactly m distinct edges exist;
* nodes are relabelled by a seeded permutation and edges sorted by
  (source, destination) into CSR.

Edge probabilities follow one of the two models the influence literature uses:

* ``wc``: weighted cascade, p(u, v) = 1 / indeg(v) (Section 6, parameter
  settings), computed as an IEEE float32 division;
* ``tri``: trivalency, p drawn uniformly from {0.1, 0.01, 0.001} (float32).

Every draw comes from numpy's PCG64 keyed by an explicit seed, so a graph is a
pure function of its parameters; ``Graph.sha256`` fingerprints the arrays.
"""
from __future__ import annotations

import dataclasses
import functools
import hashlib
import math

import numpy as np

__all__ = [
    "Graph",
    "chung_lu",
    "from_edges",
    "seeds_uniform",
    "seeds_top_out",
    "random_small_graph",
    "WORKLOADS",
    "workload",
    "GRAPHS",
    "named_graph",
    "query_mix",
]


@dataclasses.dataclass
class Graph:
    """A directed graph in CSR form with one float32 probability per edge slot.

    ``row_ptr`` is int64[n+1]; the out-edges of u are the slots
    ``row_ptr[u] .. row_ptr[u+1]-1``; ``col`` (int32) holds their heads and
    ``p`` (float32) their propagation probabilities.  The slot index is the
    edge id.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    p: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        for a in (self.row_ptr, self.col, self.p):
            h.update(np.ascontiguousarray(a).tobytes())
        return h.hexdigest()

    def out_degree(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def in_degree(self) -> np.ndarray:
        return np.bincount(self.col, minlength=self.n).astype(np.int64)

    def edges(self):
        """(src int64[m], dst int64[m]) in slot order."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.out_degree())
        return src, self.col.astype(np.int64)


def from_edges(n: int, src, dst, p, name: str = "", sort: bool = True) -> Graph:
    """CSR graph from edge arrays.  With ``sort`` the slots are ordered by
    (src, dst); otherwise edges keep their given order within each source."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    p = np.asarray(p, dtype=np.float32)
    if src.shape != dst.shape or src.shape != p.shape:
        raise ValueError("src, dst and p must have the same length")
    if src.size and (src.min() < 0 or src.max() >= n or dst.min() < 0 or dst.max() >= n):
        raise ValueError("endpoint out of range")
    order = np.lexsort((dst, src)) if sort else np.argsort(src, kind="stable")
    src, dst, p = src[order], dst[order], p[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.int32), p=p.copy(), name=name)


def _offset_for_cap(n: int, m: int, a: float, d_max: float) -> float:
    """i0 > 0 such that m * r_0 / sum_i r_i == d_max, r_i = (i + i0)^-a."""
    idx = np.arange(n, dtype=np.float64)

    def heaviest(i0: float) -> float:
        r = (idx + i0) ** (-a)
        return m * r[0] / r.sum()

    lo, hi = 1e-9, float(n)
    if heaviest(hi) > d_max:  # even a flat sequence is too concentrated
        return hi
    for _ in range(200):
        mid = math.sqrt(lo * hi) if lo > 0 else 0.5 * hi
        if heaviest(mid) > d_max:
            lo = mid
        else:
            hi = mid
        if hi / lo < 1.0 + 1e-12:
            break
    return hi


def _wc_probabilities(n: int, dst: np.ndarray) -> np.ndarray:
    indeg = np.bincount(dst, minlength=n).astype(np.float32)
    return (np.float32(1.0) / indeg[dst]).astype(np.float32)


def chung_lu(n: int, m: int, gamma: float = 2.1, prob: str = "wc", gen_seed: int = 0,
             name: str = "") -> Graph:
    """Directed Chung-Lu power-law graph with exactly m distinct edges."""
    if m > n * (n - 1):
        raise ValueError("too many edges for a simple digraph")
    rng = np.random.Generator(np.random.PCG64(gen_seed))
    a = 1.0 / (gamma - 1.0)
    d_max = float(math.ceil(math.sqrt(m)))
    i0 = _offset_for_cap(n, m, a, d_max)
    r = (np.arange(n, dtype=np.float64) + i0) ** (-a)
    w_out = r
    w_in = np.empty(n, dtype=np.float64)
    w_in[rng.permutation(n)] = r
    cdf_out = np.cumsum(w_out)
    cdf_out /= cdf_out[-1]
    cdf_in = np.cumsum(w_in)
    cdf_in /= cdf_in[-1]

    keys = np.empty(0, dtype=np.int64)
    while True:
        have = np.unique(keys).size if keys.size else 0
        batch = int((m - have) * 1.3) + 4096
        u = np.minimum(np.searchsorted(cdf_out, rng.random(batch), side="right"), n - 1)
        v = np.minimum(np.searchsorted(cdf_in, rng.random(batch), side="right"), n - 1)
        keep = u != v
        keys = np.concatenate([keys, u[keep].astype(np.int64) * n + v[keep]])
        uniq, first = np.unique(keys, return_index=True)
        if uniq.size >= m:
            keys = keys[np.sort(first)[:m]]
            break
    src, dst = keys // n, keys % n
    sigma = rng.permutation(n).astype(np.int64)
    src, dst = sigma[src], sigma[dst]
    order = np.lexsort((dst, src))
    src, dst = src[order], dst[order]

    if prob == "wc":
        p = _wc_probabilities(n, dst)
    elif prob == "tri":
        levels = np.array([0.1, 0.01, 0.001], dtype=np.float32)
        p = levels[rng.integers(0, 3, size=m)]
    else:
        raise ValueError(f"unknown probability model {prob!r}")
    return from_edges(n, src, dst, p, name=name or f"chung_lu(n={n},m={m},{prob},seed={gen_seed})")


def seeds_uniform(n: int, count: int, query_seed: int) -> np.ndarray:
    """``count`` distinct node ids drawn uniformly (int32)."""
    rng = np.random.Generator(np.random.PCG64(query_seed))
    return rng.choice(n, size=count, replace=False).astype(np.int32)


def seeds_top_out(g: Graph, count: int) -> np.ndarray:
    """The ``count`` nodes of highest out-degree, ties to the smaller id."""
    deg = g.out_degree()
    order = np.lexsort((np.arange(g.n), -deg))
    return order[:count].astype(np.int32)


def random_small_graph(n: int, m: int, seed: int, prob: str = "mixed",
                       allow_multi: bool = False) -> Graph:
    """Small random digraph for parity tests.

    ``prob``: ``mixed`` draws p from {0, 1, uniform(0,1)} so that never-live,
    always-live and coin-decided edges all occur; ``binary`` draws p from
    {0, 1}; ``uniform`` draws p uniformly; ``wc`` uses 1/indeg.
    With ``allow_multi`` repeated (u, v) pairs and self-loops are kept.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if allow_multi:
        src = rng.integers(0, n, size=m)
        dst = rng.integers(0, n, size=m)
    else:
        m = min(m, n * (n - 1))
        keys = set()
        src_l, dst_l = [], []
        while len(keys) < m:
            u, v = int(rng.integers(0, n)), int(rng.integers(0, n))
            if u == v or (u, v) in keys:
                continue
            keys.add((u, v))
            src_l.append(u)
            dst_l.append(v)
        src, dst = np.array(src_l, dtype=np.int64), np.array(dst_l, dtype=np.int64)
    if prob == "mixed":
        kind = rng.integers(0, 4, size=len(src))
        p = rng.random(len(src)).astype(np.float32)
        p[kind == 0] = 0.0
        p[kind == 1] = 1.0
    elif prob == "binary":
        p = rng.integers(0, 2, size=len(src)).astype(np.float32)
    elif prob == "uniform":
        p = rng.random(len(src)).astype(np.float32)
    elif prob == "wc":
        p = _wc_probabilities(n, np.asarray(dst, dtype=np.int64))
    else:
        raise ValueError(prob)
    return from_edges(n, src, dst, p, name=f"random(n={n},m={m},{prob},seed={seed})")


# Workloads: graph shape, probability model, seed-set rule and query sizes.
WORKLOADS = {
    # 1,000 nodes / 5,000 edges, WC, |S|=10 uniform, k=5, theta=1e4
    "small": dict(n=1_000, m=5_000, prob="wc", gen_seed=101, seeds=("uniform", 10, 1),
                  k=5, theta=10_000),
    # 100,000 nodes / 1,000,000 edges, WC, |S|=50 highest out-degree, k=100, theta=1e5
    "medium": dict(n=100_000, m=1_000_000, prob="wc", gen_seed=102, seeds=("top_out", 50, 0),
                   k=100, theta=100_000),
    # 1,000,000 nodes / 10,000,000 edges, trivalency, |S|=200 uniform, k=500, theta=2e5
    "large": dict(n=1_000_000, m=10_000_000, prob="tri", gen_seed=103, seeds=("uniform", 200, 3),
                  k=500, theta=200_000),
}


@functools.lru_cache(maxsize=4)
def workload(name: str):
    """(graph, seeds int32, k, theta) for a named workload (cached per process;
    callers must not modify the returned arrays)."""
    spec = WORKLOADS[name]
    g = chung_lu(spec["n"], spec["m"], prob=spec["prob"], gen_seed=spec["gen_seed"], name=name)
    rule, count, qseed = spec["seeds"]
    if rule == "uniform":
        seeds = seeds_uniform(g.n, count, qseed)
    else:
        seeds = seeds_top_out(g, count)
    return g, seeds, spec["k"], spec["theta"]


# Weighted-cascade graphs that batches and serving run on: the medium
# workload's graph, the weighted-cascade twin of the large workload's graph
# (same generator seed), and a 4M-node graph.
GRAPHS = {
    "wc100k": dict(n=100_000, m=1_000_000, gen_seed=102),
    "wc1m": dict(n=1_000_000, m=10_000_000, gen_seed=103),
    "wc4m": dict(n=4_000_000, m=40_000_000, gen_seed=105),
}


@functools.lru_cache(maxsize=4)
def named_graph(name: str) -> Graph:
    """A weighted-cascade Chung-Lu graph of GRAPHS (cached per process)."""
    spec = GRAPHS[name]
    return chung_lu(spec["n"], spec["m"], prob="wc", gen_seed=spec["gen_seed"], name=name)


def query_mix(count: int, n_nodes, seed: int, seeds_range, k_range, thetas, n_graphs: int = 1):
    """``count`` queries drawn from numpy PCG64(seed): a graph index uniform
    in [0, n_graphs), |S| uniform in seeds_range (inclusive) as distinct
    uniform nodes of that graph (n_nodes[g] nodes), k uniform in k_range
    (inclusive), theta uniform from ``thetas``, and a 62-bit coin key.
    Returns [(graph index, seeds int32, k, theta, coin key)]."""
    rs = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        gi = int(rs.integers(0, n_graphs))
        ns = int(rs.integers(seeds_range[0], seeds_range[1] + 1))
        seeds = rs.choice(int(n_nodes[gi]), size=ns, replace=False).astype(np.int32)
        k = int(rs.integers(k_range[0], k_range[1] + 1))
        theta = int(rs.choice(list(thetas)))
        out.append((gi, seeds, k, theta, int(rs.integers(0, 1 << 62))))
    return out
