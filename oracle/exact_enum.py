"""Exact expectations by enumerating every live-edge world of a tiny graph.

TEST INFRASTRUCTURE ONLY.  For a graph with at most ~20 edges this sums over
all 2^m realizations phi with their exact probabilities (Section 2.1, Eq. 1:
E[I_G(S)] = sum_phi p(phi) * I_phi(S)), in rational arithmetic.  Each edge is
kept with the probability the sampler realises, q_e = thr_e / 2^32 (or 1 for
an "always live" edge), so sampled estimates can be compared against exact
values with a known variance.

Nothing here is shared with the C oracle: the threshold rule, reachability and
the protected-node counts are written again in plain Python.
"""
from __future__ import annotations

from fractions import Fraction
from itertools import product

ALWAYS_LIVE = 0xFFFFFFFF
TWO32 = 1 << 32


def threshold(p: float) -> int:
    """Integer coin threshold of a float32 probability (exact rational floor)."""
    if p != p or p < 0.0 or p > 1.0:
        raise ValueError(f"probability {p!r} not in [0, 1]")
    if p == 1.0:
        return ALWAYS_LIVE
    return int(Fraction(float(p)) * TWO32)  # int() of a non-negative Fraction is its floor


def keep_probability(p: float) -> Fraction:
    t = threshold(p)
    return Fraction(1) if t == ALWAYS_LIVE else Fraction(t, TWO32)


def _reach(n, edges, live, seeds, blocked):
    """Nodes reachable from the seeds over live edges, never entering blocked nodes."""
    adj = [[] for _ in range(n)]
    for (u, v), on in zip(edges, live):
        if on:
            adj[u].append(v)
    seen = set(int(s) for s in seeds)
    stack = list(seen)
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if v in blocked or v in seen:
                continue
            seen.add(v)
            stack.append(v)
    return seen


def enumerate_worlds(n, src, dst, p):
    """Yield (probability, live tuple) for every realization."""
    edges = list(zip((int(x) for x in src), (int(x) for x in dst)))
    q = [keep_probability(float(x)) for x in p]
    for live in product((False, True), repeat=len(edges)):
        pr = Fraction(1)
        for on, qe in zip(live, q):
            pr *= qe if on else (1 - qe)
            if pr == 0:
                break
        if pr:
            yield pr, edges, live


def expected_spread(n, src, dst, p, seeds, blocked=()):
    """(E[|R(B)|], E[|R(B)|^2]) exactly."""
    blocked = set(int(b) for b in blocked)
    m1 = Fraction(0)
    m2 = Fraction(0)
    for pr, edges, live in enumerate_worlds(n, src, dst, p):
        r = len(_reach(n, edges, live, seeds, blocked))
        m1 += pr * r
        m2 += pr * r * r
    return m1, m2


def expected_protection(n, src, dst, p, seeds, blocked=()):
    """For every u: (E[c(u|B)], E[c(u|B)^2]) exactly, with
    c(u|B) = |R(B)| - |R(B + u)| (Section 2.1, the decreased spread), and 0 for
    seeds and blocked nodes."""
    blocked = set(int(b) for b in blocked)
    seeds_set = set(int(s) for s in seeds)
    m1 = [Fraction(0)] * n
    m2 = [Fraction(0)] * n
    for pr, edges, live in enumerate_worlds(n, src, dst, p):
        base = _reach(n, edges, live, seeds, blocked)
        for u in base:
            if u in seeds_set:
                continue
            c = len(base) - len(_reach(n, edges, live, seeds, blocked | {u}))
            m1[u] += pr * c
            m2[u] += pr * c * c
    return m1, m2


def expected_dominator_subtrees(n, src, dst, p, seeds, blocked=()):
    """E[size of u's subtree in the dominator tree rooted at a virtual source]
    for every u, using networkx's dominator routine on each realization
    (the quantity the dominator-tree lemma quoted in Section 2.2 equates with
    the expected protected count)."""
    import networkx as nx

    blocked = set(int(b) for b in blocked)
    seeds_set = set(int(s) for s in seeds)
    root = n  # virtual source, not in V
    acc = [Fraction(0)] * n
    for pr, edges, live in enumerate_worlds(n, src, dst, p):
        reached = _reach(n, edges, live, seeds, blocked)
        gr = nx.DiGraph()
        gr.add_node(root)
        for s in seeds_set:
            gr.add_edge(root, s)
        for (u, v), on in zip(edges, live):
            if on and u in reached and v in reached and u != v:
                gr.add_edge(u, v)
        idom = nx.immediate_dominators(gr, root)
        size = {v: 1 for v in gr.nodes}
        # children before parents: deepest first
        depth = {}
        for v in gr.nodes:
            d, x = 0, v
            while x != root:
                x = idom[x]
                d += 1
            depth[v] = d
        for v in sorted(gr.nodes, key=lambda x: -depth[x]):
            if v != root:
                size[idom[v]] += size[v]
        for v in reached:
            if v not in seeds_set:
                acc[v] += pr * size[v]
    return acc


def expected_lower_bound(n, src, dst, p, seeds, B):
    """(D^L(B), E[f^2]) exactly, where f(phi) = |union over v in B of N_phi(v)|
    and N_phi(v) is the set of nodes that stop being reached when v alone is
    blocked (Section 3.2, the lower bounding function)."""
    B = [int(b) for b in B]
    m1 = Fraction(0)
    m2 = Fraction(0)
    for pr, edges, live in enumerate_worlds(n, src, dst, p):
        base = _reach(n, edges, live, seeds, set())
        lost = set()
        for v in B:
            if v in base:
                lost |= base - _reach(n, edges, live, seeds, {v})
        m1 += pr * len(lost)
        m2 += pr * len(lost) * len(lost)
    return m1, m2


def expected_upper_bound(n, src, dst, p, seeds, B):
    """(D^U(B), E[f^2]) exactly, where f(phi) = |M_phi(B)|, the nodes reachable
    from B in phi^s: the live subgraph induced by the reached non-seeds
    (Section 3.3, the upper bounding function)."""
    B = [int(b) for b in B]
    sset = set(int(s) for s in seeds)
    m1 = Fraction(0)
    m2 = Fraction(0)
    for pr, edges, live in enumerate_worlds(n, src, dst, p):
        base = _reach(n, edges, live, seeds, set())
        inside = base - sset
        adj = {}
        for (u, v), on in zip(edges, live):
            if on and u in inside and v in inside:
                adj.setdefault(u, []).append(v)
        seen = set(b for b in B if b in inside)
        stack = list(seen)
        while stack:
            u = stack.pop()
            for v in adj.get(u, ()):
                if v not in seen:
                    seen.add(v)
                    stack.append(v)
        m1 += pr * len(seen)
        m2 += pr * len(seen) * len(seen)
    return m1, m2
