"""The reasoning behind the incremental rounds' label rule, checked by brute
force on small deterministic worlds (every edge live), with no GPU and no
oracle code: dominators straight from their definition (§2.2: u protects v
when every path from the seeds to v passes through u; the count of u is the
number of nodes u protects, itself included — §3.1's unified seed joins the
seeds).

The claim: when no edge leads from u's dominator subtree to a reached node
outside it (edges whose head dominates their tail aside), blocking u removes
exactly u's subtree; every ancestor of u loses count(u); no other count
changes; and no node that had no such edge out of its subtree gains one.
A world where the claim's condition fails is checked to need the full
recomputation the replay does (some count then differs from the rule's
prediction in at least one case of the sample)."""
import random

import pytest


def reach(n, adj, seeds, removed):
    seen = set()
    stack = [s for s in seeds if s not in removed]
    seen.update(stack)
    while stack:
        x = stack.pop()
        for y in adj[x]:
            if y not in seen and y not in removed:
                seen.add(y)
                stack.append(y)
    return seen


def dominators(n, adj, seeds, removed):
    """For every reached non-seed v, the set of reached non-seeds that
    dominate it (itself included), by definition."""
    R = reach(n, adj, seeds, removed)
    dom = {v: {v} for v in R if v not in seeds}
    for u in list(dom):
        Ru = reach(n, adj, seeds, removed | {u})
        for v in dom:
            if v != u and v not in Ru:
                dom[v].add(u)
    return R, dom


def subtree(dom, u):
    return {v for v, ds in dom.items() if u in ds}


def counts(dom):
    return {u: len(subtree(dom, u)) for u in dom}


def exits(n, adj, R, dom, u):
    """Some edge leads from u's subtree to a reached node outside it, its
    head not a dominator of its tail."""
    sub = subtree(dom, u)
    for a in sub:
        for b in adj[a]:
            if b in R and b not in sub and not (b in dom and b in dom[a]):
                if b in dom:
                    return True
    return False


def random_world(rng, n, m, n_seeds):
    adj = [[] for _ in range(n)]
    for _ in range(m):
        a, b = rng.randrange(n), rng.randrange(n)
        if a != b:
            adj[a].append(b)
    seeds = set(rng.sample(range(n), n_seeds))
    return adj, seeds


@pytest.mark.parametrize("seed", range(6))
def test_label_rule_holds_without_exits(seed):
    rng = random.Random(1000 + seed)
    checked = failed_condition_differs = 0
    for _ in range(150):
        n = rng.randint(5, 12)
        adj, seeds = random_world(rng, n, rng.randint(n, 3 * n), rng.randint(1, 2))
        R, dom = dominators(n, adj, seeds, set())
        c = counts(dom)
        for u in list(dom):
            R2, dom2 = dominators(n, adj, seeds, {u})
            c2 = counts(dom2)
            sub = subtree(dom, u)
            predicted = {}
            for v in dom:
                if v in sub:
                    continue
                predicted[v] = c[v] - c[u] if v in dom[u] else c[v]
            if not exits(n, adj, R, dom, u):
                checked += 1
                # exactly the subtree is lost
                assert R - R2 == sub
                # ancestors lose count(u), the others keep theirs
                assert c2 == predicted
                # the dominator sets of the rest are unchanged
                for v in dom2:
                    assert dom2[v] == dom[v]
                # exit bits only go from set to clear
                for v in dom2:
                    if exits(n, adj, R2, dom2, v):
                        assert exits(n, adj, R, dom, v)
            elif c2 != predicted:
                failed_condition_differs += 1
    assert checked > 100
    # the condition is not vacuous: without it the rule can be wrong
    assert failed_condition_differs > 0
