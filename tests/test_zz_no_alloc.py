"""imin_solve_static: the solve whose workspace is the library's fixed device
array, called through the C ABI, against imin_solve with a workspace of its
own (and the oracle) on two calls in a row, the second smaller."""
import sys

import numpy as np
import pytest

from paper_2405_12871_amd import synth

pytestmark = pytest.mark.gpu

IMIN_ERR_WORKSPACE = 6


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


def _same(a, b):
    assert a.n_selected == b.n_selected
    np.testing.assert_array_equal(a.blockers, b.blockers)
    np.testing.assert_array_equal(a.gains, b.gains)
    np.testing.assert_array_equal(a.spread_totals, b.spread_totals)


def test_static_solve_equals_workspace_solve(B, oracle_mod):
    calls = [  # (graph, seeds, k, theta, rng): the second input is smaller
        (synth.random_small_graph(500, 2500, seed=401, prob="mixed"), [3, 77, 140, 222, 300, 401], 8, 1500, 11),
        (synth.random_small_graph(120, 400, seed=402, prob="uniform"), [5, 9], 3, 300, 12),
    ]
    for g, seeds, k, theta, rng in calls:
        seeds = np.array(seeds, np.int32)
        _log(f"static solve n={g.n} m={g.m} |S|={len(seeds)} k={k} theta={theta}")
        G = B.Graph.from_synth(g)
        got = B.solve_static(G, seeds, k, theta, rng)
        _same(got, B.solve_ws(G, seeds, k, theta, rng))
        want = oracle_mod.Query(g, seeds).solve(k, theta, rng)
        assert got.n_selected == want["n_selected"]
        np.testing.assert_array_equal(got.blockers, want["blockers"])
        np.testing.assert_array_equal(got.spread_totals, want["spread_totals"])


def test_static_solve_rejects_a_layout_beyond_the_array(B):
    g = synth.random_small_graph(200, 800, seed=403, prob="uniform")
    G = B.Graph.from_synth(g)
    with pytest.raises(B.IminError) as ei:
        B.solve_static(G, np.array([1, 2], np.int32), 2, 1 << 20, 0)
    assert ei.value.status == IMIN_ERR_WORKSPACE
