"""Pins of the oracle's two variants (CPU only).

* R_T-only key (Alg. 1 Step 2 says "sort L based on resistances"): the order is the
  exact tree-path resistance, rounded once, descending, ties by id; with unit weights it
  coincides with the stretch order, so the whole result must equal the default one.
* Loose condition (Def. "Similar edge (Loose)", eq. cond-loose-2, with the multi-pass rule
  of Sec. II-B): checked against an all-pairs greedy written from the definition on tiny
  graphs, brute mode = indexed mode, and the paper's own remark that once the BFS step is
  at least the tree's diameter, recovering one edge covers the graph, so every pass
  recovers exactly one edge (the next one in the criticality order).
"""
import numpy as np
import pytest

import oracle
from paper_2508_20403_amd import synth
from tests import brute

SMALL = [
    lambda s: synth.random_connected(40, 70, seed=s, alpha=0.3, beta=2),
    lambda s: synth.random_connected(60, 110, seed=s, alpha=0.4, beta=1, tree="random"),
    lambda s: synth.grid((7, 6), 1.0, 100.0, seed=s, alpha=0.3, beta=2),
    lambda s: synth.path_graph(30, 40, seed=s, alpha=0.5, beta=2),
    lambda s: synth.star_graph(25, 40, seed=s, alpha=0.5, beta=1),
]


@pytest.mark.parametrize("make", SMALL)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_rt_key_matches_brute(make, seed):
    g = make(seed)
    for k in (-1, 3, g.m):
        o = oracle.recover(g, k_override=k, key_rt=True, mode=oracle.MODE_BRUTE)
        o2 = oracle.recover(g, k_override=k, key_rt=True, mode=oracle.MODE_INDEXED)
        kk = o.K
        order, passes = brute.greedy_brute_variant(g, g.beta, kk, key_rt=True)
        assert list(o.order[: o.info["n_recovered"]]) == order
        assert o.info["passes"] == passes
        np.testing.assert_array_equal(o.order, o2.order)
        np.testing.assert_array_equal(o.mask, o2.mask)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_rt_key_equals_stretch_key_on_unit_weights(seed):
    g = synth.grid((9, 8), 1.0, 1.0, seed=seed, alpha=0.3, beta=2)  # w = 1: stretch = R_T
    for k in (-1, g.m):
        a = oracle.recover(g, k_override=k, key_rt=True, full=True)
        b = oracle.recover(g, k_override=k, full=True)
        np.testing.assert_array_equal(a.order, b.order)
        np.testing.assert_array_equal(a.mask, b.mask)
        np.testing.assert_array_equal(a.rank_of, b.rank_of)


@pytest.mark.parametrize("make", SMALL)
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("c", [0, 1, 2, 3])
def test_loose_matches_brute(make, seed, c):
    g = make(seed)
    for k in (-1, 5, g.m):
        o = oracle.recover(g, beta=c, k_override=k, loose=True, mode=oracle.MODE_BRUTE)
        o2 = oracle.recover(g, beta=c, k_override=k, loose=True, mode=oracle.MODE_INDEXED)
        order, passes = brute.greedy_brute_variant(g, c, o.K, loose=True)
        assert list(o.order[: o.info["n_recovered"]]) == order, (c, k)
        assert o.info["passes"] == passes
        np.testing.assert_array_equal(o.order, o2.order)
        np.testing.assert_array_equal(o.mask, o2.mask)
        assert o.info["passes"] == o2.info["passes"]


@pytest.mark.parametrize("seed", [0, 1])
def test_loose_with_step_at_least_the_diameter_recovers_one_edge_per_pass(seed):
    g = synth.random_connected(50, 90, seed=seed, alpha=0.2, beta=2)
    adj = brute.tree_adj(g)
    diam = max(max(brute.tree_dist_from(adj, x)) for x in range(g.n))
    o = oracle.recover(g, beta=diam, loose=True, full=True)
    strict = oracle.recover(g, full=True)  # same criticality order (the stretch)
    off = np.flatnonzero(strict.is_tree == 0)
    pi = off[np.argsort(strict.rank_of[off], kind="stable")]
    K = o.K
    assert o.info["passes"] == K
    np.testing.assert_array_equal(o.order, pi[:K])


def test_loose_has_no_subtask_mode():
    g = synth.random_connected(30, 40, seed=0)
    assert oracle.recover(g, loose=True, mode=oracle.MODE_SUBTASK).status == -1
