"""The loose-condition pass computed the way the GPU does it, in rounds of local decisions
over tree-ancestor cells, reaches the oracle's serial pass exactly (CPU only).

Under feGRASS's loose condition (Def. "Similar edge (Loose)", eq. cond-loose-2) two
off-tree edges conflict when an endpoint of one lies within c tree hops of an endpoint of
the other, a symmetric relation, so one serial pass recovers the lexicographically first
maximal independent set of the conflict graph in rank order.  This file re-derives every
pass that way, with nothing taken from the oracle but the order and the endpoints:
tree hops through common ancestors (hops(x, y) <= c iff some z is the i-th ancestor of x
and the j-th of y with i + j <= c), an undecided edge with no lower-ranked undecided
conflict is recovered, an undecided edge conflicting with a recovered one is marked.  The
passes then follow the multi-pass rule of Sec. II-B (marks cleared, recovered edges
removed), and the pass of every edge must equal the oracle's, as must its output order
truncated at any K.
"""
import numpy as np
import pytest

import oracle
from paper_2508_20403_amd import synth

GRAPHS = [
    lambda s: synth.random_connected(50, 90, seed=s, alpha=0.3, beta=2),
    lambda s: synth.random_connected(70, 150, seed=s, alpha=0.4, beta=1, tree="random"),
    lambda s: synth.grid((9, 8), 1.0, 100.0, seed=s, alpha=0.3, beta=2),
    lambda s: synth.path_graph(40, 60, seed=s, alpha=0.5, beta=2),
    lambda s: synth.star_graph(30, 50, seed=s, alpha=0.5, beta=1),
]


def _ancestors(parent, x, c):
    out = []
    for _ in range(c + 1):
        out.append(int(x))
        x = parent[x] if x >= 0 else -1
    return out


def _cells(anc_pair, c):
    """(z, j) cells an edge reads: j <= c - i over the i-th ancestors z of both endpoints."""
    return [(z, j) for side in anc_pair for i, z in enumerate(side) if z >= 0 for j in range(c + 1 - i)]


def _rounds_pass(ranked, anc, n, c):
    """Decides the edges of one pass (rank order); returns the recovered ones and the rounds."""
    P = len(ranked)
    state = np.zeros(P, np.int8)  # 0 undecided, 1 recovered, 2 marked
    covered = np.zeros((n, c + 1), bool)
    rounds = 0
    while (state == 0).any():
        rounds += 1
        und = np.nonzero(state == 0)[0]
        low = np.full((n, c + 1), P, np.int64)
        for p in und:
            for side in anc[p]:
                for i, z in enumerate(side):
                    if z >= 0:
                        low[z, i] = min(low[z, i], p)
        new = [p for p in und if min(low[z, j] for z, j in _cells(anc[p], c)) == p]
        assert new, "a round must decide the lowest undecided rank"
        for p in new:
            state[p] = 1
            for side in anc[p]:
                for i, z in enumerate(side):
                    if z >= 0:
                        covered[z, i] = True
        for p in und:
            if state[p] == 0 and any(covered[z, j] for z, j in _cells(anc[p], c)):
                state[p] = 2
    return [ranked[p] for p in range(P) if state[p] == 1], rounds


def _rounds_all_passes(g, o, c):
    off = np.nonzero(o.is_tree == 0)[0]
    ranked = list(off[np.argsort(o.rank_of[off], kind="stable")])
    parent = np.asarray(g.parent)
    pass_of = np.zeros(o.m, np.int64)
    order, p = [], 0
    while ranked:
        p += 1
        anc = [(_ancestors(parent, o.eu[e], c), _ancestors(parent, o.ev[e], c)) for e in ranked]
        rec, _ = _rounds_pass(ranked, anc, g.n, c)
        for e in rec:
            pass_of[e] = p
        order += rec
        taken = set(rec)
        ranked = [e for e in ranked if e not in taken]
    return pass_of, order


@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("seed", [0, 1])
@pytest.mark.parametrize("c", [0, 1, 2, 4])
def test_rounds_reach_the_serial_passes(make, seed, c):
    g = make(seed)
    o = oracle.recover(g, beta=c, k_override=g.m, loose=True, full=True)
    assert o.ok
    pass_of, order = _rounds_all_passes(g, o, c)
    np.testing.assert_array_equal(o.pass_of.astype(np.int64), pass_of)
    M = int(np.sum(o.is_tree == 0))
    for K in (1, 5, M // 3, M):
        ok = oracle.recover(g, beta=c, k_override=K, loose=True)
        assert list(ok.order[: ok.info["n_recovered"]]) == order[:K]


def test_rounds_can_be_many():
    """On a path whose off-tree edges conflict only with their neighbours in rank order,
    each round settles about two edges: the rounds are not bounded by a constant."""
    # chords (i, i + 2) along the path; weights descending along it, so ranks follow i
    n = 60
    eu = np.concatenate([np.arange(n - 1), np.arange(n - 2)])
    ev = np.concatenate([np.arange(1, n), np.arange(2, n)])
    w = np.concatenate([np.full(n - 1, 1e6), 1000.0 - np.arange(n - 2)])
    parent = np.concatenate([[-1], np.arange(n - 1)]).astype(np.int32)
    g = synth.from_edges(n, eu, ev, w, 0.5, 0, "chords60", parent=parent, root=0)
    o = oracle.recover(g, beta=0, k_override=g.m, loose=True, full=True)
    off = np.nonzero(o.is_tree == 0)[0]
    ranked = list(off[np.argsort(o.rank_of[off], kind="stable")])
    anc = [(_ancestors(parent, o.eu[e], 0), _ancestors(parent, o.ev[e], 0)) for e in ranked]
    rec, rounds = _rounds_pass(ranked, anc, n, 0)
    assert rec == [e for e in ranked if o.pass_of[e] == 1]
    assert rounds >= len(ranked) // 4
