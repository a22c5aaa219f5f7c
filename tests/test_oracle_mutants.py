"""Planted mistakes: each mutated copy of the oracle (built on the CPU in a temp dir)
must fail at least one pin.  Shows the pins would catch a dropped term, a wrong sign or
direction, a transposed operand or a wrong radius."""
import os

import numpy as np
import pytest

import oracle
from oracle import oracle as orc_mod
from paper_2508_20403_amd import synth
from tests import brute
from tests.test_oracle_pins import GOLDEN, graph_from_json

MUTANTS = {
    "loose_condition": ("(b->stampU[x] == b->cur && b->stampV[y] == b->cur) ||",
                        "(b->stampU[x] == b->cur || b->stampV[y] == b->cur) ||"),
    "loose_indexed": ("if (r->is_tree[f] || other[r->col[k]] != b->cur) continue;",
                      "if (r->is_tree[f]) continue;"),
    "beta_ignores_depth": ("if (r->c < b) b = r->c;", "b = r->c;"),
    "ascending_order": ("if (sa > sb) return -1;\n    if (sa < sb) return 1;",
                        "if (sa < sb) return -1;\n    if (sa > sb) return 1;"),
    "ties_by_id_desc": ("return (a < b) ? -1 : (a > b);", "return (a > b) ? -1 : (a < b);"),
    "dropped_lca_term": ("u128 Rfix = (r->D[u] - r->D[l]) + (r->D[v] - r->D[l]);",
                         "u128 Rfix = (r->D[u] - r->D[l]) + r->D[v];"),
    "no_weight_in_stretch": ("double s = r->ew[e] * R;", "double s = R;"),
    "ball_radius_plus_one": ("if (d == radius) continue;", "if (d == radius + 1) continue;"),
    "marks_not_cleared": ("        memset(marked, 0, (size_t)r->m + 1);\n        int64_t got = 0;",
                          "        int64_t got = 0;"),
    "lca_one_sided_lift": ("if (r->up[k][a] != r->up[k][b]) { a = r->up[k][a]; b = r->up[k][b]; }",
                           "if (r->up[k][a] != r->up[k][b]) { a = r->up[k][a]; }"),
}


def pins_pass(lib):
    """A compact battery of the pins; False as soon as one fails."""
    import json
    spec = json.load(open(os.path.join(GOLDEN, "noncommutative.json")))
    for case in spec["cases"]:
        edges = [[a, b, 1.0] for a, b in spec["tree_edges"]] + [[3, 5, case["w_e"]], [1, 2, case["w_eprime"]]]
        g = graph_from_json(spec["n"], edges, spec["parent"], beta=case["c"])
        for mode in (oracle.MODE_INDEXED, oracle.MODE_BRUTE):
            r = oracle.recover(g, k_override=case["k"], mode=mode, lib=lib)
            if r.order_list().tolist() != case["order"] or r.info["passes"] != case["passes"]:
                return False
    # unit weights: many equal stretches, so the id tie-break decides the order
    gt = synth.grid((5, 7), 1.0, 1.0, seed=0)
    for c in (0, 2):
        for k in (5, 20):
            ref_order, _ = brute.greedy_brute(gt, c, k)
            if oracle.recover(gt, beta=c, k_override=k, lib=lib).order_list().tolist() != ref_order:
                return False
    for s in range(4):
        g = synth.random_connected(24 + 4 * s, 40 + 8 * s, seed=500 + s, tree="random" if s % 2 else "max")
        M = g.m - (g.n - 1)
        for c in (1, 2):
            ref = brute.stretch_exact(g, c)
            r = oracle.recover(g, beta=c, full=True, lib=lib)
            for e, (st, l, b) in ref.items():
                if r.stretch[e] != st or r.lca[e] != l or r.bstar[e] != b:
                    return False
            for k in (max(1, M // 2), M):
                ref_order, ref_passes = brute.greedy_brute(g, c, k)
                for mode in (oracle.MODE_INDEXED, oracle.MODE_BRUTE):
                    r = oracle.recover(g, beta=c, k_override=k, mode=mode, lib=lib)
                    if r.order_list().tolist() != ref_order or r.info["passes"] != ref_passes:
                        return False
    return True


def test_unmutated_oracle_passes_battery():
    assert pins_pass(oracle.load())


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    src = open(orc_mod.SRC).read()
    old, new = MUTANTS[name]
    assert src.count(old) >= 1, name
    lib = orc_mod.build_variant(src.replace(old, new, 1), str(tmp_path / f"mut_{name}.so"))
    assert not pins_pass(lib), f"mutation {name} was not caught"
