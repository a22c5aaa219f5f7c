"""GPU spanning tree (gss_spanning_tree: feGRASS's effective-weight tree, and the plain
maximum-weight tree) against the oracle's, element by element: the root, the ordering
weight of every edge (bit for bit) and the parent array.  Then the whole sparsifier built
on the GPU (tree and recovery) against the oracle run on the same tree.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_20403_amd import gss, synth
from tests.gpu_util import assert_same_recovery, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

GRAPHS = [
    ("grid2d", lambda: synth.grid((23, 17), 1.0, 100.0, seed=1)),
    ("grid3d", lambda: synth.grid((12, 9, 7), 1.0, 1e4, seed=2)),
    ("unit_ties", lambda: synth.random_connected(3000, 6000, seed=3, wlo=1.0, whi=1.0)),
    ("random", lambda: synth.random_connected(5000, 12000, seed=4)),
    ("star", lambda: synth.star_graph(400, 900, seed=5)),
    ("path", lambda: synth.path_graph(2000, 100, seed=6)),
    ("rmat12", lambda: synth.rmat(12, seed=7)),
    ("rgg", lambda: synth.rgg(20000, np.random.default_rng(8))),
    ("single", lambda: synth.from_edges(1, np.array([], int), np.array([], int), np.array([]), 0.5, 2, "one",
                                        parent=np.array([-1], np.int32), root=0)),
    ("edge", lambda: synth.from_edges(2, np.array([0]), np.array([1]), np.array([2.0]), 0.5, 2, "two")),
]


def _gpu_tree(ctx, g, plain):
    dev = torch.device("cuda")
    rp, col, w = (torch.from_numpy(a).to(dev) for a in (g.row_ptr, g.col, g.w))
    parent, root, weff = ctx.spanning_tree(rp, col, w, weight=plain, want_weff=True)
    torch.cuda.synchronize()
    return parent.cpu().numpy(), root, weff.cpu().numpy()


@pytest.mark.parametrize("name,make", GRAPHS, ids=[x[0] for x in GRAPHS])
@pytest.mark.parametrize("plain", [False, True], ids=["weff", "plain"])
def test_spanning_tree_matches_oracle(gpu_ctx, name, make, plain):
    g = make()
    print(f"[treegen] {name} n={g.n} m={g.m} {'plain' if plain else 'weff'}", flush=True)
    parent, root, weff = _gpu_tree(gpu_ctx, g, plain)
    ref_parent, ref_root, ref_weff, _ = oracle.spanning_tree(g, plain=plain)
    assert root == ref_root
    np.testing.assert_array_equal(weff[: g.m].view(np.uint64), ref_weff.view(np.uint64))
    np.testing.assert_array_equal(parent, ref_parent)


@pytest.mark.parametrize("name", ["grid3d", "rmat12", "unit_ties"])
def test_sparsifier_on_the_gpu_tree(gpu_ctx, name):
    """The whole sparsifier on the GPU: feGRASS's tree, then the recovery on it, against the
    oracle's recovery on the oracle's tree (the same tree, checked above)."""
    g = dict(GRAPHS)[name]()
    parent, root, _ = _gpu_tree(gpu_ctx, g, False)
    g2 = synth.Graph(g.n, g.row_ptr, g.col, g.w, parent, root, 0.1, 2, g.name + "_feGRASS_tree")
    assert_same_recovery(run_gpu(gpu_ctx, g2), run_oracle(g2))


def test_full_size_tree_matches_oracle(gpu_ctx):
    g = synth.config("grid3d_128")
    parent, root, weff = _gpu_tree(gpu_ctx, g, False)
    ref_parent, ref_root, ref_weff, _ = oracle.spanning_tree(g)
    assert root == ref_root
    np.testing.assert_array_equal(weff[: g.m].view(np.uint64), ref_weff.view(np.uint64))
    np.testing.assert_array_equal(parent, ref_parent)


def test_errors(gpu_ctx):
    dev = torch.device("cuda")
    # two components
    g = synth.from_edges(4, np.array([0, 2]), np.array([1, 3]), np.array([1.0, 1.0]), 0.5, 2, "two",
                         parent=np.array([-1, 0, -1, 2], np.int32), root=None)
    rp, col, w = (torch.from_numpy(a).to(dev) for a in (g.row_ptr, g.col, g.w))
    with pytest.raises(gss.GSSError) as e:
        gpu_ctx.spanning_tree(rp, col, w)
    assert e.value.status == -1
    # a column out of range (rejected before the search reads it)
    bad = col.clone()
    bad[0] = 7
    with pytest.raises(gss.GSSError) as e:
        gpu_ctx.spanning_tree(rp, bad, w)
    assert e.value.status == -1
