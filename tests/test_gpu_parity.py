"""GPU path vs the serial oracle, element by element (bit-exact).

Inputs are seeded and synthetic.  Small graphs span several 64-wide blocks, Euler
blocks and hash tiles and end in ragged tails; the named workloads are the full
64x64 grid and the 128^3 grid.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_20403_amd import gss, synth
from tests.gpu_util import assert_same_recovery, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

SMALL = [
    ("rand_max", lambda s: synth.random_connected(300, 900, seed=s, alpha=0.1, beta=2)),
    ("rand_tree", lambda s: synth.random_connected(517, 1400, seed=s, alpha=0.2, beta=3, tree="random")),
    ("path", lambda s: synth.path_graph(200, 300, seed=s, alpha=0.5, beta=2)),
    ("star", lambda s: synth.star_graph(150, 400, seed=s, alpha=0.5, beta=2)),
    ("grid", lambda s: synth.grid((23, 17), 1.0, 100.0, seed=s, alpha=0.1, beta=2)),
]


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("seed", [0, 1])
def test_tree_prep_matches_oracle(gpu_ctx, name, make, seed):
    g = make(seed)
    orc = run_oracle(g)
    tree = gss.Tree.from_graph(gpu_ctx, g)
    depth, dlo, dhi, scale = tree.export()
    np.testing.assert_array_equal(depth.cpu().numpy(), orc.depth)
    np.testing.assert_array_equal(dlo.cpu().numpy().view(np.uint64), orc.Dlo)
    np.testing.assert_array_equal(dhi.cpu().numpy().view(np.uint64), orc.Dhi)
    assert scale == orc.info["scale"]
    for beta in (0, 1, 2, 5):
        lca, bstar = tree.edge_lca(beta)
        o2 = run_oracle(g, beta=beta)
        np.testing.assert_array_equal(lca.cpu().numpy(), o2.lca)
        np.testing.assert_array_equal(bstar.cpu().numpy(), o2.bstar)
    tree.free()


# Graphs whose rows cross the 4096-entry tiles of the CSR passes in every way the child
# lists are built: a hub row spanning several tiles (its children linked as one segment
# per tile), tiles of more than 1024 short rows (rows past the tracked ones linked per
# child), and rows that straddle tile boundaries.
MULTI_TILE = [
    ("big_star", lambda: synth.star_graph(12000, 3000, seed=4, alpha=0.05, beta=2)),
    ("long_path", lambda: synth.path_graph(12000, 800, seed=5, alpha=0.2, beta=2)),
    ("rmat14", lambda: synth.config("rmat14")),
    ("grid3d", lambda: synth.grid((30, 20, 25), 1.0, 1e4, seed=6, alpha=0.1, beta=2)),
]


@pytest.mark.parametrize("name,make", MULTI_TILE, ids=[s[0] for s in MULTI_TILE])
def test_tree_prep_multi_tile_matches_oracle(gpu_ctx, name, make):
    g = make()
    orc = run_oracle(g)
    tree = gss.Tree.from_graph(gpu_ctx, g)
    depth, dlo, dhi, scale = tree.export()
    np.testing.assert_array_equal(depth.cpu().numpy(), orc.depth)
    np.testing.assert_array_equal(dlo.cpu().numpy().view(np.uint64), orc.Dlo)
    np.testing.assert_array_equal(dhi.cpu().numpy().view(np.uint64), orc.Dhi)
    lca, bstar = tree.edge_lca(2)
    np.testing.assert_array_equal(lca.cpu().numpy(), orc.lca)
    np.testing.assert_array_equal(bstar.cpu().numpy(), orc.bstar)
    tree.free()
    assert_same_recovery(run_gpu(gpu_ctx, g), orc)


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_recover_small(gpu_ctx, name, make, seed):
    g = make(seed)
    for beta in (0, 1, 2, 4):
        for k in (-1, 1, 7, g.m):  # k=m forces extra passes and a short result
            gpu = run_gpu(gpu_ctx, g, beta=beta, k_override=k)
            orc = run_oracle(g, beta=beta, k_override=k)
            assert_same_recovery(gpu, orc)


def test_recover_grid2d_64(gpu_ctx):
    g = synth.config("grid2d_64")
    gpu = run_gpu(gpu_ctx, g)
    orc = run_oracle(g)
    assert gpu["info"]["k"] == 81 and orc.info["n_offtree"] == 3969
    assert_same_recovery(gpu, orc)


def test_recover_grid3d_128(gpu_ctx):
    g = synth.config("grid3d_128")
    gpu = run_gpu(gpu_ctx, g)
    orc = run_oracle(g)
    assert gpu["info"]["n_subtasks"] == orc.info["n_subtasks"]
    assert gpu["info"]["largest_subtask"] == orc.info["largest_subtask"]
    assert_same_recovery(gpu, orc)


def test_recover_rmat14(gpu_ctx):
    g = synth.config("rmat14")
    for beta in (1, 2):
        gpu = run_gpu(gpu_ctx, g, beta=beta)
        orc = run_oracle(g, beta=beta)
        assert_same_recovery(gpu, orc)


@pytest.mark.parametrize("beta", [3, 5, 8])
def test_recover_large_beta(gpu_ctx, beta):
    """Every BFS-step constant c has its own work-queue and join-record kernels; c = 8 is
    the largest accepted (and feGRASS's default).  Small graphs (with forced extra passes),
    a 40^3 grid whose large subtasks take the join, and R-MAT with hub subtasks."""
    for name, make in SMALL:
        g = make(0)
        for k in (-1, g.m):
            assert_same_recovery(run_gpu(gpu_ctx, g, beta=beta, k_override=k),
                                 run_oracle(g, beta=beta, k_override=k))
    for g in (synth.grid((40, 40, 40), 1.0, 1e4, seed=3, alpha=0.05, beta=beta), synth.config("rmat14")):
        gpu = run_gpu(gpu_ctx, g, beta=beta)
        assert gpu["info"]["n_join"] > 0  # the partitioned join ran
        assert_same_recovery(gpu, run_oracle(g, beta=beta))


@pytest.mark.parametrize("name,make", SMALL[:3], ids=[s[0] for s in SMALL[:3]])
def test_trusted_prep_matches_oracle(gpu_ctx, name, make):
    """GSS_PREP_TRUSTED skips the input checks (the edge count comes from the row scan
    instead of nnz / 2); the recovery must not change."""
    g = make(1)
    dev = torch.device("cuda:0")
    arrays = [torch.from_numpy(a).to(dev) for a in (g.row_ptr, g.col, g.w, g.parent)]
    tree = gss.Tree(gpu_ctx, *arrays, trusted=True)
    assert tree.m == g.m
    st, mask, order, stretch, info = tree.recover(g.alpha, g.beta, want_stretch=True)
    torch.cuda.synchronize()
    gpu = dict(status=st, mask=mask.cpu().numpy(), order=order.cpu().numpy(),
               stretch=stretch.cpu().numpy(), info=info)
    tree.free()
    assert_same_recovery(gpu, run_oracle(g))


@pytest.mark.parametrize("make", [lambda: synth.grid((40, 40, 40), 1.0, 1e4, seed=3, alpha=0.05, beta=2),
                                  lambda: synth.random_connected(60000, 90000, seed=2, alpha=0.05, beta=2,
                                                                 tree="random")],
                         ids=["grid40", "rand60000"])
def test_rank_capacity_retry_matches_oracle(gpu_ctx, make):
    """The list ranking's capacity retry: with the first attempt's level capacities cut
    to a quarter, levels outgrow them, the device flags it and the host ranks again with
    twice and then four times the capacities (three attempts).  The prepared tree and
    the recovery must still equal the oracle's bit for bit; with the default capacities
    one attempt suffices."""
    g = make()
    orc = run_oracle(g)
    for divisor, attempts in ((4, 3), (1, 1)):
        gpu_ctx.set_rank_capacity(divisor)
        try:
            tree = gss.Tree.from_graph(gpu_ctx, g)
        finally:
            gpu_ctx.set_rank_capacity(1)
        assert tree.rank_attempts() == attempts
        depth, dlo, dhi, scale = tree.export()
        np.testing.assert_array_equal(depth.cpu().numpy(), orc.depth)
        np.testing.assert_array_equal(dlo.cpu().numpy().view(np.uint64), orc.Dlo)
        np.testing.assert_array_equal(dhi.cpu().numpy().view(np.uint64), orc.Dhi)
        st, mask, order, stretch, info = tree.recover(g.alpha, g.beta, want_stretch=True)
        torch.cuda.synchronize()
        gpu = dict(status=st, mask=mask.cpu().numpy(), order=order.cpu().numpy(), stretch=stretch.cpu().numpy(),
                   info=info)
        assert_same_recovery(gpu, orc)
        tree.free()


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_rt_key_matches_oracle(gpu_ctx, name, make):
    """GSS_F_KEY_RT (order by R_T alone): mask, order and stretch bit for bit against the
    oracle's R_T-key variant, including forced extra passes and short results."""
    g = make(3)
    for beta in (1, 2):
        for k in (-1, 7, g.m):
            gpu = run_gpu(gpu_ctx, g, beta=beta, k_override=k, key_rt=True)
            orc = run_oracle(g, beta=beta, k_override=k, key_rt=True)
            assert_same_recovery(gpu, orc)


@pytest.mark.parametrize("name", ["grid3d_32", "rmat14"])
def test_rt_key_named_workloads(gpu_ctx, name):
    g = synth.config(name)
    assert_same_recovery(run_gpu(gpu_ctx, g, key_rt=True), run_oracle(g, key_rt=True))
