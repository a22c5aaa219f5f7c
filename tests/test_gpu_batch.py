"""Batched recovery: every graph of a batch must match its own oracle run, bit-exact."""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_20403_amd import gss, synth

pytestmark = pytest.mark.gpu


def small_batch(seed=0, count=12):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(np.exp(rng.uniform(np.log(200), np.log(6000))))
        alpha = float(rng.choice([0.02, 0.05, 0.10, 0.5]))
        kind = i % 4
        if kind == 0:
            g = synth.rgg(n, rng, alpha, 2, f"rgg{i}")
        elif kind == 1:
            g = synth.random_connected(n, 2 * n, seed=seed * 100 + i, alpha=alpha, beta=2, tree="random")
        elif kind == 2:
            g = synth.grid((int(np.sqrt(n)), int(np.sqrt(n)) + 3), 1.0, 100.0, seed=i, alpha=alpha, beta=2)
        else:
            g = synth.random_connected(max(n // 4, 3), 0, seed=i, alpha=alpha, beta=2)  # a tree: M = 0
        out.append(g)
    return out


@pytest.mark.parametrize("seed", [0, 1])
def test_batch_matches_per_graph_oracle(gpu_ctx, seed):
    graphs = small_batch(seed)
    print(f"[gpu-batch] seed {seed}: sizes {[g.n for g in graphs]}", flush=True)
    b = gss.Batch(gpu_ctx, graphs)
    st, masks, orders, infos = b.recover(stats=True)
    torch.cuda.synchronize()
    for g, mk, od, inf in zip(graphs, masks, orders, infos):
        ref = oracle.recover(g)
        nrec = ref.info["n_recovered"]
        assert inf["n_recovered"] == nrec and inf["k"] == ref.K
        assert inf["passes"] == ref.info["passes"]
        assert inf["n_subtasks"] == ref.info["n_subtasks"]
        np.testing.assert_array_equal(mk.cpu().numpy(), ref.mask)
        np.testing.assert_array_equal(od.cpu().numpy()[:nrec], ref.order[:nrec])
    b.free()


@pytest.mark.parametrize("split", ["median", "all_own", "one_left"])
def test_batch_split_matches_per_graph_oracle(gpu_ctx, split):
    """Graphs at or above the batch split size are prepared and recovered on their own,
    the rest share the union; every graph still matches its oracle run, the schedule
    (edge count or learned) does not matter, and infos map back to the right graphs."""
    graphs = small_batch(2)
    nnz = sorted(len(g.col) for g in graphs)
    limit = {"median": nnz[len(nnz) // 2], "all_own": 0, "one_left": nnz[1]}[split]
    print(f"[gpu-batch] split {split}: limit {limit}, nnz {nnz}", flush=True)
    gpu_ctx.set_batch_split(limit)
    try:
        b = gss.Batch(gpu_ctx, graphs)
    finally:
        gpu_ctx.set_batch_split(1 << 25)
    assert [gss_m for gss_m in b.m] == [g.m for g in graphs]
    st, masks, orders, infos = b.recover(stats=True)
    torch.cuda.synchronize()
    for g, mk, od, inf in zip(graphs, masks, orders, infos):
        ref = oracle.recover(g)
        nrec = ref.info["n_recovered"]
        assert inf["n_recovered"] == nrec and inf["k"] == ref.K and inf["m"] == g.m
        assert inf["n_subtasks"] == ref.info["n_subtasks"]
        np.testing.assert_array_equal(mk.cpu().numpy(), ref.mask)
        np.testing.assert_array_equal(od.cpu().numpy()[:nrec], ref.order[:nrec])
    b.free()


def test_batch_of_one_equals_single(gpu_ctx):
    g = synth.config("grid3d_32")
    b = gss.Batch(gpu_ctx, [g])
    _, masks, orders, _ = b.recover()
    ref = oracle.recover(g)
    np.testing.assert_array_equal(masks[0].cpu().numpy(), ref.mask)
    np.testing.assert_array_equal(orders[0].cpu().numpy(), ref.order)
    b.free()


def test_batch_multi_pass_and_short(gpu_ctx):
    graphs = [synth.random_connected(300, 400, seed=s, alpha=0.5, beta=2) for s in range(5)]
    ks = [g.m for g in graphs]  # more than the off-tree edges: several passes, short result
    b = gss.Batch(gpu_ctx, graphs)
    st, masks, orders, infos = b.recover(k_override=ks)
    assert st == gss.GSS_SHORT
    for g, k, mk, od, inf in zip(graphs, ks, masks, orders, infos):
        ref = oracle.recover(g, k_override=k)
        nrec = ref.info["n_recovered"]
        assert inf["passes"] == ref.info["passes"] and inf["n_recovered"] == nrec
        np.testing.assert_array_equal(od.cpu().numpy()[:nrec], ref.order[:nrec])
        np.testing.assert_array_equal(mk.cpu().numpy(), ref.mask)
    b.free()


def test_batch_rejects_bad_graph(gpu_ctx):
    graphs = small_batch(3, 4)
    bad = graphs[2]
    par = bad.parent.copy()
    x = int(np.flatnonzero(par >= 0)[0])
    par[x] = -1  # two roots in one graph (the union alone would hide it)
    graphs[2] = synth.Graph(bad.n, bad.row_ptr, bad.col, bad.w, par, bad.root, bad.alpha, bad.beta, "bad")
    with pytest.raises(gss.GSSError) as e:
        gss.Batch(gpu_ctx, graphs)
    assert e.value.status == -5
