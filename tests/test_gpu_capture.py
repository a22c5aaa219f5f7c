"""Memoized graph capture of recoveries (gss_ctx_set_capture): the first call with a key
records, the second captures a HIP graph and launches it, later calls replay it with one
host synchronisation.  Every call's outputs must equal the oracle's, bit for bit; the
counters must show the record / capture / replay sequence; a changed key, a freed tree
and a disabled capture must fall back to eager calls.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_20403_amd import gss, synth
from tests.test_gpu_batch import small_batch

pytestmark = pytest.mark.gpu


def _delta(a, b):
    return {k: b[k] - a[k] for k in a}


@pytest.fixture
def cap_ctx():
    ctx = gss.Context(0)
    ctx.set_capture(True)
    yield ctx
    ctx.close()


@pytest.mark.parametrize("name,make,beta,loose", [
    ("grid3d_32", lambda: synth.config("grid3d_32"), 2, False),
    ("rmat14", lambda: synth.config("rmat14"), 2, False),
    ("rand_multipass", lambda: synth.random_connected(3000, 4000, seed=3, alpha=0.5, beta=2), 2, False),
    ("grid_loose", lambda: synth.grid((60, 50), 1.0, 100.0, seed=1, alpha=0.1, beta=3), 3, True),
])
def test_single_graph_replays_match_oracle(cap_ctx, name, make, beta, loose):
    g = make()
    k = g.m if name == "rand_multipass" else -1  # more than the off-tree edges: several passes, short
    ref = oracle.recover(g, beta=beta, k_override=k, loose=loose, full=True)
    nrec = ref.info["n_recovered"]
    tree = gss.Tree.from_graph(cap_ctx, g)
    K = tree.target_count(g.alpha, k)
    dev = torch.device("cuda")
    out = (torch.empty(g.m, dtype=torch.uint8, device=dev), torch.empty(max(K, 1), dtype=torch.int32, device=dev),
           torch.empty(g.m, dtype=torch.float64, device=dev))
    before = cap_ctx.capture_stats()
    for call in range(4):
        s0 = cap_ctx.capture_stats()
        out[0].fill_(7)  # stale outputs must be overwritten by every form of the call
        out[1].fill_(-5)
        st, mask, order, stretch, info = tree.recover(g.alpha, beta, k_override=k, out=out, loose=loose)
        torch.cuda.synchronize()
        d = _delta(s0, cap_ctx.capture_stats())
        print(f"[capture] {name} call {call}: {d} {cap_ctx.lib.gss_last_error(cap_ctx.handle).decode()}", flush=True)
        assert st == ref.status
        assert info["n_recovered"] == nrec and info["passes"] == ref.info["passes"]
        np.testing.assert_array_equal(mask.cpu().numpy(), ref.mask)
        np.testing.assert_array_equal(order.cpu().numpy()[:nrec], ref.order[:nrec])
        np.testing.assert_array_equal(stretch.cpu().numpy().view(np.uint64), ref.stretch.view(np.uint64))
        if call >= 2:
            assert d["replays"] == 1 and d["syncs"] <= 2, d
    d = _delta(before, cap_ctx.capture_stats())
    assert (d["records"], d["captures"], d["replays"]) == (1, 1, 2), d
    tree.free()


def test_batch_replays_match_oracle(cap_ctx):
    graphs = small_batch(1)
    refs = [oracle.recover(g) for g in graphs]
    b = gss.Batch(cap_ctx, graphs)
    dev = torch.device("cuda")
    Ks = b.target_counts([g.alpha for g in graphs])
    masks = [torch.empty(max(g.m, 1), dtype=torch.uint8, device=dev) for g in graphs]
    orders = [torch.empty(max(k, 1), dtype=torch.int32, device=dev) for k in Ks]
    before = cap_ctx.capture_stats()
    for call in range(3):
        for m in masks:
            m.fill_(9)
        st, mk, od, infos = b.recover(out=(masks, orders))
        torch.cuda.synchronize()
        for g, ref, m, o, inf in zip(graphs, refs, mk, od, infos):
            nrec = ref.info["n_recovered"]
            assert inf["n_recovered"] == nrec and inf["passes"] == ref.info["passes"]
            np.testing.assert_array_equal(m.cpu().numpy(), ref.mask)
            np.testing.assert_array_equal(o.cpu().numpy()[:nrec], ref.order[:nrec])
    d = _delta(before, cap_ctx.capture_stats())
    assert (d["records"], d["captures"], d["replays"]) == (1, 1, 1), d
    # a different key (another alpha) records again; the first key still replays
    s0 = cap_ctx.capture_stats()
    b.recover(alphas=[min(1.0, g.alpha * 2) for g in graphs])
    b.recover(out=(masks, orders))
    d = _delta(s0, cap_ctx.capture_stats())
    assert d["records"] == 1 and d["replays"] == 1, d
    b.free()
    # freeing the tree dropped its graphs: a new batch over the same graphs starts over
    b2 = gss.Batch(cap_ctx, graphs)
    s0 = cap_ctx.capture_stats()
    b2.recover(out=(masks, orders))
    assert _delta(s0, cap_ctx.capture_stats())["records"] == 1
    b2.free()


def test_capture_off_runs_eagerly(cap_ctx):
    g = synth.config("grid3d_32")
    ref = oracle.recover(g)
    tree = gss.Tree.from_graph(cap_ctx, g)
    K = tree.target_count(g.alpha)
    out = (torch.empty(g.m, dtype=torch.uint8, device="cuda"), torch.empty(K, dtype=torch.int32, device="cuda"), None)
    tree.recover(g.alpha, g.beta, out=out)
    tree.recover(g.alpha, g.beta, out=out)
    cap_ctx.set_capture(False)
    s0 = cap_ctx.capture_stats()
    for _ in range(2):
        _, mask, order, _, _ = tree.recover(g.alpha, g.beta, out=out)
        np.testing.assert_array_equal(mask.cpu().numpy(), ref.mask)
        np.testing.assert_array_equal(order.cpu().numpy(), ref.order)
    d = _delta(s0, cap_ctx.capture_stats())
    assert (d["records"], d["captures"], d["replays"]) == (0, 0, 0), d
    tree.free()
