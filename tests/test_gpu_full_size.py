"""Full-size workloads vs the oracle, bit for bit, through stored digests.

The serial oracle needs minutes on these graphs, so tests/golden/make_full_size.py ran
it once per workload (same seeded generators) and stored SHA-256 digests of its
recovered-edge mask, recovery order and stretch array together with its counters.  Here
the GPU path runs in the configuration the benchmark times (default flags) and its
outputs must hash to the same digests; a second run with GSS_F_STATS checks the subtask
counters.

The learned schedule is checked at full size too: on the learned-scheduling pair
(R-MAT scale 24 and the 160^3 grid) the plain kernel records per-subtask cycles, the
cost model trains on them on the GPU, and the recovery with the learned queue order must
hash to the same digests (the schedule may change only the speed).  The same holds for
the 64-graph batch with the autotuned work-queue settings.
"""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

from paper_2508_20403_amd import gss, synth

pytestmark = pytest.mark.gpu

GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "full_size.json")
GOLD = json.load(open(GOLD_PATH)) if os.path.exists(GOLD_PATH) else {}

# graphs generated once per session and shared by the tests below that need them
_CACHE = {}
_KEEP = ("grid3d_160", "rmat24")  # the learned-scheduling pair, used again by the last test


def sha(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def _graph(name):
    if name not in _CACHE:
        print(f"[full] generating {name}", flush=True)
        _CACHE[name] = synth.config(name)
    return _CACHE[name]


def _check_digests(ref, st, mask, order, stretch, info):
    nrec = info["n_recovered"]
    assert st == ref["status"]
    assert (info["n_offtree"], info["k"], nrec, info["passes"]) == \
        (ref["n_offtree"], ref["k"], ref["n_recovered"], ref["passes"])
    order_h = order.cpu().numpy()[:nrec]
    assert [int(x) for x in order_h[:16]] == ref["order_head"]
    assert sha(order_h, "<i4") == ref["order_sha256"]
    assert sha(mask.cpu().numpy(), np.uint8) == ref["mask_sha256"]
    if stretch is not None:
        assert sha(stretch.cpu().numpy().view(np.uint64), "<u8") == ref["stretch_sha256"]


@pytest.mark.timeout(900)  # generating R-MAT scale 24 on the host takes minutes
@pytest.mark.parametrize("name", ["grid3d_160", "rmat22", "rmat24"])
def test_full_size_matches_oracle(gpu_ctx, name):
    if name not in GOLD:
        pytest.skip(f"no stored oracle result for {name}")
    ref = GOLD[name]
    g = _graph(name)
    assert (g.n, g.m) == (ref["n"], ref["m"])
    print(f"[full] {name} n={g.n} m={g.m}: GPU recovery", flush=True)
    tree = gss.Tree.from_graph(gpu_ctx, g)
    st, mask, order, stretch, info = tree.recover(g.alpha, g.beta, want_stretch=True)
    torch.cuda.synchronize()
    _check_digests(ref, st, mask, order, stretch, info)
    _, _, _, _, info2 = tree.recover(g.alpha, g.beta, stats=True)
    assert (info2["n_subtasks"], info2["largest_subtask"]) == (ref["n_subtasks"], ref["largest_subtask"])
    tree.free()
    if name not in _KEEP:
        _CACHE.pop(name, None)


@pytest.mark.timeout(900)
def test_learned_schedule_full_size_matches_oracle(gpu_ctx):
    """R-MAT scale 24 + 3D grid 160^3 (alpha 0.10): cycles recorded by the plain kernel on
    both graphs train one cost model (FP32 kernels); with the learned queue order both
    recoveries hash to the oracle's digests, and the info record says the learned order
    ran."""
    names = [n for n in _KEEP if n in GOLD]
    if len(names) < 2:
        pytest.skip("no stored oracle results for the learned-scheduling pair")
    ctx = gss.Context(0)
    try:
        trees = {}
        for name in names:
            g = _graph(name)
            print(f"[full] {name}: recording subtask cycles", flush=True)
            trees[name] = gss.Tree.from_graph(ctx, g)
            trees[name].recover(g.alpha, g.beta, record=True)
        feat, cyc, size = ctx.trace_read()
        ctx.trace_clear()
        print(f"[full] training the cost model on {len(cyc)} recorded subtasks", flush=True)
        assert len(cyc) >= 1000
        loss = ctx.costmodel_train(feat, cyc, epochs=5, lr=1e-3, seed=0)
        assert np.all(np.isfinite(loss))
        for name in names:
            g = _graph(name)
            print(f"[full] {name}: learned-schedule recovery", flush=True)
            st, mask, order, stretch, info = trees[name].recover(g.alpha, g.beta, sched=gss.SCHED_LEARNED,
                                                                 want_stretch=True)
            torch.cuda.synchronize()
            assert info["sched"] == gss.SCHED_LEARNED
            _check_digests(GOLD[name], st, mask, order, stretch, info)
            trees[name].free()
    finally:
        ctx.close()
        for name in _KEEP:
            _CACHE.pop(name, None)


def _batch_digests(ref, infos, masks, orders):
    for i, (r, info) in enumerate(zip(ref, infos)):
        nrec = info["n_recovered"]
        assert (info["k"], nrec, info["passes"]) == (r["k"], r["n_recovered"], r["passes"]), i
        assert sha(orders[i].cpu().numpy()[:nrec], "<i4") == r["order_sha256"], i
        assert sha(masks[i].cpu().numpy()[:r["m"]], np.uint8) == r["mask_sha256"], i


@pytest.mark.timeout(900)
def test_full_batch_matches_oracle(gpu_ctx):
    """The 64-graph random geometric batch in one batched call: every graph's mask and
    order hash to the oracle's digests, with the default work-queue settings and again
    with the autotuned settings and the learned queue order (cost model trained on the
    batch's recorded cycles)."""
    if "rgg64" not in GOLD:
        pytest.skip("no stored oracle result for the batch")
    ref = GOLD["rgg64"]["graphs"]
    print("[full] generating the 64-graph batch", flush=True)
    graphs = synth.batch_config()
    assert [(g.n, g.m) for g in graphs] == [(r["n"], r["m"]) for r in ref]
    print("[full] batch: GPU recovery", flush=True)
    ctx = gss.Context(0)
    try:
        b = gss.Batch(ctx, graphs)
        st, masks, orders, infos = b.recover()
        torch.cuda.synchronize()
        _batch_digests(ref, infos, masks, orders)
        print("[full] batch: autotune, record, train, learned recovery", flush=True)
        lm, lb, ch, ms = b.autotune()
        assert 0 <= lm <= 1024 and 1 <= lb <= 65536 and 0 <= ch <= 64
        ctx.trace_clear()
        b.recover(record=True)
        feat, cyc, size = ctx.trace_read()
        ctx.trace_clear()
        ctx.costmodel_train(feat, cyc, epochs=5, lr=1e-3, seed=0)
        st, masks, orders, infos = b.recover(sched=gss.SCHED_LEARNED)
        torch.cuda.synchronize()
        assert all(i["sched"] == gss.SCHED_LEARNED for i in infos)
        _batch_digests(ref, infos, masks, orders)
        b.free()
    finally:
        ctx.close()


@pytest.mark.timeout(600)
def test_strict_vs_loose_full_size_matches_oracle(gpu_ctx):
    """The strict-vs-loose ablation at full size (the 128^3 grid): strict with c = 8 and
    feGRASS's loose condition with c = 2 and c = 8 (its default BFS step, where a pass
    ends short and further passes run), at alpha = 0.02 and 0.10, against the oracle run
    live (a few seconds each)."""
    import oracle
    from tests.gpu_util import assert_same_recovery, run_gpu
    g = _graph("grid3d_128")
    for alpha in (0.02, 0.1):
        for c, loose in ((8, False), (2, True), (8, True)):
            gpu = run_gpu(gpu_ctx, g, alpha=alpha, beta=c, loose=loose, want_stretch=False)
            orc = oracle.recover(g, alpha=alpha, beta=c, loose=loose)
            assert_same_recovery(gpu, orc)
            print(f"[full] grid3d_128 alpha={alpha} c={c} {'loose' if loose else 'strict'}: "
                  f"{orc.info['passes']} passes", flush=True)
