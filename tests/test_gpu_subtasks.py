"""LCA-subtask work queue: the output must not depend on the schedule (queue order,
local/global split, number of workgroups), and the recorder must deliver per-subtask
features and cycles."""
import numpy as np
import pytest

import oracle
from paper_2508_20403_amd import gss, synth
from tests.gpu_util import assert_same_recovery, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

GRAPHS = [
    lambda: synth.config("grid3d_32"),
    lambda: synth.config("rmat14"),
    lambda: synth.random_connected(3000, 9000, seed=5, alpha=0.2, beta=3, tree="random"),
    lambda: synth.grid((40, 50), 1.0, 1.0, seed=0, alpha=0.2, beta=2, name="unitgrid"),
]


@pytest.mark.parametrize("make", GRAPHS, ids=["grid32", "rmat14", "rand3000", "unitgrid"])
def test_output_independent_of_schedule(gpu_ctx, make):
    g = make()
    orc = run_oracle(g)
    try:
        for local_max, blocks in ((1024, 2048), (0, 2048), (1, 2048), (64, 3), (300, 1), (1024, 7)):
            gpu_ctx.set_tuning(local_max, blocks)
            gpu = run_gpu(gpu_ctx, g)
            assert_same_recovery(gpu, orc)
        gpu_ctx.set_tuning(64, 2048)
        # the short sorts: radix sort, and sample sort with buckets sorted in global memory
        for radix, cap in ((True, 0), (False, 16), (False, 2)):
            gpu_ctx.set_sort(radix, cap)
            gpu = run_gpu(gpu_ctx, g)
            assert_same_recovery(gpu, orc)
    finally:
        gpu_ctx.set_tuning(64, 2048)
        gpu_ctx.set_sort(False, 0)


def test_trace_records_features_and_cycles(gpu_ctx):
    g = synth.config("grid3d_32")
    gpu_ctx.trace_clear()
    tree = gss.Tree.from_graph(gpu_ctx, g)
    st, mask, order, _, info = tree.recover(g.alpha, g.beta, record=True)
    tree.free()
    feat, cyc, size = gpu_ctx.trace_read()
    assert len(cyc) > 0 and np.all(cyc > 0)
    assert np.all(np.isfinite(feat))
    assert np.all(size >= 1) and np.all(size <= 1024)
    # feature 0 is log2(1 + size)
    np.testing.assert_allclose(feat[:, 0], np.log2(1.0 + size), rtol=1e-6)
    gpu_ctx.trace_clear()
    assert len(gpu_ctx.trace_read()[1]) == 0


def _features_from_oracle(orc, g, P, lca_vertex):
    """The twelve cost-model features of the subtask {prefix edges with LCA l}, from the
    oracle's per-edge LCA, beta*, depths and criticality ranks and the tree degrees of
    the parent array, in float64 (definitions: include/gss.h, cost-model block)."""
    off = np.flatnonzero(orc.is_tree == 0)
    pi = off[np.argsort(orc.rank_of[off], kind="stable")]
    pre = pi[:P]
    E = pre[orc.lca[pre] == lca_vertex]
    par = g.parent
    deg = np.bincount(par[par >= 0], minlength=g.n) + (par >= 0)
    d = orc.depth
    dl = int(d[lca_vertex])
    u, v = orc.eu[E], orc.ev[E]
    path = (d[u] - dl) + (d[v] - dl)
    b = orc.bstar[E]
    dsum = deg[u] + deg[v]
    S = float(len(E))
    f = np.array([np.log2(1 + S), path.sum() / S, path.max(), b.sum() / S, (b == 0).sum() / S,
                  dsum.sum() / S, dsum.max(), np.log2(1 + deg[lca_vertex]), np.log2(1 + dl), S / max(P, 1),
                  np.log2(1 + path.sum()), np.log2(1 + S * S)])
    return len(E), f


@pytest.mark.parametrize("make", [lambda: synth.config("grid3d_32"),
                                  lambda: synth.random_connected(4000, 12000, seed=8, alpha=0.1, beta=3,
                                                                 tree="random")],
                         ids=["grid32", "rand4000"])
def test_trace_features_match_oracle_quantities(gpu_ctx, make):
    """Every recorded feature row is recomputed from the oracle's per-edge outputs (LCA,
    beta*, depth, criticality rank) and the tree degrees: a wrong feature would otherwise
    only degrade the schedule silently.  Tolerance: float32 rounding of the kernel's
    exact integer sums (relative 2e-6)."""
    g = make()
    orc = oracle.recover(g, full=True)
    assert orc.info["passes"] == 1
    gpu_ctx.trace_clear()
    tree = gss.Tree.from_graph(gpu_ctx, g)
    _, _, _, _, info = tree.recover(g.alpha, g.beta, record=True)
    tree.free()
    feat, cyc, size, lca, plen = gpu_ctx.trace_read(extended=True)
    gpu_ctx.trace_clear()
    assert len(cyc) > 0
    for i in range(len(cyc)):
        S, f = _features_from_oracle(orc, g, int(plen[i]), int(lca[i]))
        assert S == size[i], (i, S, size[i])
        np.testing.assert_allclose(feat[i].astype(np.float64), f, rtol=2e-6, atol=1e-6, err_msg=f"row {i}")


def test_learned_schedule_without_model_falls_back(gpu_ctx):
    """GSS_SCHED_LEARNED on a context with no cost model runs the edge-count order: the
    call succeeds, reports the fallback, and the output is the oracle's bit for bit."""
    ctx = gss.Context(0)
    try:
        for g in (synth.config("grid3d_32"), synth.config("rmat14")):
            orc = run_oracle(g)
            gpu = run_gpu(ctx, g, sched=gss.SCHED_LEARNED)
            assert gpu["info"]["sched"] == gss.SCHED_EDGECOUNT
            assert_same_recovery(gpu, orc)
    finally:
        ctx.close()
