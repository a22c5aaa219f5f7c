"""What the trained cost model gains over the edge-count queue: the makespan of the
persistent work-queue kernel on a workload whose tail is on the critical path.

synth.skewed_cost builds LCA subtasks that all hold 256 off-tree edges but cost very
differently in the greedy: in a light one the first recovered edge marks the other 255
(beta* = 2), in a heavy one nothing is marked (beta* = 0) and every edge is compared with
every earlier candidate.  Ordered by edge count the subtasks tie, so the queue keeps
them in LCA order and the few heavy ones (highest vertex ids) start last: the wavefronts
that pull them finish long after the rest.  The cost model, trained on the cycles the
plain kernel recorded on this workload, ranks the heavy subtasks first, so they start
at once and the light ones fill in around them.  The kernel's time is measured with
HIP events around its last launch: the resolved prefix grows over a few rounds, and only
the last one holds every subtask whole (earlier ones see a few edges of each, where the
two orders cost the same).  Outputs are identical under both orders.
"""
import numpy as np
import pytest
import torch

from paper_2508_20403_amd import gss, synth

pytestmark = pytest.mark.gpu

BLOCKS = 64             # workgroups of the persistent kernel: 256 wavefronts
WAVES = 4 * BLOCKS


def _queue_ms(ctx, tree, K, sched, reps=3):
    best, out = None, None
    for _ in range(reps):
        torch.cuda.synchronize()
        ctx.profile(True, None)
        st, mask, order, _, info = tree.recover(1.0, 2, k_override=K, sched=sched)
        torch.cuda.synchronize()
        table = ctx.profile_read(last=True)
        ctx.profile(False)
        ms = sum(v[3] for k, v in table.items() if k.startswith("k_local_recover"))
        best = ms if best is None else min(best, ms)
        out = (st, mask.cpu().numpy(), order.cpu().numpy(), info)
    return best, out


def test_learned_queue_cuts_the_makespan():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nheavy, nlight = WAVES // 4, 16 * WAVES
    g = synth.skewed_cost(nheavy, nlight, side=16)
    K = nlight + 256 * nheavy  # one candidate per light subtask, 256 per heavy one
    print(f"[gain] {g.name} n={g.n} m={g.m} K={K}", flush=True)
    ctx = gss.Context(0)
    try:
        ctx.set_tuning(256, BLOCKS, 1)
        tree = gss.Tree.from_graph(ctx, g)
        ctx.trace_clear()
        st, _, _, _, info = tree.recover(1.0, 2, k_override=K, record=True)
        assert info["passes"] == 1 and info["n_recovered"] == K
        # the prefix grows over a few rounds before it holds all K candidates; every round
        # records its queued subtasks (the last one all of them, at 256 edges each)
        feat, cyc, size = ctx.trace_read()
        ctx.trace_clear()
        assert np.sum(size == 256) >= nheavy + nlight
        ctx.costmodel_train(feat, cyc, epochs=40, lr=3e-3, seed=0)
        t_edge, out_e = _queue_ms(ctx, tree, K, gss.SCHED_EDGECOUNT)
        t_learn, out_l = _queue_ms(ctx, tree, K, gss.SCHED_LEARNED)
        assert out_l[3]["sched"] == gss.SCHED_LEARNED
        assert out_e[0] == out_l[0]
        np.testing.assert_array_equal(out_e[1], out_l[1])
        np.testing.assert_array_equal(out_e[2], out_l[2])
        whole = size == 256  # subtasks of the rounds that held them whole
        heavy = whole & (feat[:, 4] > 0.5)  # share of beta* = 0
        light = whole & (feat[:, 4] <= 0.5)
        print(f"[gain] cycles heavy {np.median(cyc[heavy]):.0f} light {np.median(cyc[light]):.0f}; "
              f"queue kernel: edge-count {t_edge:.3f} ms, learned {t_learn:.3f} ms ({t_edge / t_learn:.2f}x)",
              flush=True)
        assert t_learn < t_edge / 1.15, (t_edge, t_learn)
        tree.free()
    finally:
        ctx.close()
