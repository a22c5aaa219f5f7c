"""The allocation-free entry point (gss_recover_noalloc) against gss_recover.

Both are called through the C ABI on the same prepared trees; the outputs must agree
bit for bit (mask, order, stretch) together with the counters, on two calls in a row
where the second input is smaller than the first (the shared scratch keeps the first
call's contents).  An input whose scratch would exceed the static array is rejected with
GSS_ERR_OOM before anything runs, and the context stays usable."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2508_20403_amd import gss, synth

pytestmark = pytest.mark.gpu


def _call(ctx, tree, g, entry, k_override=-1):
    k = tree.target_count(g.alpha, k_override)
    dev = torch.device("cuda")
    mask = torch.full((max(tree.m, 1),), 7, dtype=torch.uint8, device=dev)
    order = torch.full((max(k, 1),), -5, dtype=torch.int32, device=dev)
    stretch = torch.full((max(tree.m, 1),), -1.0, dtype=torch.float64, device=dev)
    p = gss.Params(float(g.alpha), int(g.beta), gss.SCHED_EDGECOUNT, int(k_override), gss.GSS_F_STATS, 0)
    info = gss.Info()
    fn = getattr(ctx.lib, entry)
    st = fn(ctx.handle, tree.handle, ctypes.byref(p), ctypes.c_void_p(mask.data_ptr()),
            ctypes.c_void_p(order.data_ptr()), ctypes.c_void_p(stretch.data_ptr()), ctypes.byref(info))
    torch.cuda.synchronize()
    return st, mask[:tree.m].cpu().numpy(), order[:k].cpu().numpy(), stretch[:tree.m].cpu().numpy(), info.as_dict()


def _same(a, b):
    assert a[0] == b[0] and a[0] in (gss.GSS_OK, gss.GSS_SHORT), (a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[3].view(np.uint64), b[3].view(np.uint64))
    assert a[4] == b[4]


def test_noalloc_matches_recover_twice():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = gss.Context(0)
    try:
        graphs = [synth.grid((40, 40, 40), 1.0, 1e4, seed=5, alpha=0.05, beta=2, name="grid40"),
                  synth.random_connected(3000, 9000, seed=7, alpha=0.1, beta=3, tree="random")]
        for g in graphs:  # the second input is smaller than the first
            print(f"[noalloc] {g.name} n={g.n} m={g.m}", flush=True)
            tree = gss.Tree.from_graph(ctx, g)
            ref = _call(ctx, tree, g, "gss_recover")
            got = _call(ctx, tree, g, "gss_recover_noalloc")
            _same(got, ref)
            tree.free()
        # too large for the static scratch: rejected up front, the context still works
        g = synth.grid((80, 80, 80), 1.0, 1e4, seed=1, alpha=0.05, beta=2, name="grid80")
        print(f"[noalloc] oversized {g.name} n={g.n} m={g.m}", flush=True)
        tree = gss.Tree.from_graph(ctx, g)
        big_k = g.m - g.n + 1
        st = _call(ctx, tree, g, "gss_recover_noalloc", k_override=big_k)[0]
        assert st == -9, st
        assert b"allocation-free" in ctx.lib.gss_last_error(ctx.handle)
        tree.free()
        g = graphs[1]
        tree = gss.Tree.from_graph(ctx, g)
        _same(_call(ctx, tree, g, "gss_recover_noalloc"), _call(ctx, tree, g, "gss_recover"))
        tree.free()
    finally:
        ctx.close()
