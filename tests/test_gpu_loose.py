"""GSS_F_LOOSE: feGRASS's loose similarity (Def. "Similar edge (Loose)", eq.
cond-loose-2) with the multi-pass rule of Sec. II-B, on the GPU against the oracle's
loose variant, element by element (mask, order, pass count, status).

The GPU decides a prefix by rounds over tree-ancestor cells; the oracle walks the order
serially with BFS balls on the tree.  Covered: the radius c from 0 to 8, targets that
need many passes (K = m: every off-tree edge, a short result), hub trees where one
recovered edge covers almost everything, the R_T-only key together with the loose
condition, batches (the virtual root above the graphs' trees must not join their balls),
and the 32^3 grid and R-MAT 14 workloads.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_20403_amd import gss, synth
from tests.gpu_util import assert_same_recovery, run_gpu, run_oracle
from tests.test_gpu_batch import small_batch

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
def test_loose_matches_oracle(gpu_ctx, name, make, seed):
    g = make(seed)
    for beta in (0, 1, 2, 5, 8):
        for k in (-1, 7, g.m):
            gpu = run_gpu(gpu_ctx, g, beta=beta, k_override=k, loose=True)
            orc = run_oracle(g, beta=beta, k_override=k, loose=True)
            assert_same_recovery(gpu, orc)


@pytest.mark.parametrize("name,make", SMALL[:2] + SMALL[4:], ids=["rand_max", "rand_tree", "grid"])
def test_loose_with_rt_key_matches_oracle(gpu_ctx, name, make):
    g = make(5)
    for k in (-1, g.m):
        gpu = run_gpu(gpu_ctx, g, beta=2, k_override=k, loose=True, key_rt=True)
        orc = run_oracle(g, beta=2, k_override=k, loose=True, key_rt=True)
        assert_same_recovery(gpu, orc)


@pytest.mark.parametrize("name", ["grid3d_32", "rmat14"])
def test_loose_named_workloads(gpu_ctx, name):
    g = synth.config(name)
    gpu = run_gpu(gpu_ctx, g, loose=True)
    orc = run_oracle(g, loose=True)
    assert_same_recovery(gpu, orc)
    print(f"[loose] {name}: {orc.info['passes']} passes, {gpu['info']['rounds']} rounds in the last prefix",
          flush=True)


@pytest.mark.parametrize("seed", [0, 1])
def test_loose_batch_matches_per_graph_oracle(gpu_ctx, seed):
    graphs = small_batch(seed)
    print(f"[gpu-batch loose] seed {seed}: sizes {[g.n for g in graphs]}", flush=True)
    b = gss.Batch(gpu_ctx, graphs)
    for beta, ks in ((2, None), (3, [g.m for g in graphs])):
        st, masks, orders, infos = b.recover(beta=beta, k_override=ks, loose=True)
        torch.cuda.synchronize()
        for i, (g, mk, od, inf) in enumerate(zip(graphs, masks, orders, infos)):
            ref = oracle.recover(g, beta=beta, k_override=ks[i] if ks else -1, loose=True)
            nrec = ref.info["n_recovered"]
            assert inf["n_recovered"] == nrec and inf["k"] == ref.K
            assert inf["passes"] == ref.info["passes"]
            np.testing.assert_array_equal(mk.cpu().numpy(), ref.mask)
            np.testing.assert_array_equal(od.cpu().numpy()[:nrec], ref.order[:nrec])
    b.free()


def test_batch_rejects_mixed_conditions(gpu_ctx):
    graphs = small_batch(0, count=3)
    b = gss.Batch(gpu_ctx, graphs)
    nb = len(graphs)
    params = b._params([g.alpha for g in graphs], 2, 0, None, False, False, True)
    params[1].flags = 0  # one graph strict, the others loose
    masks = [torch.empty(max(b.m[i], 1), dtype=torch.uint8, device="cuda") for i in range(nb)]
    import ctypes
    mp = (ctypes.c_void_p * nb)(*[m.data_ptr() for m in masks])
    st = gpu_ctx.lib.gss_recover_batch(gpu_ctx.handle, b.handle, ctypes.cast(params, ctypes.c_void_p),
                                       ctypes.cast(mp, ctypes.c_void_p), None, None)
    assert st == -1
    b.free()
