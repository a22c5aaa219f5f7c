"""Helpers shared by the GPU parity tests: run the HIP path and the oracle side by side."""
import numpy as np
import torch

import oracle
from paper_2508_20403_amd import gss


def run_gpu(ctx, g, alpha=None, beta=None, k_override=-1, want_stretch=True, sched=0, mask_tree=False,
            key_rt=False, loose=False):
    alpha = g.alpha if alpha is None else alpha
    beta = g.beta if beta is None else beta
    print(f"[gpu] {g.name} n={g.n} m={g.m} alpha={alpha} beta={beta} k={k_override}"
          f"{' key_rt' if key_rt else ''}{' loose' if loose else ''}", flush=True)
    tree = gss.Tree.from_graph(ctx, g)
    st, mask, order, stretch, info = tree.recover(alpha, beta, k_override, sched=sched,
                                                  want_stretch=want_stretch, mask_tree=mask_tree, stats=True,
                                                  key_rt=key_rt, loose=loose)
    torch.cuda.synchronize()
    out = dict(status=st, mask=mask.cpu().numpy(), order=order.cpu().numpy() if order is not None else None,
               stretch=stretch.cpu().numpy() if stretch is not None else None, info=info)
    tree.free()
    return out


def run_oracle(g, alpha=None, beta=None, k_override=-1, mode=oracle.MODE_INDEXED, full=True, key_rt=False,
               loose=False):
    return oracle.recover(g, alpha=alpha, beta=beta, k_override=k_override, mode=mode, full=full, key_rt=key_rt,
                          loose=loose)


def assert_same_recovery(gpu, orc):
    """Bit-exact comparison of mask, order and (when present) stretch."""
    assert gpu["status"] == orc.status, (gpu["status"], orc.status_name)
    nrec = orc.info["n_recovered"]
    assert gpu["info"]["n_recovered"] == nrec
    assert gpu["info"]["passes"] == orc.info["passes"]
    np.testing.assert_array_equal(gpu["order"][:nrec], orc.order[:nrec])
    np.testing.assert_array_equal(gpu["mask"], orc.mask)
    if gpu["stretch"] is not None:
        a = gpu["stretch"].view(np.uint64)
        b = orc.stretch.view(np.uint64)
        bad = np.flatnonzero(a != b)
        assert bad.size == 0, f"{bad.size} stretches differ, first id {bad[:5]}"
