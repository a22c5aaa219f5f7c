"""Benchmark: one step = gss_tree_prep + gss_recover for one sparsifier on one GPU.

Prints ONE JSON line (see the repository's benchmark contract).  The workload is the
3D 7-point grid 128^3 (2,097,152 vertices, 6,242,304 edges), weights log-uniform in
[1, 1e4], maximum-weight spanning tree, alpha = 0.05, beta = 2, seed 0.  Inputs are
resident in HBM before the timed region.  `value` is off-tree edges processed per
second (M / step time).

The roofline entry is for the dominant kernel: its launches are bracketed live by HIP
events on the library's stream during the timed steps; `achieved` is that kernel's
algorithmic bytes per launch divided by its mean launch time.  The CPU baseline is the
serial oracle (test infrastructure, never tuned) on the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s

WORKLOADS = {
    "grid3d_128": "3D 7-point grid 128^3 (2,097,152 vertices, 6,242,304 edges), w log-uniform [1,1e4] "
                  "fp64, max-weight spanning tree, alpha=0.05, beta=2, seed 0",
    "grid2d_64": "2D 4-connected grid 64x64 (4096 vertices, 8064 edges), w log-uniform [1,100] fp64, "
                 "max-weight spanning tree, alpha=0.02, beta=2, seed 0",
    "rmat22": "R-MAT scale 22 (a=.57,b=c=.19,d=.05, avg degree 16) symmetrised, deduplicated, largest CC, "
              "w uniform (0,1] fp64, max-weight spanning tree, alpha=0.10, beta=2, seed 0",
    "grid3d_160": "3D 7-point grid 160^3, w log-uniform [1,1e4], alpha=0.10, beta=2, seed 0",
    "rmat24": "R-MAT scale 24 LCC, w uniform (0,1], alpha=0.10, beta=2, seed 0",
}


def kernel_bytes(name, g, info, tree_M):
    """Algorithmic bytes one launch of `name` must move (per-unit figure x units)."""
    n, m, nnz, M = g.n, g.m, g.nnz, tree_M
    if name == "k_edge_stretch":
        # per off-tree edge: read u,v (8) and w (8); gather first[u],first[v] (8),
        # depth[u],depth[v] (8), D[u],D[v],D[lca] (48), two Euler entries for the
        # RMQ answer (16); write key (8), lca (4), beta* (1)  -> 109 B
        return 109 * M
    if name == "k_walk2_euler":
        # per arc (2(n-1)): succ (4) + term (16) read, and per vertex first/depth (8),
        # D (16) and two Euler entries (16) written -> 20*2 + 40 per vertex
        return 40 * (n - 1) + 40 * (n - 1)
    if name == "k_walk1":
        return 20 * 2 * (n - 1)
    return None


def src_digest(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="grid3d_128", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--kernel", default=None, help="kernel for the roofline entry (default: dominant)")
    ap.add_argument("--breakdown", action="store_true", help="print a per-kernel time table to stderr")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (this build has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2508_20403_amd import gss, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    g = synth.config(args.workload)
    print(f"[bench] workload {args.workload}: n={g.n} m={g.m} ({time.time() - t0:.1f}s to build)",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    row_ptr = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    parent = torch.from_numpy(g.parent).to(dev)
    K = synth.k_of(g.alpha, g.n)
    mask = torch.empty(g.m, dtype=torch.uint8, device=dev)
    order = torch.empty(max(K, 1), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    ctx = gss.Context(0, torch.cuda.current_stream())

    def step():
        tree = gss.Tree(ctx, row_ptr, col, w, parent)
        r = tree.recover(g.alpha, g.beta, out=(mask, order, None))
        tree.free()
        return r

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-kernel breakdown (an untimed pass) to find the dominant kernel
    ctx.profile(True, None)
    st, _, _, _, info = step()
    torch.cuda.synchronize()
    table = ctx.profile_read()
    ctx.profile(False)
    dominant = args.kernel or max(table, key=lambda k: table[k][0])
    if args.breakdown:
        tot = sum(v[0] for v in table.values())
        for k, (ms, nl) in sorted(table.items(), key=lambda kv: -kv[1][0]):
            print(f"  {k:24s} {ms:9.3f} ms  {nl:5d} launches  {100 * ms / tot:5.1f}%", file=sys.stderr)
    print(f"[bench] dominant kernel {dominant}; info {info}", file=sys.stderr, flush=True)

    ctx.profile(True, dominant)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    prof = ctx.profile_read()
    ctx.profile(False)
    ms_step = 1e3 * (t_end - t_start) / args.steps
    M = info["n_offtree"]
    value = M / (ms_step * 1e-3)

    dom_ms, dom_n = prof.get(dominant, (float("nan"), 0))
    dom_avg_ms = dom_ms / max(dom_n, 1)
    nbytes = kernel_bytes(dominant, g, info, M)
    roofline = None
    if nbytes is not None and dom_n > 0:
        ach = nbytes / (dom_avg_ms * 1e-3) / 1e9
        roofline = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dominant,
                    "kernel_ms": round(dom_avg_ms, 4), "alg_bytes": int(nbytes)}
        tfile = os.path.join(ROOT, "profiles", f"traffic_{dominant}_{args.workload}.json")
        if os.path.exists(tfile):
            tr = json.load(open(tfile))
            csrc = os.path.join(ROOT, "paper_2508_20403_amd", "csrc")
            digest = src_digest([os.path.join(csrc, f) for f in sorted(os.listdir(csrc))])
            if tr.get("source_digest") == digest:
                roofline["traffic"] = tr.get("traffic_bytes")

    # parity of the benchmarked output and the CPU baseline: the serial oracle
    cpu = None
    bit_exact = None
    if not args.no_cpu:
        import oracle
        os.environ.setdefault("OMP_NUM_THREADS", "1")
        t = time.perf_counter()
        ref = oracle.recover(g)
        cpu_s = time.perf_counter() - t
        cpu = {"value": round(M / cpu_s, 1), "unit": "off-tree edges/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole {args.workload} workload once (tree preparation + recovery of one "
                         f"sparsifier), {cpu_s:.2f} s on one host core",
               "ms_per_sparsifier": round(cpu_s * 1e3, 1)}
        bit_exact = bool(np.array_equal(mask.cpu().numpy(), ref.mask) and
                         np.array_equal(order[:K].cpu().numpy(), ref.order))

    out = {
        "metric": "off-tree edges recovered/s + ms per sparsifier, learned-sched vs plain, bit-exact",
        "value": round(value, 1),
        "unit": "off-tree edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload], "n": g.n, "m": g.m, "offtree_edges": M, "k": K,
                   "alpha": g.alpha, "beta": g.beta, "ms_per_sparsifier": round(ms_step, 4),
                   "recovered_per_s": round(K / (ms_step * 1e-3), 1), "bit_exact_vs_oracle": bit_exact,
                   "prefix_len": info["prefix_len"], "passes": info["passes"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
