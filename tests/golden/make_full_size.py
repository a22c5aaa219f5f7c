"""Writes tests/golden/full_size.json: the oracle's results on the full-size workloads.

The full-size workloads (R-MAT scale 22 and 24, the 160^3 grid, the 64-graph random
geometric batch) take the serial oracle minutes, too long to run inside a GPU test.  This script runs the oracle once per
workload and stores digests of its outputs (SHA-256 of the recovered-edge mask bytes,
of the recovery order as little-endian int32 and of the stretch array as little-endian
float64 bits) plus its counters, so that the GPU tests can compare their outputs with
the oracle's bit for bit.  Only the seeded input generators and the oracle are used.

    python tests/golden/make_full_size.py [name ...]
"""
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2508_20403_amd import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size.json")


def digest(a, dtype):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()


def batch_entry():
    """The 64-graph random geometric batch: per-graph digests of the oracle's outputs."""
    t0 = time.time()
    graphs = synth.batch_config()
    t1 = time.time()
    per = []
    for g in graphs:
        ref = oracle.recover(g, full=False)
        nrec = ref.info["n_recovered"]
        per.append({"n": int(g.n), "m": int(g.m), "k": int(ref.info["k"]), "n_recovered": int(nrec),
                    "passes": int(ref.info["passes"]), "status": int(ref.status),
                    "mask_sha256": digest(ref.mask, np.uint8), "order_sha256": digest(ref.order[:nrec], "<i4")})
    t2 = time.time()
    return {"graphs": per, "oracle_seconds": round(t2 - t1, 1), "generate_seconds": round(t1 - t0, 1)}


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        if name == "rgg64":
            data[name] = batch_entry()
            print(name, data[name]["oracle_seconds"], flush=True)
            with open(OUT + ".tmp", "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(OUT + ".tmp", OUT)
            continue
        t0 = time.time()
        g = synth.config(name)
        t1 = time.time()
        ref = oracle.recover(g, full=True)
        t2 = time.time()
        nrec = ref.info["n_recovered"]
        data[name] = {
            "n": int(g.n), "m": int(g.m), "n_offtree": int(ref.info["n_offtree"]), "k": int(ref.info["k"]),
            "n_recovered": int(nrec), "passes": int(ref.info["passes"]), "status": int(ref.status),
            "n_subtasks": int(ref.info["n_subtasks"]), "largest_subtask": int(ref.info["largest_subtask"]),
            "mask_sha256": digest(ref.mask, np.uint8),
            "order_sha256": digest(ref.order[:nrec], "<i4"),
            "stretch_sha256": digest(ref.stretch.view(np.uint64), "<u8"),
            "order_head": [int(x) for x in ref.order[:16]],
            "oracle_seconds": round(t2 - t1, 1), "generate_seconds": round(t1 - t0, 1),
        }
        print(name, data[name], flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main(sys.argv[1:] or ["grid3d_160", "rmat22", "rmat24", "rgg64"])
