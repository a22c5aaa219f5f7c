"""ctypes front end of the serial C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "gss_oracle.c")
SRC_TREE = os.path.join(HERE, "gss_oracle_tree.c")
LIB = os.path.join(HERE, "libgss_oracle.so")

MODE_INDEXED, MODE_BRUTE, MODE_SUBTASK = 0, 1, 2
KEY_RT, LOOSE = 1, 2  # variants: sort by R_T instead of the stretch; feGRASS's loose condition
STATUS = {0: "OK", 1: "SHORT", -1: "ERR_ARG", -2: "ERR_NOT_SIMPLE", -3: "ERR_ASYM",
          -4: "ERR_WEIGHT", -5: "ERR_NOT_TREE", -6: "ERR_TREE_EDGE", -7: "ERR_RANGE",
          -9: "ERR_OOM"}
INFO_KEYS = ["m", "n_offtree", "k", "n_recovered", "passes", "n_subtasks", "largest_subtask",
             "ball_verts", "row_entries", "scale"]

_lib = None


def build(verbose=False):
    """Compile the oracle with plain gcc: FP64, no contraction, no fast-math."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-Wall", "-o", LIB + ".tmp", SRC, SRC_TREE, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    global _lib
    _lib = None


def _bind(lib):
    P = ctypes.c_void_p
    lib.orc_recover.restype = ctypes.c_int
    lib.orc_recover.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                                ctypes.c_int64, ctypes.c_int32, ctypes.c_int32] + [P] * 15
    lib.orc_num_edges.restype = ctypes.c_int64
    lib.orc_num_edges.argtypes = [ctypes.c_int32, P]
    if hasattr(lib, "orc_spanning_tree"):
        lib.orc_spanning_tree.restype = ctypes.c_int
        lib.orc_spanning_tree.argtypes = [ctypes.c_int32, P, P, P, ctypes.c_int, P, P, P, P]
    return lib


def build_variant(src_text, out_path):
    """Compiles a (test-only) variant of the oracle source into out_path and loads it."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.run(["gcc", "-O1", "-std=gnu11", "-ffp-contract=off", "-fPIC", "-shared", "-o", out_path,
                    src, "-lm"], check=True)
    return _bind(ctypes.CDLL(out_path))


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(SRC),
                                                                  os.path.getmtime(SRC_TREE)):
            build()
        lib = ctypes.CDLL(LIB)
        _lib = _bind(lib)
    return _lib


class OracleResult:
    """Outputs of one oracle run (host numpy arrays)."""

    def __init__(self, status, **kw):
        self.status = status
        self.status_name = STATUS.get(status, str(status))
        self.__dict__.update(kw)

    @property
    def ok(self):
        return self.status in (0, 1)

    def order_list(self):
        return self.order[: self.info["n_recovered"]]


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def recover(g=None, *, n=None, row_ptr=None, col=None, w=None, parent=None, alpha=None,
            beta=None, k_override=-1, mode=MODE_INDEXED, full=False, lib=None, key_rt=False, loose=False):
    """Run the oracle on a synth.Graph (or raw arrays).  ``full`` also returns per-edge data.
    key_rt: order by R_T instead of the stretch; loose: feGRASS's loose similarity."""
    lib = lib or load()
    if g is not None:
        n = g.n if n is None else n
        row_ptr = g.row_ptr if row_ptr is None else row_ptr
        col = g.col if col is None else col
        w = g.w if w is None else w
        parent = g.parent if parent is None else parent
        alpha = g.alpha if alpha is None else alpha
        beta = g.beta if beta is None else beta
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    if len(row_ptr) != n + 1 or len(parent) != n:
        raise ValueError("array sizes do not match n")
    m = max(0, int(row_ptr[-1]) // 2) if n >= 1 else 0
    K = int(k_override) if k_override >= 0 else int(np.floor(float(alpha) * float(n)))
    mask = np.zeros(m + 1, np.uint8)
    order = np.full(K + 1, -1, np.int32)
    pass_of = np.zeros(m + 1, np.uint8)
    info = np.zeros(16, np.int64)
    times = np.zeros(4, np.float64)
    per_edge = {}
    if full:
        per_edge = dict(stretch=np.zeros(m + 1, np.float64), lca=np.zeros(m + 1, np.int32),
                        bstar=np.zeros(m + 1, np.int32), eu=np.zeros(m + 1, np.int32),
                        ev=np.zeros(m + 1, np.int32), is_tree=np.zeros(m + 1, np.uint8),
                        depth=np.zeros(n, np.int32), Dlo=np.zeros(n, np.uint64),
                        Dhi=np.zeros(n, np.uint64), rank_of=np.zeros(m + 1, np.int32))
    pe = per_edge
    st = lib.orc_recover(int(n), _ptr(row_ptr), _ptr(col), _ptr(w), _ptr(parent), float(alpha),
                         int(beta), int(k_override), int(mode),
                         (KEY_RT if key_rt else 0) | (LOOSE if loose else 0), _ptr(mask), _ptr(order),
                         _ptr(pass_of), _ptr(pe.get("stretch")), _ptr(pe.get("lca")),
                         _ptr(pe.get("bstar")), _ptr(pe.get("eu")), _ptr(pe.get("ev")),
                         _ptr(pe.get("is_tree")), _ptr(pe.get("depth")), _ptr(pe.get("Dlo")),
                         _ptr(pe.get("Dhi")), _ptr(pe.get("rank_of")), _ptr(info), _ptr(times))
    inf = {k: int(info[i]) for i, k in enumerate(INFO_KEYS)}
    out = dict(mask=mask[:m], order=order[:K], pass_of=pass_of[:m], info=inf, times=times.copy(),
               m=m, K=K)
    for k, v in pe.items():
        out[k] = v[:m] if len(v) == m + 1 else v
    return OracleResult(st, **out)


def spanning_tree(g=None, *, n=None, row_ptr=None, col=None, w=None, lib=None, plain=False):
    """feGRASS's spanning tree (gss_oracle_tree.c): returns (parent, root, ordering weight per
    edge id, BFS distance from the root), or raises ValueError for a graph that is not
    connected.  plain: order by w itself (a maximum-weight spanning tree)."""
    lib = lib or load()
    if g is not None:
        n = g.n if n is None else n
        row_ptr = g.row_ptr if row_ptr is None else row_ptr
        col = g.col if col is None else col
        w = g.w if w is None else w
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float64)
    m = int(row_ptr[-1]) // 2
    parent = np.zeros(n, np.int32)
    root = ctypes.c_int32(-1)
    weff = np.zeros(m + 1, np.float64)
    dist = np.zeros(n, np.int32)
    st = lib.orc_spanning_tree(int(n), _ptr(row_ptr), _ptr(col), _ptr(w), 1 if plain else 0, _ptr(parent),
                               ctypes.cast(ctypes.pointer(root), ctypes.c_void_p), _ptr(weff), _ptr(dist))
    if st != 0:
        raise ValueError("spanning tree: bad arguments or a graph that is not connected")
    return parent, int(root.value), weff[:m], dist
