"""Thin ctypes binding of libgss.so (include/gss.h).

Argument marshalling only: every step of the recovery runs in the library's HIP
kernels.  PyTorch supplies device memory and the stream.  There is no fallback: if the
library is missing this module raises on load.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgss.so")

GSS_OK, GSS_SHORT = 0, 1
STATUS_NAMES = {0: "GSS_OK", 1: "GSS_SHORT", -1: "GSS_ERR_ARG", -2: "GSS_ERR_NOT_SIMPLE",
                -3: "GSS_ERR_ASYM", -4: "GSS_ERR_WEIGHT", -5: "GSS_ERR_NOT_TREE",
                -6: "GSS_ERR_TREE_EDGE", -7: "GSS_ERR_RANGE", -8: "GSS_ERR_HIP", -9: "GSS_ERR_OOM"}
GSS_F_MASK_TREE = 1
GSS_PREP_TRUSTED = 1
SCHED_EDGECOUNT, SCHED_LEARNED = 0, 1

# the symbols include/gss.h declares
EXPORTS = ["gss_ctx_create", "gss_ctx_set_stream", "gss_ctx_destroy", "gss_tree_prep",
           "gss_tree_free", "gss_recover", "gss_tree_export", "gss_edge_lca",
           "gss_tree_num_edges", "gss_status_str", "gss_last_error", "gss_ctx_profile",
           "gss_ctx_profile_read", "gss_ctx_set_tuning", "gss_trace_read", "gss_trace_clear",
           "gss_costmodel_train", "gss_costmodel_load", "gss_costmodel_save", "gss_costmodel_predict",
           "gss_costmodel_grad", "gss_batch_prep", "gss_recover_batch", "gss_tree_num_graphs",
           "gss_tree_graph_edges", "gss_autotune", "gss_ctx_set_batch_split", "gss_target_count",
           "gss_ctx_set_rank_capacity", "gss_tree_rank_attempts", "gss_ctx_set_sort", "gss_ctx_set_capture",
           "gss_ctx_capture_stats", "gss_spanning_tree",
           "gss_recover_noalloc"]
GSS_F_RECORD = 2
GSS_F_STATS = 4
GSS_F_KEY_RT = 8
GSS_F_LOOSE = 16
GSS_TREE_WEIGHT = 1
NFEAT = 12
COSTMODEL_FLOATS = 5081
COSTMODEL_PARAMS = 5057


class GSSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_int32), ("sched", ctypes.c_int32),
                ("k_override", ctypes.c_int64), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n_offtree", ctypes.c_int64), ("k", ctypes.c_int64),
                ("n_recovered", ctypes.c_int64), ("n_subtasks", ctypes.c_int64),
                ("largest_subtask", ctypes.c_int64), ("prefix_len", ctypes.c_int64),
                ("n_arcs", ctypes.c_int64), ("n_join", ctypes.c_int64), ("passes", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("sched", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def load_library(path=LIB_PATH):
    """Loads libgss.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2508_20403_amd.build.build()")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.gss_ctx_create.argtypes = [ctypes.c_int, P, ctypes.POINTER(P)]
    lib.gss_ctx_set_stream.argtypes = [P, P]
    lib.gss_ctx_destroy.argtypes = [P]
    lib.gss_tree_prep.argtypes = [P, ctypes.POINTER(Csr), P, ctypes.c_uint32, ctypes.POINTER(P)]
    lib.gss_tree_free.argtypes = [P]
    lib.gss_recover.argtypes = [P, P, ctypes.POINTER(Params), P, P, P, ctypes.POINTER(Info)]
    lib.gss_recover_noalloc.argtypes = [P, P, ctypes.POINTER(Params), P, P, P, ctypes.POINTER(Info)]
    lib.gss_recover_noalloc.restype = ctypes.c_int32
    lib.gss_tree_export.argtypes = [P, P, P, P, ctypes.POINTER(ctypes.c_int32)]
    lib.gss_edge_lca.argtypes = [P, P, ctypes.c_int32, P, P]
    lib.gss_tree_num_edges.argtypes = [P]
    lib.gss_tree_num_edges.restype = ctypes.c_int64
    lib.gss_status_str.argtypes = [ctypes.c_int32]
    lib.gss_status_str.restype = ctypes.c_char_p
    lib.gss_last_error.argtypes = [P]
    lib.gss_last_error.restype = ctypes.c_char_p
    lib.gss_ctx_profile.argtypes = [P, ctypes.c_int32, ctypes.c_char_p]
    lib.gss_ctx_profile.restype = ctypes.c_int32
    lib.gss_ctx_profile_read.argtypes = [P, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
    lib.gss_ctx_profile_read.restype = ctypes.c_int32
    lib.gss_ctx_set_tuning.argtypes = [P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    lib.gss_target_count.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Params)]
    lib.gss_target_count.restype = ctypes.c_int64
    lib.gss_trace_read.argtypes = [P, P, P, P, P, P, ctypes.c_int64]
    lib.gss_trace_read.restype = ctypes.c_int64
    lib.gss_trace_clear.argtypes = [P]
    lib.gss_costmodel_train.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_uint64,
                                        ctypes.c_uint32, P]
    lib.gss_costmodel_load.argtypes = [P, P]
    lib.gss_costmodel_save.argtypes = [P, P]
    lib.gss_costmodel_predict.argtypes = [P, P, ctypes.c_int64, P]
    lib.gss_costmodel_grad.argtypes = [P, P, P, ctypes.c_int32, P, P]
    lib.gss_batch_prep.argtypes = [P, ctypes.c_int32, P, P, ctypes.c_uint32, ctypes.POINTER(P)]
    lib.gss_recover_batch.argtypes = [P, P, P, P, P, P]
    lib.gss_ctx_set_sort.argtypes = [P, ctypes.c_int32, ctypes.c_int32]
    lib.gss_ctx_set_sort.restype = ctypes.c_int32
    lib.gss_spanning_tree.argtypes = [P, P, ctypes.c_uint32, P, ctypes.POINTER(ctypes.c_int32), P]
    lib.gss_spanning_tree.restype = ctypes.c_int32
    lib.gss_ctx_set_capture.argtypes = [P, ctypes.c_int32]
    lib.gss_ctx_set_capture.restype = ctypes.c_int32
    lib.gss_ctx_capture_stats.argtypes = [P] + [ctypes.POINTER(ctypes.c_int64)] * 4
    lib.gss_ctx_capture_stats.restype = ctypes.c_int32
    lib.gss_ctx_set_rank_capacity.argtypes = [P, ctypes.c_int32]
    lib.gss_ctx_set_rank_capacity.restype = ctypes.c_int32
    lib.gss_tree_rank_attempts.argtypes = [P]
    lib.gss_tree_rank_attempts.restype = ctypes.c_int32
    lib.gss_ctx_set_batch_split.argtypes = [P, ctypes.c_int64]
    lib.gss_ctx_set_batch_split.restype = ctypes.c_int32
    lib.gss_tree_num_graphs.argtypes = [P]
    lib.gss_tree_num_graphs.restype = ctypes.c_int32
    lib.gss_tree_graph_edges.argtypes = [P, ctypes.c_int32]
    lib.gss_tree_graph_edges.restype = ctypes.c_int64
    lib.gss_autotune.argtypes = [P, P, P, P, P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_double)]
    for name in ("gss_autotune", "gss_batch_prep", "gss_recover_batch", "gss_ctx_create", "gss_ctx_set_stream", "gss_ctx_destroy", "gss_tree_prep",
                 "gss_tree_free", "gss_recover", "gss_tree_export", "gss_edge_lca", "gss_ctx_set_tuning",
                 "gss_trace_clear", "gss_costmodel_train", "gss_costmodel_load", "gss_costmodel_save",
                 "gss_costmodel_predict", "gss_costmodel_grad"):
        getattr(lib, name).restype = ctypes.c_int32
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_handle(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Context:
    """A gss_ctx bound to a torch stream on one device."""

    def __init__(self, device=0, stream=None):
        self.lib = load_library()
        self.device = device
        self.handle = ctypes.c_void_p()
        with torch.cuda.device(device):
            st = self.lib.gss_ctx_create(device, _stream_handle(stream), ctypes.byref(self.handle))
        if st != GSS_OK:
            raise GSSError(st, self.lib.gss_last_error(None).decode())

    def check(self, st):
        if st not in (GSS_OK, GSS_SHORT):
            raise GSSError(st, self.lib.gss_last_error(self.handle).decode())
        return st

    def set_stream(self, stream):
        self.check(self.lib.gss_ctx_set_stream(self.handle, _stream_handle(stream)))

    def profile(self, enable=True, kernel=None):
        """Starts (or stops) live HIP-event timing of one kernel (None: all kernels)."""
        self.check(self.lib.gss_ctx_profile(self.handle, 1 if enable else 0,
                                            kernel.encode() if kernel else None))

    def profile_read(self, last=False):
        """{kernel name: (total ms, launches, algorithmic bytes)} accumulated since profile();
        with last=True each tuple also carries the milliseconds of the latest launch."""
        out = {}
        count = self.lib.gss_ctx_profile_read(self.handle, 0, None, 0, None, None, None, None)
        buf = ctypes.create_string_buffer(128)
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        nb = ctypes.c_int64()
        lm = ctypes.c_double()
        for i in range(max(count, 0)):
            self.lib.gss_ctx_profile_read(self.handle, i, buf, 128, ctypes.byref(ms), ctypes.byref(n),
                                          ctypes.byref(nb), ctypes.byref(lm))
            out[buf.value.decode()] = (ms.value, n.value, nb.value) + ((lm.value,) if last else ())
        return out

    # ---- subtask scheduling and the learned cost model --------------------------------
    def set_batch_split(self, own_nnz):
        """Batch graphs with at least own_nnz CSR entries are prepared on their own."""
        self.check(self.lib.gss_ctx_set_batch_split(self.handle, int(own_nnz)))

    def spanning_tree(self, row_ptr, col, w, weight=False, want_weff=False):
        """feGRASS's spanning tree on the GPU (gss_spanning_tree) of a device CSR: returns
        (parent tensor, root, per-edge ordering weight tensor or None).  weight=True orders
        the edges by w itself (a maximum-weight spanning tree)."""
        n = row_ptr.numel() - 1
        csr = Csr(n, col.numel(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                  w.data_ptr() if w.numel() else None)
        parent = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
        weff = torch.empty(max(col.numel() // 2, 1), dtype=torch.float64, device=row_ptr.device) if want_weff \
            else None
        root = ctypes.c_int32(-1)
        self.check(self.lib.gss_spanning_tree(self.handle, ctypes.byref(csr), GSS_TREE_WEIGHT if weight else 0,
                                              parent.data_ptr(), ctypes.byref(root), _ptr(weff)))
        return parent, int(root.value), (weff[: col.numel() // 2] if weff is not None else None)

    def set_capture(self, enable=True):
        """Memoized graph capture of recoveries (gss_ctx_set_capture): a repeated call with the
        same tree, parameters and output buffers replays a HIP graph."""
        self.check(self.lib.gss_ctx_set_capture(self.handle, 1 if enable else 0))

    def capture_stats(self):
        """{records, captures, replays, syncs} counted since the context was created."""
        v = [ctypes.c_int64() for _ in range(4)]
        self.check(self.lib.gss_ctx_capture_stats(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(("records", "captures", "replays", "syncs"), (x.value for x in v)))

    def set_sort(self, radix=False, bucket_cap=0):
        """Short sorts by the radix sort (radix=True) or the sample sort with at most
        bucket_cap pairs per LDS bucket (0: the kernel's limit); diagnostic."""
        self.check(self.lib.gss_ctx_set_sort(self.handle, 1 if radix else 0, int(bucket_cap)))

    def set_rank_capacity(self, divisor):
        """Divides the list ranking's first-attempt capacities (diagnostic; 1 = default)."""
        self.check(self.lib.gss_ctx_set_rank_capacity(self.handle, int(divisor)))

    def set_tuning(self, local_max, local_blocks, chunk=0):
        """Work-queue settings; chunk 0 derives the queue entries per pop from the queue length."""
        self.check(self.lib.gss_ctx_set_tuning(self.handle, int(local_max), int(local_blocks), int(chunk)))

    def trace_read(self, extended=False):
        """(features [rows,12] float32, cycles [rows] float64, sizes [rows] int32) recorded so
        far; with extended=True also (LCA vertex [rows] int32, prefix length [rows] int64)."""
        import numpy as np
        rows = self.lib.gss_trace_read(self.handle, None, None, None, None, None, 0)
        feat = np.zeros((rows, NFEAT), np.float32)
        cyc = np.zeros(rows, np.float64)
        size = np.zeros(rows, np.int32)
        lca = np.zeros(rows, np.int32)
        plen = np.zeros(rows, np.int64)
        if rows:
            vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
            self.lib.gss_trace_read(self.handle, vp(feat), vp(cyc), vp(size), vp(lca), vp(plen), rows)
        return (feat, cyc, size, lca, plen) if extended else (feat, cyc, size)

    def trace_clear(self):
        self.check(self.lib.gss_trace_clear(self.handle))

    def costmodel_train(self, feat, cycles, epochs=10, lr=1e-3, seed=0, warm=False):
        import numpy as np
        feat = np.ascontiguousarray(feat, np.float32)
        cycles = np.ascontiguousarray(cycles, np.float64)
        loss = np.zeros(epochs, np.float32)
        self.check(self.lib.gss_costmodel_train(self.handle, feat.ctypes.data_as(ctypes.c_void_p),
                                                cycles.ctypes.data_as(ctypes.c_void_p), len(cycles),
                                                int(epochs), float(lr), int(seed), 1 if warm else 0,
                                                loss.ctypes.data_as(ctypes.c_void_p)))
        return loss

    def costmodel_load(self, weights):
        import numpy as np
        w = np.ascontiguousarray(weights, np.float32)
        assert w.size == COSTMODEL_FLOATS
        self.check(self.lib.gss_costmodel_load(self.handle, w.ctypes.data_as(ctypes.c_void_p)))

    def costmodel_save(self):
        import numpy as np
        w = np.zeros(COSTMODEL_FLOATS, np.float32)
        self.check(self.lib.gss_costmodel_save(self.handle, w.ctypes.data_as(ctypes.c_void_p)))
        return w

    def costmodel_predict(self, feat):
        """feat: device float32 tensor [n,12]; returns device float32 [n] of log2(cycles)."""
        n = feat.shape[0]
        out = torch.empty(max(n, 1), dtype=torch.float32, device=feat.device)
        self.check(self.lib.gss_costmodel_predict(self.handle, _ptr(feat.contiguous()), n, _ptr(out)))
        return out[:n]

    def costmodel_grad(self, x, y):
        import numpy as np
        x = np.ascontiguousarray(x, np.float32)
        y = np.ascontiguousarray(y, np.float32)
        g = np.zeros(COSTMODEL_PARAMS, np.float32)
        loss = np.zeros(1, np.float32)
        self.check(self.lib.gss_costmodel_grad(self.handle, x.ctypes.data_as(ctypes.c_void_p),
                                               y.ctypes.data_as(ctypes.c_void_p), len(y),
                                               g.ctypes.data_as(ctypes.c_void_p),
                                               loss.ctypes.data_as(ctypes.c_void_p)))
        return g, float(loss[0])

    def close(self):
        if self.handle:
            self.lib.gss_ctx_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Tree:
    """A prepared graph + spanning tree (gss_tree).  Keeps the device arrays alive."""

    def __init__(self, ctx, row_ptr, col, w, parent, trusted=False):
        self.ctx = ctx
        self.arrays = (row_ptr, col, w, parent)  # the library borrows them
        n = parent.numel()
        csr = Csr(n, col.numel(), row_ptr.data_ptr(), col.data_ptr() if col.numel() else None,
                  w.data_ptr() if w.numel() else None)
        self.n = n
        self.handle = ctypes.c_void_p()
        st = ctx.lib.gss_tree_prep(ctx.handle, ctypes.byref(csr), _ptr(parent),
                                   GSS_PREP_TRUSTED if trusted else 0, ctypes.byref(self.handle))
        ctx.check(st)
        self.m = ctx.lib.gss_tree_num_edges(self.handle)

    @classmethod
    def from_graph(cls, ctx, g, device="cuda", trusted=False):
        """Copies a synth.Graph to the device and prepares it."""
        t = lambda a: torch.from_numpy(a).to(device)  # noqa: E731
        return cls(ctx, t(g.row_ptr), t(g.col), t(g.w), t(g.parent), trusted)

    def rank_attempts(self):
        return int(self.ctx.lib.gss_tree_rank_attempts(self.handle))

    def export(self):
        dev = self.arrays[3].device
        depth = torch.empty(self.n, dtype=torch.int32, device=dev)
        dlo = torch.empty(self.n, dtype=torch.int64, device=dev)
        dhi = torch.empty(self.n, dtype=torch.int64, device=dev)
        scale = ctypes.c_int32()
        self.ctx.check(self.ctx.lib.gss_tree_export(self.handle, _ptr(depth), _ptr(dlo), _ptr(dhi),
                                                    ctypes.byref(scale)))
        return depth, dlo, dhi, scale.value

    def edge_lca(self, beta):
        dev = self.arrays[3].device
        lca = torch.empty(self.m, dtype=torch.int32, device=dev)
        bstar = torch.empty(self.m, dtype=torch.int32, device=dev)
        self.ctx.check(self.ctx.lib.gss_edge_lca(self.ctx.handle, self.handle, int(beta), _ptr(lca),
                                                 _ptr(bstar)))
        return lca, bstar

    def target_count(self, alpha, k_override=-1):
        """K as the library computes it (gss_target_count)."""
        p = Params(float(alpha), 0, 0, int(k_override), 0, 0)
        k = self.ctx.lib.gss_target_count(self.handle, 0, ctypes.byref(p))
        if k < 0:
            raise GSSError(-1, "bad arguments for gss_target_count")
        return int(k)

    def recover(self, alpha, beta, k_override=-1, sched=SCHED_EDGECOUNT, mask_tree=False,
                want_order=True, want_stretch=False, out=None, record=False, stats=False, key_rt=False,
                loose=False):
        """Runs gss_recover.  Returns (status, mask, order, stretch, info dict).  key_rt: order
        by R_T alone; loose: feGRASS's loose similarity with the constant radius beta."""
        dev = self.arrays[3].device
        k = self.target_count(alpha, k_override)
        if out is None:
            mask = torch.empty(max(self.m, 1), dtype=torch.uint8, device=dev)
            order = torch.empty(max(k, 1), dtype=torch.int32, device=dev) if want_order else None
            stretch = torch.empty(max(self.m, 1), dtype=torch.float64, device=dev) if want_stretch else None
        else:
            mask, order, stretch = out
        flags = (GSS_F_MASK_TREE if mask_tree else 0) | (GSS_F_RECORD if record else 0) | \
            (GSS_F_STATS if stats else 0) | (GSS_F_KEY_RT if key_rt else 0) | (GSS_F_LOOSE if loose else 0)
        p = Params(float(alpha), int(beta), int(sched), int(k_override), flags, 0)
        info = Info()
        st = self.ctx.lib.gss_recover(self.ctx.handle, self.handle, ctypes.byref(p), _ptr(mask),
                                      _ptr(order), _ptr(stretch), ctypes.byref(info))
        self.ctx.check(st)
        return st, mask[: self.m], (order[:k] if order is not None else None), \
            (stretch[: self.m] if stretch is not None else None), info.as_dict()

    def free(self):
        if self.handle:
            self.ctx.lib.gss_tree_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Batch:
    """Many graphs prepared as one union (gss_batch_prep) and recovered together."""

    def __init__(self, ctx, graphs, device="cuda", trusted=False, arrays=None):
        """graphs: synth.Graph list; arrays: optional device tensors (row_ptr, col, w, parent)
        per graph, already resident (else they are copied from the graphs)."""
        self.ctx = ctx
        self.graphs = list(graphs)
        nb = len(self.graphs)
        t = lambda a: torch.from_numpy(a).to(device)  # noqa: E731
        # kept alive with the batch: graphs prepared on their own are borrowed, not copied
        self.arrays = arrays if arrays is not None else \
            [(t(g.row_ptr), t(g.col), t(g.w), t(g.parent)) for g in self.graphs]
        csrs = (Csr * nb)()
        parents = (ctypes.c_void_p * nb)()
        for i, (rp, col, w, par) in enumerate(self.arrays):
            csrs[i] = Csr(par.numel(), col.numel(), rp.data_ptr(), col.data_ptr() if col.numel() else None,
                          w.data_ptr() if w.numel() else None)
            parents[i] = par.data_ptr()
        self.handle = ctypes.c_void_p()
        st = ctx.lib.gss_batch_prep(ctx.handle, nb, ctypes.cast(csrs, ctypes.c_void_p),
                                    ctypes.cast(parents, ctypes.c_void_p), GSS_PREP_TRUSTED if trusted else 0,
                                    ctypes.byref(self.handle))
        ctx.check(st)
        self.m = [ctx.lib.gss_tree_graph_edges(self.handle, i) for i in range(nb)]
        self.n = [g.n for g in self.graphs]

    def _params(self, alphas, beta, sched, k_override, record, stats=False, loose=False):
        nb = len(self.graphs)
        params = (Params * nb)()
        for i in range(nb):
            params[i] = Params(float(alphas[i]), int(beta), int(sched),
                               int(k_override[i]) if k_override is not None else -1,
                               (GSS_F_RECORD if record else 0) | (GSS_F_STATS if stats else 0) |
                               (GSS_F_LOOSE if loose else 0), 0)
        return params

    def autotune(self, cache_path=None, sched=SCHED_EDGECOUNT):
        """Picks the work-queue settings for this batch; returns (local_max, blocks, chunk, ms)."""
        nb = len(self.graphs)
        params = self._params([g.alpha for g in self.graphs], self.graphs[0].beta, sched, None, False)
        dev = torch.device("cuda")
        masks = [torch.empty(max(self.m[i], 1), dtype=torch.uint8, device=dev) for i in range(nb)]
        mp = (ctypes.c_void_p * nb)(*[m.data_ptr() for m in masks])
        lm, lb, ch, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        self.ctx.check(self.ctx.lib.gss_autotune(self.ctx.handle, self.handle, ctypes.cast(params, ctypes.c_void_p),
                                                 ctypes.cast(mp, ctypes.c_void_p), None,
                                                 cache_path.encode() if cache_path else None,
                                                 ctypes.byref(lm), ctypes.byref(lb), ctypes.byref(ch),
                                                 ctypes.byref(ms)))
        return lm.value, lb.value, ch.value, ms.value

    def target_counts(self, alphas, k_override=None):
        """Per-graph K as the library computes it (gss_target_count)."""
        out = []
        for i in range(len(self.graphs)):
            p = Params(float(alphas[i]), 0, 0, int(k_override[i]) if k_override is not None else -1, 0, 0)
            k = self.ctx.lib.gss_target_count(self.handle, i, ctypes.byref(p))
            if k < 0:
                raise GSSError(-1, "bad arguments for gss_target_count")
            out.append(int(k))
        return out

    def recover(self, alphas=None, beta=None, sched=SCHED_EDGECOUNT, k_override=None, out=None, record=False,
                stats=False, loose=False):
        """Returns (status, masks, orders, infos) lists over the graphs."""
        nb = len(self.graphs)
        dev = torch.device("cuda")
        alphas = [g.alpha for g in self.graphs] if alphas is None else alphas
        beta = self.graphs[0].beta if beta is None else beta
        ks = self.target_counts(alphas, k_override)
        if out is None:
            masks = [torch.empty(max(self.m[i], 1), dtype=torch.uint8, device=dev) for i in range(nb)]
            orders = [torch.empty(max(ks[i], 1), dtype=torch.int32, device=dev) for i in range(nb)]
        else:
            masks, orders = out
        params = self._params(alphas, beta, sched, k_override, record, stats, loose)
        mp = (ctypes.c_void_p * nb)(*[m.data_ptr() for m in masks])
        op = (ctypes.c_void_p * nb)(*[o.data_ptr() for o in orders])
        infos = (Info * nb)()
        st = self.ctx.lib.gss_recover_batch(self.ctx.handle, self.handle, ctypes.cast(params, ctypes.c_void_p),
                                            ctypes.cast(mp, ctypes.c_void_p), ctypes.cast(op, ctypes.c_void_p),
                                            ctypes.cast(infos, ctypes.c_void_p))
        self.ctx.check(st)
        return st, [masks[i][: self.m[i]] for i in range(nb)], [orders[i][: ks[i]] for i in range(nb)], \
            [infos[i].as_dict() for i in range(nb)]

    def free(self):
        if self.handle:
            self.ctx.lib.gss_tree_free(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass
