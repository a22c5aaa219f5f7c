"""Seeded synthetic inputs: weighted undirected graphs plus a spanning-tree parent array.

This module only *builds inputs*. It holds none of the recovery method's arithmetic
(no LCA, no resistance, no stretch, no similarity): both the CPU oracle and the GPU
path consume what it produces.

Conventions shared by every generator
-------------------------------------
* Undirected edges are listed once as (u, v) with u < v, sorted by (u, v).  This is
  the *edge id* order: id = rank of (u, v) among the upper-triangle CSR entries.
* Weights are float64, drawn per undirected edge in edge-id order.
* The graph is returned as a symmetric CSR (rows ascending, columns ascending within
  a row, no self-loops, no duplicates) with int32 indices.
* The spanning tree is the maximum-weight spanning tree under the total order
  (w descending, id ascending).  With that order all keys are distinct, so the tree
  is unique and any MST routine returns it.  It is rooted at the lowest-id vertex of
  maximum degree in G, and ``parent`` comes from a BFS over the tree (root: -1).

The paper evaluates on public sparse-matrix graphs (meshes, redistricting graphs,
social and collaboration networks) that are not available here; grids and random
geometric graphs stand in for the uniform ones and R-MAT for the skewed ones.
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

__all__ = [
    "Graph", "grid", "rmat", "rgg", "random_connected", "path_graph", "star_graph", "skewed_cost",
    "from_edges", "max_spanning_tree_parent", "config", "batch_config", "CONFIGS",
    "k_of", "data_dir",
]


class Graph:
    """A CSR graph plus its rooted spanning tree.  All arrays are host numpy arrays."""

    def __init__(self, n, row_ptr, col, w, parent, root, alpha=0.02, beta=2, name="graph"):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.parent = np.ascontiguousarray(parent, dtype=np.int32)
        self.root = int(root)
        self.alpha = float(alpha)
        self.beta = int(beta)
        self.name = name

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    @property
    def m(self):
        return self.nnz // 2

    def upper_edges(self):
        """(eu, ev, ew) in edge-id order."""
        rows = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        keep = self.col > rows
        return rows[keep].astype(np.int32), self.col[keep], self.w[keep]

    def __repr__(self):
        return f"Graph({self.name}: n={self.n}, m={self.m}, alpha={self.alpha}, beta={self.beta})"


def k_of(alpha, n, k_override=-1):
    """Number of edges to recover: floor(fl(alpha * n)) unless overridden."""
    if k_override >= 0:
        return int(k_override)
    return int(math.floor(float(alpha) * float(n)))


# ----------------------------------------------------------------------------------------
# assembly helpers
# ----------------------------------------------------------------------------------------

def _sort_edges(u, v, w=None):
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    # one int64 key per edge orders like (a, b); inputs that are already in order (most
    # generators emit them so) skip the sort
    key = a * (int(b.max(initial=0)) + 1) + b
    if key.size > 1 and not bool(np.all(key[1:] >= key[:-1])):
        o = np.argsort(key, kind="stable")
        a, b = a[o], b[o]
        if w is not None:
            w = np.asarray(w, dtype=np.float64)[o]
    if w is None:
        return a, b
    return a, b, np.asarray(w, dtype=np.float64)


def to_csr(n, eu, ev, ew):
    """Symmetric CSR from upper edges (eu < ev) in edge-id order, columns sorted in each row.

    A counting sort by row keeps the input order inside a row.  Listing the mirrored
    entries (row ev, column eu) before the upper ones (row eu, column ev) therefore gives
    sorted rows: for a fixed row r the mirrored entries have columns < r in ascending
    order (edge-id order sorts them by eu), the upper ones columns > r in ascending order.
    """
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    ew = np.asarray(ew, dtype=np.float64)
    if 2 * len(eu) >= 2 ** 31:
        raise ValueError("graph too large for int32 CSR")
    rows = np.concatenate([ev, eu]).astype(np.int32)
    cols = np.concatenate([eu, ev]).astype(np.int32)
    vals = np.concatenate([ew, ew])
    # scipy's COO -> CSR conversion is such a counting sort (linear, input order kept
    # within a row); the rows come out sorted, so no entry moves afterwards
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    del rows, cols, vals
    if not A.has_sorted_indices or A.nnz != 2 * len(eu):
        raise ValueError("edges are not simple or not in edge-id order")
    return A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64)


def max_spanning_tree_parent(n, eu, ev, ew, root=None):
    """Parent array of the maximum spanning tree under (w desc, id asc), BFS-rooted.

    Edges must be given in edge-id order.  Raises if G is disconnected.

    The tree is found by a filtered Kruskal: the spanning forest F of the edges heavier
    than the (4n)-th largest weight first, then the spanning tree of F plus the other
    edges that join two components of F.  Such a lighter edge inside one component of F
    is the lightest edge of a cycle, so it is in no maximum spanning tree; the keys
    (w desc, id asc) are distinct, so the tree is unique and equals the one of the whole
    graph.
    """
    eu = np.asarray(eu, dtype=np.int64)
    ev = np.asarray(ev, dtype=np.int64)
    w = np.asarray(ew, dtype=np.float64)
    m = len(eu)
    deg = np.bincount(eu, minlength=n) + np.bincount(ev, minlength=n)
    if root is None:
        root = int(np.argmax(deg))  # lowest id among the maximum-degree vertices
    if n == 1:
        return np.array([-1], dtype=np.int32), root
    rank = np.zeros(m, dtype=np.float64)
    by_rank = []  # edge ids in (w desc, id asc) order, one array per group

    def ranked(sel):
        """Gives the edges sel (ascending ids, all lighter than every edge ranked so far)
        the next ranks in (w desc, id asc) order."""
        o = sel[np.argsort(-w[sel], kind="stable")]
        start = sum(len(x) for x in by_rank)
        rank[o] = np.arange(start + 1, start + len(o) + 1, dtype=np.float64)
        by_rank.append(o)

    def msf(sel):
        sel = np.sort(sel)
        A = sp.coo_matrix((rank[sel], (eu[sel], ev[sel])), shape=(n, n)).tocsr()
        T = csg.minimum_spanning_tree(A).tocoo()
        return np.concatenate(by_rank)[T.data.astype(np.int64) - 1]  # rank r is by_rank[r - 1]

    h = min(m, 4 * n)
    if h < m:
        thr = np.partition(w, m - h)[m - h]  # the h-th largest weight
        heavy = np.flatnonzero(w > thr)
        light = np.flatnonzero(w <= thr)
    else:
        heavy = np.arange(m)
        light = np.zeros(0, dtype=np.int64)
    ranked(heavy)
    forest = msf(heavy)
    if len(light):
        F = sp.coo_matrix((np.ones(len(forest), dtype=np.int8), (eu[forest], ev[forest])), shape=(n, n))
        _, lab = csg.connected_components(F, directed=False)
        light = light[lab[eu[light]] != lab[ev[light]]]
        ranked(light)
        forest = msf(np.concatenate([forest, light]))
    if len(forest) != n - 1:
        raise ValueError("graph is not connected")
    T = sp.coo_matrix((np.ones(n - 1, dtype=np.int8), (eu[forest], ev[forest])), shape=(n, n)).tocsr()
    bfs, pred = csg.breadth_first_order(T, root, directed=False, return_predecessors=True)
    if len(bfs) != n:
        raise ValueError("graph is not connected")
    parent = pred.astype(np.int64)
    parent[root] = -1
    return parent.astype(np.int32), root


def from_edges(n, eu, ev, ew, alpha=0.02, beta=2, name="graph", parent=None, root=None):
    eu, ev, ew = _sort_edges(eu, ev, ew)
    if parent is None:
        parent, root = max_spanning_tree_parent(n, eu, ev, ew, root)
    row_ptr, col, w = to_csr(n, eu, ev, ew)
    if root is None:
        root = int(np.flatnonzero(np.asarray(parent) < 0)[0])
    return Graph(n, row_ptr, col, w, parent, root, alpha, beta, name)


def _largest_cc(n, x, y):
    """Largest connected component of the edges (x, y), compactly relabelled in id order
    (x, y sorted by (x, y), so the upper-triangle CSR is built without a sort)."""
    x = np.asarray(x, dtype=np.int64)
    y = np.asarray(y, dtype=np.int64)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(x, minlength=n), out=indptr[1:])
    A = sp.csr_matrix((np.ones(len(x), dtype=np.int8), y, indptr), shape=(n, n))
    _, lab = csg.connected_components(A, directed=False)
    big = np.argmax(np.bincount(lab))
    keepv = lab == big
    newid = np.full(n, -1, dtype=np.int64)
    newid[keepv] = np.arange(int(keepv.sum()))
    ke = keepv[x]
    return int(keepv.sum()), newid[x[ke]], newid[y[ke]]


# ----------------------------------------------------------------------------------------
# workload families
# ----------------------------------------------------------------------------------------

def grid(dims, wlo, whi, seed=0, alpha=0.02, beta=2, name=None):
    """d-dimensional 2d-connected grid; vertex id is row-major; w log-uniform in [wlo, whi)."""
    rng = np.random.default_rng(seed)
    idx = np.arange(int(np.prod(dims)), dtype=np.int64).reshape(dims)
    us, vs = [], []
    for ax in range(len(dims)):
        s0 = [slice(None)] * len(dims)
        s1 = [slice(None)] * len(dims)
        s0[ax] = slice(0, -1)
        s1[ax] = slice(1, None)
        us.append(idx[tuple(s0)].ravel())
        vs.append(idx[tuple(s1)].ravel())
    eu, ev = _sort_edges(np.concatenate(us), np.concatenate(vs))
    ew = np.exp(rng.uniform(math.log(wlo), math.log(whi), len(eu)))
    return from_edges(idx.size, eu, ev, ew, alpha, beta,
                      name or "grid" + "x".join(map(str, dims)))


def _log(msg):
    """Progress line for long generator runs (GSS_VERBOSE=1)."""
    if os.environ.get("GSS_VERBOSE") == "1":
        print(f"[synth] {msg}", file=sys.stderr, flush=True)


def rmat(scale, avg_deg=16, a=0.57, b=0.19, c=0.19, seed=0, alpha=0.10, beta=2, name=None):
    """R-MAT with avg_deg*2^scale/2 samples, symmetrised, deduplicated, largest CC; w in (0,1]."""
    rng = np.random.default_rng(seed)
    nfull = 1 << scale
    samples = (avg_deg * nfull) // 2
    # vertex bits accumulate in int32 (scale <= 30); each level's draws are processed in
    # cache-sized chunks (the draw order, level by level, is unchanged)
    ab, abc = a + b, a + b + c
    u = np.zeros(samples, dtype=np.int32)
    v = np.zeros(samples, dtype=np.int32)
    r = np.empty(samples, dtype=np.float64)
    CH = 1 << 18
    bit = np.empty(CH, dtype=np.int32)
    t0 = np.empty(CH, dtype=bool)
    t1 = np.empty(CH, dtype=bool)
    for lvl in range(scale):
        rng.random(out=r)
        for s0 in range(0, samples, CH):
            rr = r[s0:s0 + CH]
            k = len(rr)
            b0, b1, bb = t0[:k], t1[:k], bit[:k]
            np.greater_equal(rr, ab, out=b0)                  # quadrants c, d set the row bit
            bb[...] = b0
            bb <<= lvl
            u[s0:s0 + k] |= bb
            np.greater_equal(rr, a, out=b1)                   # quadrant b, or d, sets the column bit
            np.logical_and(b1, np.less(rr, ab, out=b0), out=b1)
            np.logical_or(b1, np.greater_equal(rr, abc, out=b0), out=b1)
            bb[...] = b1
            bb <<= lvl
            v[s0:s0 + k] |= bb
        _log(f"rmat{scale}: level {lvl + 1}/{scale}")
    del r, bit, t0, t1
    perm = rng.permutation(nfull)
    u = perm[u]
    v = perm[v]
    keep = u != v
    u, v = u[keep], v[keep]
    x = np.minimum(u, v)
    y = np.maximum(u, v)
    del u, v, keep
    key = np.unique(x * nfull + y)
    x, y = key // nfull, key % nfull
    del key
    _log(f"rmat{scale}: {len(x)} distinct edges")
    n, x, y = _largest_cc(nfull, x, y)
    x, y = _sort_edges(x, y)
    w = 1.0 - rng.random(len(x))
    _log(f"rmat{scale}: largest component n={n} m={len(x)}; spanning tree")
    return from_edges(n, x, y, w, alpha, beta, name or f"rmat{scale}")


def rgg(n, rng, alpha=0.02, beta=2, name=None):
    """Random geometric graph in the unit square, radius for average degree ~10, w = 1/dist."""
    from scipy.spatial import cKDTree
    pts = rng.random((n, 2))
    r = math.sqrt(10.0 / (math.pi * n))
    pr = cKDTree(pts).query_pairs(r, output_type="ndarray").astype(np.int64)
    d = np.linalg.norm(pts[pr[:, 0]] - pts[pr[:, 1]], axis=1)
    ok = d > 0
    pr, d = pr[ok], d[ok]
    # the largest component, compactly relabelled; weights follow the surviving pairs
    A = sp.coo_matrix((np.ones(len(pr), dtype=np.int8), (pr[:, 0], pr[:, 1])), shape=(n, n))
    _, lab = csg.connected_components(A, directed=False)
    big = np.argmax(np.bincount(lab))
    kv = lab == big
    nid = np.full(n, -1, dtype=np.int64)
    nid[kv] = np.arange(int(kv.sum()))
    ke = kv[pr[:, 0]]
    x, y, w = nid[pr[ke, 0]], nid[pr[ke, 1]], 1.0 / d[ke]
    return from_edges(int(kv.sum()), x, y, w, alpha, beta, name or f"rgg{n}")


def random_connected(n, extra, seed=0, alpha=0.1, beta=2, wlo=1.0, whi=100.0,
                     tree="max", name=None):
    """Small random connected graph: random recursive tree + ``extra`` random edges.

    tree="max": spanning tree input is the max-weight spanning tree;
    tree="random": it is the random recursive tree used to build G (rooted at vertex 0
    after relabelling), which gives deeper, less weight-correlated trees.
    """
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    par = np.array([-1] + [int(rng.integers(0, i)) for i in range(1, n)], dtype=np.int64)
    tu = perm[np.arange(1, n)]
    tv = perm[par[1:]]
    eu = [tu]
    ev = [tv]
    if extra > 0 and n > 2:
        a = rng.integers(0, n, 3 * extra + 8)
        b = rng.integers(0, n, 3 * extra + 8)
        eu.append(a)
        ev.append(b)
    u = np.concatenate(eu)
    v = np.concatenate(ev)
    keep = u != v
    x = np.minimum(u[keep], v[keep])
    y = np.maximum(u[keep], v[keep])
    key, first = np.unique(x * n + y, return_index=True)
    # keep every tree edge and the first `extra` distinct random edges
    is_tree = first < (n - 1)
    nontree = np.flatnonzero(~is_tree)
    nontree = nontree[np.argsort(first[nontree], kind="stable")][:extra]
    sel = np.sort(np.concatenate([np.flatnonzero(is_tree), nontree]))
    key = key[sel]
    x, y = key // n, key % n
    w = np.exp(rng.uniform(math.log(wlo), math.log(whi), len(x)))
    if tree == "max":
        return from_edges(n, x, y, w, alpha, beta, name or f"rand{n}")
    parent = np.full(n, -1, dtype=np.int64)
    # orient the recursive tree from the relabelled root perm[0]
    T = sp.coo_matrix((np.ones(n - 1), (tu, tv)), shape=(n, n)).tocsr()
    T = (T + T.T).tocsr()
    root = int(perm[0])
    _, pred = csg.breadth_first_order(T, root, directed=False, return_predecessors=True)
    parent[:] = pred
    parent[root] = -1
    return from_edges(n, x, y, w, alpha, beta, name or f"rand{n}", parent=parent.astype(np.int32),
                      root=root)


def path_graph(n, extra, seed=0, alpha=0.5, beta=2):
    """Path 0-1-...-(n-1) as the tree (rooted at 0, an end) plus random chords."""
    rng = np.random.default_rng(seed)
    tu = np.arange(n - 1)
    tv = tu + 1
    a = rng.integers(0, n, 4 * extra + 8)
    b = rng.integers(0, n, 4 * extra + 8)
    keep = np.abs(a - b) > 1
    x = np.minimum(a[keep], b[keep])
    y = np.maximum(a[keep], b[keep])
    key = np.unique(x * n + y)[:extra]
    x = np.concatenate([tu, key // n])
    y = np.concatenate([tv, key % n])
    w = np.exp(rng.uniform(0.0, math.log(100.0), len(x)))
    parent = np.concatenate([[-1], np.arange(n - 1)]).astype(np.int32)
    return from_edges(n, x, y, w, alpha, beta, f"path{n}", parent=parent, root=0)


def star_graph(n, extra, seed=0, alpha=0.5, beta=2):
    """Star rooted at 0 as the tree plus random leaf-leaf chords."""
    rng = np.random.default_rng(seed)
    tu = np.zeros(n - 1, dtype=np.int64)
    tv = np.arange(1, n)
    a = rng.integers(1, n, 4 * extra + 8)
    b = rng.integers(1, n, 4 * extra + 8)
    keep = a != b
    x = np.minimum(a[keep], b[keep])
    y = np.maximum(a[keep], b[keep])
    key = np.unique(x * n + y)[:extra]
    x = np.concatenate([tu, key // n])
    y = np.concatenate([tv, key % n])
    w = np.exp(rng.uniform(0.0, math.log(100.0), len(x)))
    parent = np.concatenate([[-1], np.zeros(n - 1)]).astype(np.int32)
    return from_edges(n, x, y, w, alpha, beta, f"star{n}", parent=parent, root=0)


def skewed_cost(nheavy, nlight, side=16, seed=0, beta=2, name=None):
    """A forest of LCA gadgets under one root whose subtasks all hold side^2 off-tree
    edges but cost very differently in the greedy, so a queue ordered by edge count
    cannot tell them apart.

    light gadget: LCA x with children a and b, each with `side` leaves; the off-tree
      edges join every leaf of a to every leaf of b (beta* = 2: the first recovered edge
      marks all the others, one candidate per subtask);
    heavy gadget: LCA y with `side` children, each with `side` leaves; the off-tree edges
      join y to every grandchild (beta* = 0: nothing is marked, every edge is a candidate).
    Heavy gadgets get the highest vertex ids.  Weights are drawn from [1, 10); the tree is
    given (not a maximum spanning tree), rooted at vertex 0.  K should be the number of
    candidates, nlight + side^2 * nheavy, so that one pass over every edge recovers it."""
    rng = np.random.default_rng(seed)
    S = side * side
    nl_v = 3 + 2 * side
    nh_v = 1 + side + S
    n = 1 + nlight * nl_v + nheavy * nh_v
    parent = np.full(n, -1, dtype=np.int64)
    eu, ev = [], []
    base = 1
    for _ in range(nlight):
        x, a, b = base, base + 1, base + 2
        la = np.arange(base + 3, base + 3 + side)
        lb = la + side
        parent[[x, a, b]] = [0, x, x]
        parent[la] = a
        parent[lb] = b
        eu.append(np.repeat(la, side))
        ev.append(np.tile(lb, side))
        base += nl_v
    for _ in range(nheavy):
        y = base
        ch = np.arange(base + 1, base + 1 + side)
        gc = np.arange(base + 1 + side, base + 1 + side + S)
        parent[y] = 0
        parent[ch] = y
        parent[gc] = np.repeat(ch, side)
        eu.append(np.full(S, y))
        ev.append(gc)
        base += nh_v
    tx = np.arange(1, n)
    eu = np.concatenate([tx] + eu)
    ev = np.concatenate([parent[1:]] + ev)
    w = rng.uniform(1.0, 10.0, len(eu))
    return from_edges(n, eu, ev, w, 1.0, beta, name or f"skewed{nheavy}x{nlight}", parent=parent.astype(np.int32),
                      root=0)


# ----------------------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------------------

CONFIGS = {
    # 2D 4-connected grid 64x64, w log-uniform [1,100], alpha 0.02, beta 2
    "grid2d_64": dict(kind="grid", dims=(64, 64), wlo=1.0, whi=100.0, alpha=0.02, beta=2),
    # 3D 7-point grid 128^3, w log-uniform [1,1e4], alpha 0.05, beta 2
    "grid3d_128": dict(kind="grid", dims=(128, 128, 128), wlo=1.0, whi=1e4, alpha=0.05, beta=2),
    # R-MAT scale 22, avg degree 16, (.57,.19,.19,.05), LCC, w uniform (0,1], alpha 0.10
    "rmat22": dict(kind="rmat", scale=22, alpha=0.10, beta=2),
    # learned-scheduling pair: R-MAT scale 24 and 3D grid 160^3, alpha 0.10
    "rmat24": dict(kind="rmat", scale=24, alpha=0.10, beta=2),
    "grid3d_160": dict(kind="grid", dims=(160, 160, 160), wlo=1.0, whi=1e4, alpha=0.10, beta=2),
    # scaled-down stand-ins used by fast tests
    "grid3d_32": dict(kind="grid", dims=(32, 32, 32), wlo=1.0, whi=1e4, alpha=0.05, beta=2),
    "rmat14": dict(kind="rmat", scale=14, alpha=0.10, beta=2),
    "rmat16": dict(kind="rmat", scale=16, alpha=0.10, beta=2),
}

_GEN_VERSION = 1


def data_dir():
    d = os.environ.get("GSS_DATA_DIR")
    if not d:
        d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_data")
    os.makedirs(d, exist_ok=True)
    return d


def _save(g, path):
    tmp = path + ".tmp.npz"
    np.savez(tmp, n=g.n, row_ptr=g.row_ptr, col=g.col, w=g.w, parent=g.parent, root=g.root,
             alpha=g.alpha, beta=g.beta)
    os.replace(tmp, path)


def _load(path, name):
    with np.load(path, allow_pickle=False) as z:
        return Graph(int(z["n"]), z["row_ptr"], z["col"], z["w"], z["parent"], int(z["root"]),
                     float(z["alpha"]), int(z["beta"]), name)


def config(name, seed=0, cache=True):
    """Build (or load from the on-disk cache) one named workload."""
    spec = CONFIGS[name]
    path = os.path.join(data_dir(), f"{name}_s{seed}_v{_GEN_VERSION}.npz")
    if cache and os.path.exists(path):
        return _load(path, name)
    if spec["kind"] == "grid":
        g = grid(spec["dims"], spec["wlo"], spec["whi"], seed, spec["alpha"], spec["beta"], name)
    elif spec["kind"] == "rmat":
        g = rmat(spec["scale"], seed=seed, alpha=spec["alpha"], beta=spec["beta"], name=name)
    else:
        raise KeyError(name)
    if cache:
        _save(g, path)
    return g


def batch_config(count=64, nmin=1e4, nmax=1e6, seed=0, cache=True):
    """Batch of random geometric graphs, sizes log-uniform in [nmin, nmax), alpha in {.02,.05,.10}."""
    rng = np.random.default_rng(seed)
    ns = np.floor(np.exp(rng.uniform(math.log(nmin), math.log(nmax), count))).astype(np.int64)
    alphas = rng.choice(np.array([0.02, 0.05, 0.10]), count)
    out = []
    for i in range(count):
        path = os.path.join(data_dir(), f"rgg_b{count}_{int(nmin)}_{int(nmax)}_s{seed}_{i}_v{_GEN_VERSION}.npz")
        if cache and os.path.exists(path):
            g = _load(path, f"rgg{i}")
            # keep the generator stream aligned with an uncached run
            rng.random((int(ns[i]), 2))
        else:
            g = rgg(int(ns[i]), rng, float(alphas[i]), 2, f"rgg{i}")
            if cache:
                _save(g, path)
        out.append(g)
    return out
