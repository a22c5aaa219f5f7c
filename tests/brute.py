"""Brute-force, exact reference pieces used to pin the oracle on tiny inputs.

Nothing here shares code with oracle/ or with the GPU library: tree distances come from
plain BFS over the tree's adjacency, path resistances from exact rational sums along
explicit root paths, and the greedy from an all-pairs scan.
"""
from __future__ import annotations

import math
from collections import deque
from fractions import Fraction

import numpy as np


def edges_of(g):
    """(eu, ev, ew) in edge-id order and the tree-edge flags."""
    eu, ev, ew = g.upper_edges()
    par = g.parent
    is_tree = np.array([par[a] == b or par[b] == a for a, b in zip(eu, ev)], dtype=bool)
    return eu.astype(np.int64), ev.astype(np.int64), ew, is_tree


def tree_adj(g):
    adj = [[] for _ in range(g.n)]
    for x in range(g.n):
        p = int(g.parent[x])
        if p >= 0:
            adj[x].append(p)
            adj[p].append(x)
    return adj


def tree_dist_from(adj, src):
    """Hop distance on the tree from src to every vertex (BFS)."""
    d = [-1] * len(adj)
    d[src] = 0
    q = deque([src])
    while q:
        x = q.popleft()
        for y in adj[x]:
            if d[y] < 0:
                d[y] = d[x] + 1
                q.append(y)
    return d


def root_path(g, x):
    """Vertices on the path x -> root, x first."""
    out = [int(x)]
    while g.parent[out[-1]] >= 0:
        out.append(int(g.parent[out[-1]]))
    return out


def weight_of(g, a, b):
    r0, r1 = g.row_ptr[a], g.row_ptr[a + 1]
    k = r0 + int(np.searchsorted(g.col[r0:r1], b))
    assert g.col[k] == b
    return float(g.w[k])


def lca_naive(g, a, b):
    pa = root_path(g, a)
    sb = set(root_path(g, b))
    for x in pa:
        if x in sb:
            return x
    raise AssertionError("no common ancestor")


def exact_path_resistance(g, a, b):
    """Exact rational sum of RN(1/w) over the tree path a..b (walks both root paths)."""
    l = lca_naive(g, a, b)
    total = Fraction(0)
    for s in (a, b):
        x = s
        while x != l:
            p = int(g.parent[x])
            total += Fraction(1.0 / weight_of(g, x, p))
            x = p
    return total, l


def depth_bfs(g):
    adj = tree_adj(g)
    root = int(np.flatnonzero(g.parent < 0)[0])
    return np.array(tree_dist_from(adj, root), dtype=np.int64)


def stretch_exact(g, c):
    """Per off-tree edge: (stretch, lca, beta*) from exact arithmetic and brute trees."""
    eu, ev, ew, is_tree = edges_of(g)
    dep = depth_bfs(g)
    out = {}
    for e in np.flatnonzero(~is_tree):
        a, b = int(eu[e]), int(ev[e])
        R, l = exact_path_resistance(g, a, b)
        s = ew[e] * float(R)  # float(Fraction) rounds to nearest, ties to even
        beta = min(int(dep[a] - dep[l]), int(dep[b] - dep[l]), c)
        out[int(e)] = (s, l, beta)
    return out


def greedy_brute(g, c, k):
    """The serial greedy of the paper's recovery step, from scratch, all-pairs.

    Returns (order, passes).  Similarity uses tree BFS distances: x in S_u iff
    dist_T(x,u) <= beta*(e).
    """
    eu, ev, ew, is_tree = edges_of(g)
    info = stretch_exact(g, c)
    off = sorted(info, key=lambda e: (-info[e][0], e))
    adj = tree_adj(g)
    dist_cache = {}

    def dist(src):
        if src not in dist_cache:
            dist_cache[src] = tree_dist_from(adj, src)
        return dist_cache[src]

    recovered = []
    rec_set = set()
    passes = 0
    while len(recovered) < k:
        marked = set()
        got = 0
        for i, e in enumerate(off):
            if len(recovered) == k:
                break
            if e in rec_set or e in marked:
                continue
            recovered.append(e)
            rec_set.add(e)
            got += 1
            u, v, beta = int(eu[e]), int(ev[e]), info[e][2]
            du, dv = dist(u), dist(v)
            for f in off[i + 1:]:
                if f in rec_set:
                    continue
                x, y = int(eu[f]), int(ev[f])
                if (du[x] <= beta and dv[y] <= beta) or (dv[x] <= beta and du[y] <= beta):
                    marked.add(f)
        if got == 0:
            break
        passes += 1
    return recovered, passes


def strictly_similar(dist_fn, eu, ev, bstar, e, f):
    """Is off-tree edge f strictly similar to e under e's beta*?"""
    u, v, beta = int(eu[e]), int(ev[e]), int(bstar[e])
    x, y = int(eu[f]), int(ev[f])
    du, dv = dist_fn(u), dist_fn(v)
    return (du[x] <= beta and dv[y] <= beta) or (dv[x] <= beta and du[y] <= beta)


def pinv_resistance(g, pairs):
    """Effective resistance of vertex pairs in the tree alone, via the dense pseudo-inverse."""
    n = g.n
    Lt = np.zeros((n, n))
    for x in range(n):
        p = int(g.parent[x])
        if p >= 0:
            w = weight_of(g, x, p)
            Lt[x, x] += w
            Lt[p, p] += w
            Lt[x, p] -= w
            Lt[p, x] -= w
    Lp = np.linalg.pinv(Lt)
    out = []
    for a, b in pairs:
        out.append(Lp[a, a] + Lp[b, b] - 2 * Lp[a, b])
    return np.array(out)


def laplacian(n, eu, ev, ew):
    import scipy.sparse as sp
    rows = np.concatenate([eu, ev, eu, ev])
    cols = np.concatenate([ev, eu, eu, ev])
    vals = np.concatenate([-ew, -ew, ew, ew])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()


def pcg_iterations(g, keep_mask, tol=1e-6, seed=0, maxiter=5000):
    """PCG iterations on grounded L_G with grounded L_P (P = edges in keep_mask)."""
    import scipy.sparse.linalg as spla
    eu, ev, ew, _ = edges_of(g)
    n = g.n
    LG = laplacian(n, eu, ev, ew)
    k = keep_mask.astype(bool)
    LP = laplacian(n, eu[k], ev[k], ew[k])
    root = int(np.flatnonzero(g.parent < 0)[0])
    keep = np.array([i for i in range(n) if i != root])
    A = LG[keep][:, keep].tocsc()
    Pm = LP[keep][:, keep].tocsc()
    solve = spla.factorized(Pm)
    b = np.random.default_rng(seed).standard_normal(n - 1)
    M = spla.LinearOperator(A.shape, matvec=solve)
    it = [0]

    def cb(_):
        it[0] += 1

    x, info = spla.cg(A, b, rtol=tol, atol=0.0, M=M, maxiter=maxiter, callback=cb)
    assert info == 0
    assert np.linalg.norm(A @ x - b) <= tol * np.linalg.norm(b) * 1.0001
    return it[0]


def log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def greedy_brute_variant(g, c, k, key_rt=False, loose=False):
    """The greedy with the two variants, from the definitions, all-pairs.

    key_rt: edges ordered by the exact tree-path resistance R_T (rounded once), ties by
    id, instead of the stretch.  loose: feGRASS's condition (eq. cond-loose-2): a later
    edge is marked when either endpoint is within the constant c tree hops of u or of v.
    Returns (order, passes)."""
    eu, ev, ew, is_tree = edges_of(g)
    dep = depth_bfs(g)
    key, bstar = {}, {}
    for e in np.flatnonzero(~is_tree):
        a, b = int(eu[e]), int(ev[e])
        R, l = exact_path_resistance(g, a, b)
        key[int(e)] = float(R) if key_rt else ew[e] * float(R)
        bstar[int(e)] = min(int(dep[a] - dep[l]), int(dep[b] - dep[l]), c)
    off = sorted(key, key=lambda e: (-key[e], e))
    adj = tree_adj(g)
    cache = {}

    def dist(src):
        if src not in cache:
            cache[src] = tree_dist_from(adj, src)
        return cache[src]

    recovered, rec_set, passes = [], set(), 0
    while len(recovered) < k:
        marked, got = set(), 0
        for i, e in enumerate(off):
            if len(recovered) == k:
                break
            if e in rec_set or e in marked:
                continue
            recovered.append(e)
            rec_set.add(e)
            got += 1
            u, v = int(eu[e]), int(ev[e])
            du, dv = dist(u), dist(v)
            r = c if loose else bstar[e]
            for f in off[i + 1:]:
                if f in rec_set:
                    continue
                x, y = int(eu[f]), int(ev[f])
                if loose:
                    hit = min(du[x], dv[x]) <= r or min(du[y], dv[y]) <= r
                else:
                    hit = (du[x] <= r and dv[y] <= r) or (dv[x] <= r and du[y] <= r)
                if hit:
                    marked.add(f)
        if got == 0:
            break
        passes += 1
    return recovered, passes
