"""Error paths of the GPU library: the same invalid inputs as the oracle's status-code
test must give the same status through the C ABI (nothing here faults: every input is
rejected by the library's own checks before it could be used to index memory)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2508_20403_amd import gss, synth
from tests.test_oracle_pins import RANGE_CASES, graph_from_json, range_case_graph

pytestmark = pytest.mark.gpu


def gpu_status(ctx, g, *, row_ptr=None, col=None, w=None, parent=None, alpha=None, beta=None):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    rp = t(g.row_ptr if row_ptr is None else row_ptr)
    c = t(g.col if col is None else col)
    ww = t(g.w if w is None else w)
    p = t(g.parent if parent is None else parent)
    print(f"[gpu-err] {g.name}", flush=True)
    try:
        tree = gss.Tree(ctx, rp, c, ww, p)
    except gss.GSSError as e:
        return e.status
    try:
        st = tree.recover(g.alpha if alpha is None else alpha, g.beta if beta is None else beta)[0]
    except gss.GSSError as e:
        st = e.status
    tree.free()
    return st


def both(ctx, g, **kw):
    o = oracle.recover(**{**dict(n=g.n, row_ptr=g.row_ptr, col=g.col, w=g.w, parent=g.parent, alpha=g.alpha,
                                 beta=g.beta), **kw}).status
    return gpu_status(ctx, g, **kw), o


def test_error_statuses_match_oracle(gpu_ctx):
    g = synth.random_connected(30, 40, seed=9)
    rp, col, w, par = g.row_ptr, g.col, g.w, g.parent
    cases = []
    cases.append(dict(alpha=1.5))
    cases.append(dict(beta=-1))
    c2 = col.copy(); c2[3] = g.n + 5; cases.append(dict(col=c2))
    c2 = col.copy(); c2[rp[4]] = 4; cases.append(dict(col=c2))
    r0 = rp[7]; c2 = col.copy(); c2[r0], c2[r0 + 1] = c2[r0 + 1], c2[r0]; cases.append(dict(col=c2))
    for bad in (0.0, -1.0, np.nan, np.inf):
        w2 = w.copy(); w2[5] = bad; cases.append(dict(w=w2))
    w2 = w.copy(); w2[rp[2]] *= 2.0; cases.append(dict(w=w2))
    x = int(np.flatnonzero(par >= 0)[0])
    p2 = par.copy(); p2[x] = -1; cases.append(dict(parent=p2))
    ch = [v for v in range(g.n) if par[v] >= 0 and par[par[v]] >= 0][0]
    p2 = par.copy(); p2[par[ch]] = ch; cases.append(dict(parent=p2))
    p2 = par.copy(); p2[x] = g.n; cases.append(dict(parent=p2))
    root = int(np.flatnonzero(par < 0)[0])
    leaf = [v for v in range(g.n) if v != root and not np.any(par == v)][0]
    nb = set(col[rp[leaf]:rp[leaf + 1]].tolist())
    target = [v for v in range(g.n) if v not in nb and v != leaf][0]
    p2 = par.copy(); p2[leaf] = target; cases.append(dict(parent=p2))
    rp2 = rp.copy(); rp2[5] = rp2[6] + 1; cases.append(dict(row_ptr=rp2))
    for kw in cases:
        got, want = both(gpu_ctx, g, **kw)
        assert got == want and want < 0, (list(kw), got, want)


def test_range_error(gpu_ctx):
    edges = [[0, 1, 1.0], [1, 2, 2.0 ** 80], [2, 3, 1.0], [3, 4, 1.0], [0, 4, 1.0]]
    g = graph_from_json(5, edges, [-1, 0, 1, 2, 3])
    assert gpu_status(gpu_ctx, g) == oracle.recover(g).status == -7


@pytest.mark.parametrize("w12,ok", RANGE_CASES)
def test_range_limits_match_oracle(gpu_ctx, w12, ok):
    """Both sides of the 74-binade term limit and of the 2^127 sum limit."""
    g = range_case_graph(w12)
    st = oracle.recover(g).status
    assert (st >= 0) if ok else (st == -7)
    assert gpu_status(gpu_ctx, g) == st


def test_missing_mirror_is_asym(gpu_ctx):
    """Drop one lower entry: triangle sizes differ."""
    g = synth.random_connected(40, 60, seed=3)
    rp, col, w = g.row_ptr.copy(), g.col.copy(), g.w.copy()
    u = 10
    r0, r1 = rp[u], rp[u + 1]
    lower = [k for k in range(r0, r1) if col[k] < u]
    assert lower
    k = lower[0]
    col2 = np.delete(col, k)
    w2 = np.delete(w, k)
    rp2 = rp.copy(); rp2[u + 1:] -= 1
    o = oracle.recover(n=g.n, row_ptr=rp2, col=col2, w=w2, parent=g.parent, alpha=g.alpha, beta=g.beta).status
    assert o == -3
    assert gpu_status(gpu_ctx, g, row_ptr=rp2, col=col2, w=w2) == -3


def test_tree_only_and_tiny(gpu_ctx):
    for n in (1, 2, 5):
        g = synth.random_connected(n, 0, seed=1) if n > 1 else synth.Graph(
            1, np.zeros(2, np.int32), np.zeros(0, np.int32), np.zeros(0), np.array([-1], np.int32), 0, 0.5, 2, "one")
        st = gpu_status(gpu_ctx, g)
        assert st == oracle.recover(g, k_override=-1).status


def _swap_lower_mirror(g):
    """A CSR with as many lower as upper entries whose lower triangle is not the mirror
    of the upper one: in some row u, one lower entry (u, c) is moved to a column c' < u
    that is not a neighbour of u (the row stays sorted and simple)."""
    rp, col, w = g.row_ptr, g.col.copy(), g.w.copy()
    for u in range(g.n):
        row = col[rp[u]:rp[u + 1]]
        lower = [k for k in range(rp[u], rp[u + 1]) if col[k] < u]
        if not lower:
            continue
        k = lower[-1]
        lo = col[k - 1] + 1 if k > rp[u] else 0
        free = [c for c in range(lo, col[k]) if c not in row and c != u]
        if free:
            col[k] = free[0]
            return col, w
    raise AssertionError("no row to alter")


def test_unmirrored_lower_entry_with_equal_counts_is_asym(gpu_ctx):
    """Triangle sizes agree, so only an exact mirror check can reject this CSR."""
    g = synth.random_connected(60, 90, seed=4)
    col2, w2 = _swap_lower_mirror(g)
    o = oracle.recover(n=g.n, row_ptr=g.row_ptr, col=col2, w=w2, parent=g.parent, alpha=g.alpha, beta=g.beta)
    assert o.status == -3
    assert gpu_status(gpu_ctx, g, col=col2, w=w2) == -3


def test_swapped_lower_weights_is_asym(gpu_ctx):
    """Two lower entries exchange their weights: same columns, same multiset of weights."""
    g = synth.random_connected(60, 90, seed=6)
    rp, col, w = g.row_ptr, g.col, g.w.copy()
    lows = [k for u in range(g.n) for k in range(rp[u], rp[u + 1]) if col[k] < u]
    a, b = lows[3], lows[17]
    assert w[a] != w[b]
    w[a], w[b] = w[b], w[a]
    o = oracle.recover(n=g.n, row_ptr=rp, col=col, w=w, parent=g.parent, alpha=g.alpha, beta=g.beta)
    assert o.status == -3
    assert gpu_status(gpu_ctx, g, w=w) == -3


def _multi_tile_cases():
    """Lower entries of a CSR spanning many 4096-entry tiles (the entry checks work tile by
    tile): mirrors in the same row neighbourhood (row u - 1, searched inside the tile),
    far back (row u - 480, about 3300 entries back: in an earlier tile), and entries at
    the first and last offsets of tiles (rows that straddle a tile boundary)."""
    g = synth.grid((40, 40, 12), 1.0, 100.0, seed=5)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    lower = np.flatnonzero(g.col < rows)
    off = lower % 4096
    d = rows[lower] - g.col[lower]
    later = lower >= 2 * 4096  # tiles with earlier tiles before them
    picks = {
        "near_mid_tile": lower[later & (d == 1) & (off > 1500) & (off < 2500)][[0, 5]],
        "far_back": lower[later & (d == 480) & (off < 3000)][[0, 5]],
        "tile_first": lower[later & (off < 4)][:2],
        "tile_last": lower[later & (off > 4090)][:2],
        "row_after_tile_start": lower[later & (d == 1) & (off < 12)][:2],
    }
    return g, picks


@pytest.mark.parametrize("kind", ["near_mid_tile", "far_back", "tile_first", "tile_last", "row_after_tile_start"])
def test_asym_weight_found_across_tiles(gpu_ctx, kind):
    """One lower entry's weight changed: the mirror search must see it whether the mirror's
    row lies inside the entry's tile or not (same status as the oracle's)."""
    g, picks = _multi_tile_cases()
    ks = picks[kind]
    assert len(ks) >= 1
    for j, k in enumerate(ks):
        w = g.w.copy()
        w[k] *= 1.5
        if j == 0:
            o = oracle.recover(n=g.n, row_ptr=g.row_ptr, col=g.col, w=w, parent=g.parent, alpha=g.alpha,
                               beta=g.beta).status
            assert o == -3
        assert gpu_status(gpu_ctx, g, w=w) == -3, (kind, int(k))
    # and the unchanged graph passes
    assert gpu_status(gpu_ctx, g) >= 0


@pytest.mark.parametrize("kind", ["near_mid_tile", "far_back", "tile_first", "tile_last"])
def test_asym_column_found_across_tiles(gpu_ctx, kind):
    """One lower entry (u, c) moved to another column c' < u that is not a neighbour of u
    (rows stay sorted and simple, triangle sizes agree): only the exact mirror search can
    reject it, wherever the mirror row lies."""
    g, picks = _multi_tile_cases()
    k = int(picks[kind][0])
    rp, col = g.row_ptr, g.col.copy()
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    u = int(rows[k])
    lo = col[k - 1] + 1 if k > rp[u] else 0
    hi = col[k + 1] if k + 1 < rp[u + 1] else u
    hi = min(hi, u)
    free = [c for c in range(lo, hi) if c != col[k] and c not in set(col[rp[u]:rp[u + 1]].tolist())]
    if not free:
        pytest.skip("no free column next to this entry")
    col[k] = free[len(free) // 2]
    o = oracle.recover(n=g.n, row_ptr=rp, col=col, w=g.w, parent=g.parent, alpha=g.alpha, beta=g.beta).status
    assert o == -3
    assert gpu_status(gpu_ctx, g, col=col) == -3


def _rmat_cases():
    """R-MAT 14 (random columns): its lower entries mostly have their mirror rows outside
    their own tile, so symmetry is checked by transposition (sort by column, compare)."""
    g = synth.config("rmat14")
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    lower = np.flatnonzero(g.col < rows)
    off = lower % 4096
    later = lower >= 2 * 4096
    return g, rows, {"tile_first": lower[later & (off < 4)][0], "mid": lower[later & (off > 2000)][0],
                     "tile_last": lower[later & (off > 4090)][0], "last_entry": lower[-1]}


@pytest.mark.parametrize("kind", ["tile_first", "mid", "tile_last", "last_entry"])
def test_asym_weight_found_by_transposition(gpu_ctx, kind):
    g, rows, picks = _rmat_cases()
    k = int(picks[kind])
    w = g.w.copy()
    w[k] = w[k] * 0.5 + 1e-3
    o = oracle.recover(n=g.n, row_ptr=g.row_ptr, col=g.col, w=w, parent=g.parent, alpha=g.alpha, beta=g.beta).status
    assert o == -3
    assert gpu_status(gpu_ctx, g, w=w) == -3
    assert gpu_status(gpu_ctx, g) >= 0


def test_asym_column_found_by_transposition(gpu_ctx):
    """A lower entry moved to a free column below its row (sorted, simple, equal triangle
    sizes): only the exact comparison of the transposed lower triangle can reject it."""
    g, rows, picks = _rmat_cases()
    rp, col = g.row_ptr, g.col.copy()
    done = False
    for k in (int(picks["mid"]), int(picks["tile_first"]), int(picks["tile_last"])):
        u = int(rows[k])
        lo = col[k - 1] + 1 if k > rp[u] else 0
        hi = min(col[k + 1] if k + 1 < rp[u + 1] else u, u)
        free = [c for c in range(lo, hi) if c != col[k]]
        if free:
            col[k] = free[len(free) // 2]
            done = True
            break
    assert done
    o = oracle.recover(n=g.n, row_ptr=rp, col=col, w=g.w, parent=g.parent, alpha=g.alpha, beta=g.beta).status
    assert o == -3
    assert gpu_status(gpu_ctx, g, col=col) == -3
