// gss_treegen.hip -- feGRASS's spanning tree on the GPU, the step before the recovery
// (Sec. II-B "feGRASS Algorithm"; Def. "Effective weight", eq. weff):
//   1. root = the vertex of largest degree (smallest id among ties),
//   2. unweighted distances from the root by a level-synchronous breadth-first search,
//   3. per edge W_eff = (w * log(max(deg u, deg v))) / (dist u + dist v), each operation
//      rounded once (the logarithms come from a host table, one per degree value),
//   4. the maximum spanning tree under the total order (W_eff descending, edge id
//      ascending) by Boruvka's algorithm: every component takes its best outgoing edge
//      (a cut edge of the unique tree), mutual choices hook the larger label onto the
//      smaller, and pointer jumping relabels the vertices,
//   5. the tree rooted at the root: an Euler tour of its half-edges, ranked by pointer
//      jumping; a vertex's parent is the neighbour whose half-edge into it comes first.
// With GSS_TREE_WEIGHT the order is by the edge weight itself (a plain maximum-weight
// spanning tree) instead of W_eff.
#include <cmath>

#include "gss_impl.h"

namespace {

constexpr int TG_BLOCK = 256;
constexpr int TG_GRID = 2048;  // grid of the grid-stride kernels
constexpr int32_t TG_INF = 0x7f7f7f7f;

__global__ void tg_iota(int32_t *__restrict__ p, int32_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

// largest (degree, -id): the root; also rejects columns out of range and self loops
__global__ void tg_root(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t n,
                        unsigned long long *__restrict__ best, uint32_t *flags)
{
    unsigned long long key = 0;
    uint32_t f = 0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int32_t a = rp[x], b = rp[x + 1];
        if (b < a) f |= F_ARG;
        const unsigned long long k = ((unsigned long long)(uint32_t)(b - a) << 32) | (uint32_t)(0x7fffffff - x);
        key = k > key ? k : key;
        for (int32_t j = a; j < b; j++) {
            const int32_t y = col[j];
            if (y < 0 || y >= n || y == x) f |= F_ARG;
        }
    }
    for (int d = GSS_WAVE / 2; d > 0; d >>= 1) {
        const unsigned long long o = __shfl_xor(key, d, GSS_WAVE);
        key = o > key ? o : key;
        f |= __shfl_xor(f, d, GSS_WAVE);
    }
    if (lane_id() == 0) {
        atomicMax(best, key);
        if (f) atomicOr(flags, f);
    }
}

// one breadth-first level: the frontier of level L (count cnt[L]) expands into level L+1
__global__ void tg_bfs_level(int32_t L, const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                             const int32_t *__restrict__ fin, int32_t *__restrict__ fout, int32_t *__restrict__ cnt,
                             int32_t *__restrict__ dist)
{
    const int32_t nin = cnt[L];
    if (nin == 0) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nin; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t x = fin[i];
        for (int32_t j = rp[x]; j < rp[x + 1]; j++) {
            const int32_t y = col[j];
            if (dist[y] == -1 && atomicCAS(&dist[y], -1, L + 1) == -1) fout[atomicAdd(&cnt[L + 1], 1)] = y;
        }
    }
}

// upper entries (u < v) of each row: the first one's CSR index and their count
__global__ void tg_upper(const int32_t *__restrict__ rp, const int32_t *__restrict__ col, int32_t n,
                         int32_t *__restrict__ ufirst, int32_t *__restrict__ nup)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    int32_t lo = rp[x], hi = rp[x + 1];
    const int32_t end = hi;
    while (lo < hi) {  // rows are strictly increasing: the upper entries are a suffix
        const int32_t mid = (lo + hi) >> 1;
        if (col[mid] > (int32_t)x) hi = mid;
        else lo = mid + 1;
    }
    ufirst[x] = lo;
    nup[x] = end - lo;
}

// per edge id: endpoints and the ordering weight (W_eff, or w itself)
__global__ void tg_weights(const int32_t *__restrict__ rp, const int32_t *__restrict__ col,
                           const double *__restrict__ w, int32_t n, const int32_t *__restrict__ ufirst,
                           const int32_t *__restrict__ uptr, const int32_t *__restrict__ dist,
                           const double *__restrict__ logdeg, int plain, int32_t *__restrict__ eu,
                           int32_t *__restrict__ ev, double *__restrict__ we)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int32_t dx = rp[x + 1] - rp[x];
    int32_t id = uptr[x];
    for (int32_t j = ufirst[x]; j < rp[x + 1]; j++, id++) {
        const int32_t y = col[j];
        eu[id] = (int32_t)x;
        ev[id] = y;
        if (plain) {
            we[id] = w[j];
        } else {
            const int32_t dy = rp[y + 1] - rp[y];
            const double num = w[j] * logdeg[dx > dy ? dx : dy];  // rounded once (no contraction)
            we[id] = num / (double)(dist[x] + dist[y]);
        }
    }
}

// Boruvka, pass 1: the largest ordering weight leaving each component
__global__ void tg_best_weight(int64_t m, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                               const double *__restrict__ we, const int32_t *__restrict__ comp,
                               unsigned long long *__restrict__ bw)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t cu = comp[eu[e]], cv = comp[ev[e]];
        if (cu == cv) continue;
        const unsigned long long b = (unsigned long long)__double_as_longlong(we[e]);  // w >= 0: bits order
        atomicMax(&bw[cu], b);
        atomicMax(&bw[cv], b);
    }
}

// pass 2: among those, the smallest edge id
__global__ void tg_best_edge(int64_t m, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                             const double *__restrict__ we, const int32_t *__restrict__ comp,
                             const unsigned long long *__restrict__ bw, int32_t *__restrict__ be)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t cu = comp[eu[e]], cv = comp[ev[e]];
        if (cu == cv) continue;
        const unsigned long long b = (unsigned long long)__double_as_longlong(we[e]);
        if (b == bw[cu]) atomicMin(&be[cu], (int32_t)e);
        if (b == bw[cv]) atomicMin(&be[cv], (int32_t)e);
    }
}

// pass 3: every component label takes its edge into the tree and hooks onto the other
// side's label; of two labels that chose the same edge, the smaller stays a root
__global__ void tg_hook(int32_t n, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                        const int32_t *__restrict__ comp, const int32_t *__restrict__ be,
                        int32_t *__restrict__ nxt, uint8_t *__restrict__ intree, int32_t *__restrict__ hooks)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    if (comp[c] != (int32_t)c || be[c] == TG_INF) {
        nxt[c] = comp[c];
        return;
    }
    const int32_t e = be[c];
    intree[e] = 1;
    const int32_t a = comp[eu[e]], b = comp[ev[e]];
    const int32_t other = (a == (int32_t)c) ? b : a;
    if (be[other] == e && (int32_t)c < other) {
        nxt[c] = (int32_t)c;
    } else {
        nxt[c] = other;
        atomicAdd(hooks, 1);
    }
}

// pointer jumping: comp = nxt[nxt] until every label is a root; counts the changes
__global__ void tg_jump(int32_t n, const int32_t *__restrict__ src, int32_t *__restrict__ dst,
                        int32_t *__restrict__ changed)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int32_t p = src[x], q = src[p];
    dst[x] = q;
    if (q != p) atomicOr(changed, 1);
}

// tree adjacency: every tree edge fills its two half-edges (slot order within a row is
// arbitrary: the rooted tree does not depend on it)
__global__ void tg_tree_degree(int64_t m, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                               const uint8_t *__restrict__ intree, int32_t *__restrict__ tdeg)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        if (intree[e]) {
            atomicAdd(&tdeg[eu[e]], 1);
            atomicAdd(&tdeg[ev[e]], 1);
        }
}

__global__ void tg_tree_fill(int64_t m, const int32_t *__restrict__ eu, const int32_t *__restrict__ ev,
                             const uint8_t *__restrict__ intree, const int32_t *__restrict__ tptr,
                             int32_t *__restrict__ cur, int32_t *__restrict__ tail, int32_t *__restrict__ head,
                             int32_t *__restrict__ twin)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        if (!intree[e]) continue;
        const int32_t u = eu[e], v = ev[e];
        const int32_t su = tptr[u] + atomicAdd(&cur[u], 1), sv = tptr[v] + atomicAdd(&cur[v], 1);
        tail[su] = u;
        head[su] = v;
        tail[sv] = v;
        head[sv] = u;
        twin[su] = sv;
        twin[sv] = su;
    }
}

// Euler tour: after u -> v comes the half-edge following v -> u in v's row (cyclically);
// the tour starts at the root's first half-edge, so the one leading back to it ends it
__global__ void tg_succ(int64_t H, const int32_t *__restrict__ head, const int32_t *__restrict__ twin,
                        const int32_t *__restrict__ tptr, int32_t h0, int32_t *__restrict__ nx,
                        int32_t *__restrict__ rank)
{
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    const int32_t v = head[h], t = twin[h];
    int32_t s = (t + 1 < tptr[v + 1]) ? t + 1 : tptr[v];
    if (s == h0) s = -1;
    nx[h] = s;
    rank[h] = 1;
}

// pointer jumping over the tour: rank = half-edges from h to the end, inclusive
__global__ void tg_rank_step(int64_t H, const int32_t *__restrict__ nx, const int32_t *__restrict__ rank,
                             int32_t *__restrict__ nx2, int32_t *__restrict__ rank2)
{
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    const int32_t s = nx[h];
    if (s < 0) {
        nx2[h] = -1;
        rank2[h] = rank[h];
    } else {
        nx2[h] = nx[s];
        rank2[h] = rank[h] + rank[s];
    }
}

// the half-edge of a tree edge that the tour takes first points from parent to child
__global__ void tg_parent(int64_t H, const int32_t *__restrict__ tail, const int32_t *__restrict__ head,
                          const int32_t *__restrict__ twin, const int32_t *__restrict__ rank,
                          int32_t *__restrict__ parent)
{
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    if (rank[h] > rank[twin[h]]) parent[head[h]] = tail[h];
}

}  // namespace

// see gss_spanning_tree in gss.h
void spanning_tree_impl(gss_ctx ctx, const gss_csr *g, int32_t *parent, int32_t *root_out, double *weff_out,
                        uint32_t flags)
{
    hipStream_t st = ctx->stream;
    const int32_t n = g->n;
    const int64_t nnz = g->nnz;
    const bool plain = (flags & GSS_TREE_WEIGHT) != 0;
    const dim3 b(TG_BLOCK), gn(grid_for(n, TG_BLOCK));
    const dim3 gs((unsigned)std::min<int64_t>(TG_GRID, std::max<int64_t>(1, (nnz / 2 + TG_BLOCK - 1) / TG_BLOCK)));
    // 1. root (and the column checks)
    fill_bytes(ctx, ctx->d_flags, 0, sizeof(uint32_t));
    unsigned long long *best = (unsigned long long *)(ctx->d_counters + 16);
    fill_bytes(ctx, best, 0, sizeof(unsigned long long));
    GSS_LAUNCH(tg_root, dim3(std::min<unsigned>(gn.x, TG_GRID)), b, 0, st, g->row_ptr, g->col, n, best,
               ctx->d_flags);
    ctx->readback(ctx->h_counters + 16, best, sizeof(unsigned long long));
    const uint32_t f = read_flags(ctx);
    if (f & F_ARG) throw gss_error{GSS_ERR_ARG, "spanning tree: a row is not ordered, or a column is out of range"};
    const int32_t root = 0x7fffffff - (int32_t)((uint64_t)ctx->h_counters[16] & 0xffffffffu);
    const int32_t maxdeg = (int32_t)((uint64_t)ctx->h_counters[16] >> 32);
    *root_out = root;
    if (n == 1) {
        const int32_t m1 = -1;
        ctx->h2d(parent, &m1, sizeof m1);
        ctx->sync();
        return;
    }
    // 2. breadth-first distances from the root
    int32_t *dist = ctx->alloc<int32_t>(n);
    int32_t *fa = ctx->alloc<int32_t>(n), *fb = ctx->alloc<int32_t>(n);
    int32_t *cnt = ctx->alloc<int32_t>((int64_t)n + 2);
    fill_bytes(ctx, dist, 0xff, sizeof(int32_t) * n);
    fill_bytes(ctx, cnt, 0, sizeof(int32_t) * ((size_t)n + 2));
    {
        const int32_t zero = 0, one = 1;
        ctx->h2d(dist + root, &zero, sizeof zero);
        ctx->h2d(fa, &root, sizeof root);
        ctx->h2d(cnt, &one, sizeof one);
    }
    int32_t level = 0, visited = 1;
    for (int32_t batch = 8;; batch = std::min(2 * batch, 256)) {
        for (int32_t i = 0; i < batch && level < n; i++, level++)
            GSS_LAUNCH(tg_bfs_level, gs, b, 0, st, level, g->row_ptr, g->col, (level & 1) ? fb : fa,
                       (level & 1) ? fa : fb, cnt, dist);
        int32_t last = 0;
        ctx->readback(&last, cnt + level, sizeof last);
        if (last == 0 || level >= n) break;
    }
    {
        std::vector<int32_t> hc((size_t)level + 1);
        ctx->readback(hc.data(), cnt, sizeof(int32_t) * hc.size());
        int64_t tot = 0;
        for (int32_t c : hc) tot += c;
        visited = (int32_t)tot;
    }
    if (visited != n) throw gss_error{GSS_ERR_ARG, "spanning tree: the graph is not connected"};
    // 3. edges in id order and their ordering weights
    int32_t *ufirst = ctx->alloc<int32_t>(n), *uptr = ctx->alloc<int32_t>((int64_t)n + 1);
    GSS_LAUNCH(tg_upper, gn, b, 0, st, g->row_ptr, g->col, n, ufirst, uptr);
    const int64_t m = scan_exclusive_i32(ctx, uptr, n, true);
    if (2 * m != nnz) throw gss_error{GSS_ERR_ASYM, "spanning tree: the CSR is not symmetric"};
    std::vector<double> lg((size_t)maxdeg + 1, 0.0);
    for (int32_t k = 1; k <= maxdeg; k++) lg[k] = std::log((double)k);
    double *logdeg = ctx->alloc<double>(lg.size());
    ctx->h2d(logdeg, lg.data(), sizeof(double) * lg.size());
    int32_t *eu = ctx->alloc<int32_t>(m + 1), *ev = ctx->alloc<int32_t>(m + 1);
    double *we = weff_out ? weff_out : ctx->alloc<double>(m + 1);
    GSS_LAUNCH(tg_weights, gn, b, 0, st, g->row_ptr, g->col, g->w, n, ufirst, uptr, dist, logdeg, plain ? 1 : 0,
               eu, ev, we);
    ctx->free(fa);
    ctx->free(fb);
    ctx->free(cnt);
    ctx->free(ufirst);
    ctx->free(uptr);
    ctx->free(logdeg);
    // 4. Boruvka
    int32_t *comp = ctx->alloc<int32_t>(n), *nxt = ctx->alloc<int32_t>(n);
    unsigned long long *bw = ctx->alloc<unsigned long long>(n);
    int32_t *be = ctx->alloc<int32_t>(n);
    uint8_t *intree = ctx->alloc<uint8_t>(m + 1);
    int32_t *ctr = ctx->alloc<int32_t>(2);  // hooks, changed
    fill_bytes(ctx, intree, 0, (size_t)m + 1);
    GSS_LAUNCH(tg_iota, gn, b, 0, st, comp, n);
    const dim3 ge((unsigned)std::min<int64_t>(TG_GRID, std::max<int64_t>(1, (m + TG_BLOCK - 1) / TG_BLOCK)));
    for (int round = 0;; round++) {
        if (round > 64) throw gss_error{GSS_ERR_HIP, "spanning tree: Boruvka did not converge"};
        fill_bytes(ctx, bw, 0, sizeof(unsigned long long) * n);
        fill_bytes(ctx, be, 0x7f, sizeof(int32_t) * n);
        fill_bytes(ctx, ctr, 0, 2 * sizeof(int32_t));
        GSS_LAUNCH(tg_best_weight, ge, b, 0, st, m, eu, ev, we, comp, bw);
        GSS_LAUNCH(tg_best_edge, ge, b, 0, st, m, eu, ev, we, comp, bw, be);
        GSS_LAUNCH(tg_hook, gn, b, 0, st, n, eu, ev, comp, be, nxt, intree, ctr);
        int32_t hooks = 0;
        ctx->readback(&hooks, ctr, sizeof hooks);
        if (hooks == 0) break;
        // relabel: jump until every label is a root (at most log2 n + 1 doublings)
        for (int j = 0;; j++) {
            if (j > 40) throw gss_error{GSS_ERR_HIP, "spanning tree: pointer jumping did not converge"};
            fill_bytes(ctx, ctr + 1, 0, sizeof(int32_t));
            GSS_LAUNCH(tg_jump, gn, b, 0, st, n, nxt, comp, ctr + 1);
            GSS_LAUNCH(tg_jump, gn, b, 0, st, n, comp, nxt, ctr + 1);
            int32_t changed = 0;
            ctx->readback(&changed, ctr + 1, sizeof changed);
            if (!changed) break;
        }
        HIP_OK(hipMemcpyAsync(comp, nxt, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    }
    ctx->free(bw);
    ctx->free(be);
    ctx->free(nxt);
    ctx->free(comp);
    if (!weff_out) ctx->free(we);
    // 5. root the tree: Euler tour of the half-edges, ranked by pointer jumping
    const int64_t H = 2 * (int64_t)(n - 1);
    int32_t *tptr = ctx->alloc<int32_t>((int64_t)n + 1), *cur = ctx->alloc<int32_t>(n);
    fill_bytes(ctx, tptr, 0, sizeof(int32_t) * ((size_t)n + 1));
    fill_bytes(ctx, cur, 0, sizeof(int32_t) * n);
    GSS_LAUNCH(tg_tree_degree, ge, b, 0, st, m, eu, ev, intree, tptr);
    const int64_t halves = scan_exclusive_i32(ctx, tptr, (int64_t)n + 1, true);
    if (halves != H) throw gss_error{GSS_ERR_HIP, "spanning tree: wrong number of tree edges"};
    int32_t *tail = ctx->alloc<int32_t>(H), *head = ctx->alloc<int32_t>(H), *twin = ctx->alloc<int32_t>(H);
    int32_t *nx = ctx->alloc<int32_t>(H), *nx2 = ctx->alloc<int32_t>(H);
    int32_t *rank = ctx->alloc<int32_t>(H), *rank2 = ctx->alloc<int32_t>(H);
    GSS_LAUNCH(tg_tree_fill, ge, b, 0, st, m, eu, ev, intree, tptr, cur, tail, head, twin);
    int32_t h0 = 0;
    ctx->readback(&h0, tptr + root, sizeof h0);
    const dim3 gh(grid_for(H, TG_BLOCK));
    GSS_LAUNCH(tg_succ, gh, b, 0, st, H, head, twin, tptr, h0, nx, rank);
    int steps = 0;
    while (((int64_t)1 << steps) < H) steps++;
    for (int s = 0; s <= steps; s++) {
        GSS_LAUNCH(tg_rank_step, gh, b, 0, st, H, nx, rank, nx2, rank2);
        std::swap(nx, nx2);
        std::swap(rank, rank2);
    }
    fill_bytes(ctx, parent, 0xff, sizeof(int32_t) * n);  // -1 at the root
    GSS_LAUNCH(tg_parent, gh, b, 0, st, H, tail, head, twin, rank, parent);
    HIP_OK(hipGetLastError());
    ctx->sync();
    for (void *p : {(void *)dist, (void *)eu, (void *)ev, (void *)intree, (void *)ctr, (void *)tptr, (void *)cur,
                    (void *)tail, (void *)head, (void *)twin, (void *)nx, (void *)nx2, (void *)rank, (void *)rank2})
        ctx->free(p);
}
