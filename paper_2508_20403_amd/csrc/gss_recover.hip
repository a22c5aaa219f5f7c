// gss_recover.hip -- off-tree edge recovery on gfx950.
//
// Paper: Alg. 1 (Steps 1-4), eq. RT, eq. beta-new, Def. "Similar edge (Strict)",
// Lemma "strictly similar edges share their LCA".
//
// Path of one pass:
//  1. k_edge_stretch  every off-tree edge: LCA by RMQ over the preorder sequence, exact
//                     R_T = RN(D(u)+D(v)-2D(lca)), stretch = RN(w*R_T), beta*, sort key;
//                     a 12-bit histogram of the key for the prefix selection.
//  2. radix select    the smallest key threshold T whose set {key >= T} holds at least
//                     P0 edges: that set is a prefix of the criticality order (stretch
//                     descending, id ascending).  Decisions about edges in a prefix never
//                     depend on edges after it, so only the prefix is resolved.
//  3. compaction + stable LSD radix sort of the prefix -> rank order.
//  4. strict-similarity discovery by an anchor hash join.  For tree distance,
//     dist(a,b) <= beta  <=>  anc_i(a) = anc_j(b) for some i+j <= beta.  Every prefix
//     edge (x,y) is inserted under the keys (anc_i(x), anc_k(y)) for i,k <= c (both
//     orientations); every edge (u,v) with beta* >= 1 probes (anc_j(u), anc_l(v)) for
//     j,l <= beta* and keeps entries with i <= beta*-j, k <= beta*-l.  Each hit with a
//     later rank is a dependency arc "marker -> target".
//  5. dependency rounds: an edge with no arcs in is recovered; an edge with an arc from a
//     recovered edge is marked; an edge whose in-arcs all come from marked edges is
//     recovered.  This reproduces the serial greedy exactly (arcs point forward in rank).
//  6. the first K recovered edges in rank order form the output.
// Arcs only join edges with the same LCA (the Lemma), so the join runs inside the
// paper's LCA subtasks without materialising them; grouping is reported as statistics.
#include <algorithm>
#include <cmath>
#include <functional>

#include "gss_impl.h"
#include "gss_lookback.h"
#include "gss_subtask.h"

#define RB 256
#define SEL_BITS 12
#define SEL_BINS (1 << SEL_BITS)

enum : uint8_t { ST_UNDEC = 0, ST_CAND = 1, ST_MARK = 2 };

struct RmqView {
    const uint64_t *epk, *pmask, *ppre, *psuf, *bmin, *bmask, *bpre, *bsuf, *sbst;
    int32_t nsb;
};

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int ctz64(uint64_t x) { return __ffsll((long long)x) - 1; }

// RMQ over preorder positions i..j (i <= j) with every load addressable from (i, j) issued
// up front; only the in-block argmin reads depend on an earlier load.
struct RmqPlan {
    int32_t i, j, bi, bj, b0, b1, s0, s1, a, c, k;
    bool same_block, has_blocks, same_super, has_super;
};

__device__ __forceinline__ RmqPlan rmq_plan(const RmqView &, int32_t i, int32_t j)
{
    RmqPlan P;
    P.i = i;
    P.j = j;
    P.bi = i >> 6;
    P.bj = j >> 6;
    P.same_block = P.bi == P.bj;
    P.b0 = P.bi + 1;
    P.b1 = P.bj - 1;
    P.has_blocks = !P.same_block && P.b0 <= P.b1;
    P.s0 = P.b0 >> 6;
    P.s1 = P.b1 >> 6;
    P.same_super = P.has_blocks && P.s0 == P.s1;
    P.a = P.s0 + 1;
    P.c = P.s1 - 1;
    P.has_super = P.has_blocks && !P.same_super && P.a <= P.c;
    P.k = P.has_super ? 31 - __clz(P.c - P.a + 1) : 0;
    if (!P.has_blocks) {  // keep every index valid; the loads are then ignored
        P.b0 = P.b1 = 0;
        P.s0 = P.s1 = 0;
    }
    if (!P.has_super) P.a = P.c = 0;
    return P;
}

struct RmqLoads {
    uint64_t psuf, ppre, pmask, bsuf, bpre, bmask, st0, st1;
};

// Only the loads the query's case needs are issued: the position-level arrays are far
// larger than the caches, so a wasted load there costs a random HBM access.
__device__ __forceinline__ RmqLoads rmq_issue(const RmqView &q, const RmqPlan &P)
{
    RmqLoads L = {~0ull, ~0ull, 0ull, ~0ull, ~0ull, 0ull, ~0ull, ~0ull};
    if (P.same_block) {
        L.pmask = q.pmask[P.j];
    } else {
        L.psuf = q.psuf[P.i];
        L.ppre = q.ppre[P.j];
    }
    if (P.has_blocks) {
        L.bmask = q.bmask[P.b1];
        L.bsuf = q.bsuf[P.b0];
        L.bpre = q.bpre[P.b1];
    }
    if (P.has_super) {
        const uint64_t *lv = q.sbst + (int64_t)P.k * q.nsb;
        L.st0 = lv[P.a];
        L.st1 = lv[P.c - (1 << P.k) + 1];
    }
    return L;
}

__device__ __forceinline__ uint64_t rmq_finish(const RmqView &q, const RmqPlan &P, const RmqLoads &L)
{
    if (P.same_block) {
        uint64_t m = L.pmask & (~0ull << (P.i & 63));
        return q.epk[(P.bi << 6) + ctz64(m)];
    }
    uint64_t best = umin64(L.psuf, L.ppre);
    if (P.same_super) {
        uint64_t m = L.bmask & (~0ull << (P.b0 & 63));
        best = umin64(best, q.bmin[(P.s0 << 6) + ctz64(m)]);
    } else if (P.has_blocks) {
        best = umin64(best, umin64(L.bsuf, L.bpre));
        if (P.has_super) best = umin64(best, umin64(L.st0, L.st1));
    }
    return best;
}

// minimum packed (depth<<32|parent) over preorder positions i..j (i <= j)
__device__ __forceinline__ uint64_t rmq(const RmqView &q, int32_t i, int32_t j)
{
    RmqPlan P = rmq_plan(q, i, j);
    RmqLoads L = rmq_issue(q, P);
    return rmq_finish(q, P, L);
}

// ------------------------------------------------------------------------------------
// 1. per-edge LCA / resistance / stretch / beta*
// ------------------------------------------------------------------------------------
#define EDGE_ITEMS 2
#define EDGE_GRID 2048  // workgroups of the grid-stride per-edge kernel
#define STRETCH_HIST 1  // single graphs: the per-edge kernel also builds the first key histogram
template <bool HIST>
__global__ __launch_bounds__(RB) void k_edge_stretch(
    int64_t M, const int32_t *__restrict__ off_id, const int32_t *__restrict__ off_u,
    const int32_t *__restrict__ off_v, const double *__restrict__ off_w,
    const VRec *__restrict__ vrec, RmqView q, int32_t scale, int32_t c, uint64_t *__restrict__ key,
    int32_t *__restrict__ lca, uint8_t *__restrict__ bst, double *__restrict__ stretch_out,
    uint32_t *__restrict__ hist, int32_t *__restrict__ lcacnt, uint32_t *flags, int key_rt)
{
    // the first-level key histogram (HIST only: the LDS array limits occupancy)
    __shared__ uint32_t sh[HIST ? SEL_BINS : 1];
    if (HIST) {
        for (int i = threadIdx.x; i < SEL_BINS; i += RB) sh[i] = 0;
        __syncthreads();
    }
    // grid-stride over tiles of RB * EDGE_ITEMS edges, so the histogram is flushed once
    // per workgroup rather than once per tile
    const int64_t ntiles = (M + RB * EDGE_ITEMS - 1) / (RB * EDGE_ITEMS);
    for (int64_t t0 = blockIdx.x; t0 < ntiles; t0 += gridDim.x) {
        const int64_t tile = xcd_tile(t0, ntiles);  // contiguous edge ranges per XCD
        const int64_t base = tile * RB * EDGE_ITEMS + threadIdx.x;
        int64_t jj[EDGE_ITEMS];
        bool ok[EDGE_ITEMS];
        int32_t u[EDGE_ITEMS], v[EDGE_ITEMS];
        double w[EDGE_ITEMS];
#pragma unroll
        for (int t = 0; t < EDGE_ITEMS; t++) {
            jj[t] = base + (int64_t)t * RB;
            ok[t] = jj[t] < M;
            int64_t j = ok[t] ? jj[t] : 0;
            u[t] = off_u[j];
            v[t] = off_v[j];
            w[t] = off_w[j];
        }
        VRec ru[EDGE_ITEMS], rv[EDGE_ITEMS];
#pragma unroll
        for (int t = 0; t < EDGE_ITEMS; t++) {
            ru[t] = vrec[u[t]];
            rv[t] = vrec[v[t]];
        }
        RmqPlan pl[EDGE_ITEMS];
        RmqLoads ld[EDGE_ITEMS];
#pragma unroll
        for (int t = 0; t < EDGE_ITEMS; t++) {
            // preorder positions (min, max]: u != v, so the range is not empty
            const int32_t fu = ru[t].first, fv = rv[t].first;
            const int32_t hi = max(fu, fv);
            pl[t] = rmq_plan(q, min(min(fu, fv) + 1, hi), hi);
            ld[t] = rmq_issue(q, pl[t]);
        }
        uint64_t pk[EDGE_ITEMS];
#pragma unroll
        for (int t = 0; t < EDGE_ITEMS; t++) pk[t] = rmq_finish(q, pl[t], ld[t]);
        u128 Dl[EDGE_ITEMS];
#pragma unroll
        for (int t = 0; t < EDGE_ITEMS; t++) Dl[t] = vrec[(int32_t)(uint32_t)pk[t]].D;
        int32_t lw[EDGE_ITEMS];
#pragma unroll
        for (int t = 0; t < EDGE_ITEMS; t++) {
            lw[t] = -1;
            if (!ok[t]) continue;
            const int64_t j = jj[t];
            const int32_t l = (int32_t)(uint32_t)pk[t];
            const int32_t dl = (int32_t)(pk[t] >> 32) - 1;  // the minimum is a child of l
            const int32_t du = ru[t].depth - dl, dv = rv[t].depth - dl;
            u128 R = add128(sub128(ru[t].D, Dl[t]), sub128(rv[t].D, Dl[t]));
            double r;
            bool good = u128_to_double_rne(R, scale, &r);
            double s = w[t] * r;
            const uint64_t sbits = (uint64_t)__double_as_longlong(s);
            // the sort key: the stretch, or R_T itself (positive doubles order like their bits)
            uint64_t bits = key_rt ? (uint64_t)__double_as_longlong(r) : sbits;
            if (!good || ((sbits >> 52) & 0x7ff) == 0x7ff) {
                atomicOr(flags, F_RANGE);
                bits = 1;
            }
            int32_t b = du < dv ? du : dv;
            if (c < b) b = c;
            key[j] = bits;
            lca[j] = l;
            bst[j] = (uint8_t)b;
            if (stretch_out) stretch_out[off_id[j]] = s;
            if (HIST) atomicAdd(&sh[(uint32_t)(bits >> 51) & (SEL_BINS - 1)], 1u);
            lw[t] = l;
        }
        // subtask sizes (only when asked for): one atomic per distinct LCA of the wavefront
        if (lcacnt) {
#pragma unroll
            for (int t = 0; t < EDGE_ITEMS; t++) {
                const int32_t l = lw[t];
                uint64_t active = __ballot(l >= 0);
                while (active) {
                    const int leader = ctz64(active);
                    const int32_t lv = __shfl(l, leader, GSS_WAVE);
                    const uint64_t same = __ballot(l == lv) & active;
                    if (lane_id() == leader) atomicAdd(&lcacnt[lv], __popcll(same));
                    active &= ~same;
                }
            }
        }
    }
    if (HIST) {
        __syncthreads();
        for (int i = threadIdx.x; i < SEL_BINS; i += RB)
            if (sh[i]) atomicAdd(&hist[i], sh[i]);
    }
}

// number of subtasks (non-zero LCA counts) and the largest
__global__ __launch_bounds__(RB) void k_lca_stats(const int32_t *__restrict__ lcacnt, int32_t n,
                                                  int64_t *counters)
{
    __shared__ int32_t snz[RB / GSS_WAVE], smx[RB / GSS_WAVE];
    int32_t nz = 0, mx = 0;
    for (int64_t x = (int64_t)blockIdx.x * RB + threadIdx.x; x < n; x += (int64_t)gridDim.x * RB) {
        int32_t c = lcacnt[x];
        nz += c > 0;
        mx = max(mx, c);
    }
    for (int d = 32; d > 0; d >>= 1) {
        nz += __shfl_xor(nz, d, GSS_WAVE);
        mx = max(mx, __shfl_xor(mx, d, GSS_WAVE));
    }
    if (lane_id() == 0) {
        snz[threadIdx.x / GSS_WAVE] = nz;
        smx[threadIdx.x / GSS_WAVE] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < RB / GSS_WAVE; i++) {
            nz += snz[i];
            mx = max(mx, smx[i]);
        }
        atomicAdd((unsigned long long *)&counters[0], (unsigned long long)nz);
        atomicMax((long long *)&counters[1], (long long)mx);
    }
}

// ------------------------------------------------------------------------------------
// 2. radix select of each graph's prefix threshold
// ------------------------------------------------------------------------------------
// histogram of key digit [shift, shift+width) over eligible keys of refining graphs whose
// higher digits match that graph's selected prefix; hist is [G][SEL_BINS]
__global__ __launch_bounds__(RB) void k_key_hist(const uint64_t *__restrict__ key, int64_t M,
                                                 const int32_t *__restrict__ off_g, int shift, int width,
                                                 const uint64_t *__restrict__ pmask, const uint64_t *__restrict__ pval,
                                                 const int64_t *__restrict__ need, uint32_t *__restrict__ hist,
                                                 const int32_t *__restrict__ active)
{
    __shared__ uint32_t sh[SEL_BINS];
    __shared__ int32_t gblk;
    if (*active == 0) return;  // no graph refines at this level
    for (int i = threadIdx.x; i < SEL_BINS; i += RB) sh[i] = 0;
    const int64_t per = ((M + gridDim.x - 1) / gridDim.x + RB - 1) / RB * RB;  // contiguous range per block
    const int64_t j0 = (int64_t)blockIdx.x * per, j1 = min(M, j0 + per);
    if (threadIdx.x == 0) gblk = (off_g && j0 < M) ? off_g[j0] : 0;
    __syncthreads();
    const uint32_t dmask = (1u << width) - 1;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += RB) {
        uint64_t k = key[j];
        int32_t g = off_g ? off_g[j] : 0;
        if (k == 0 || need[g] <= 0 || (k & pmask[g]) != pval[g]) continue;
        uint32_t d = (uint32_t)(k >> shift) & dmask;
        if (g == gblk) atomicAdd(&sh[d], 1u);
        else atomicAdd(&hist[(int64_t)g * SEL_BINS + d], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SEL_BINS; i += RB)
        if (sh[i]) atomicAdd(&hist[(int64_t)gblk * SEL_BINS + i], sh[i]);
}

// Device state of the threshold selection, one entry per graph (arrays of G):
//   need      keys wanted (<= 0: the graph is not refining any more)
//   above     keys above the bucket the fixed high digits select
//   pmask/pval the fixed high digits
//   thr, plen the threshold so far and the number of keys at or above it
//   eligible  the graph's eligible keys
// active[lv] counts the graphs refining at level lv.
struct SelState {
    int64_t *need, *above, *plen, *eligible;
    uint64_t *pmask, *pval, *thr;
    int32_t *active;
};

// Per graph (block): the digit at this level that holds the target-th largest key of the
// selected bucket (target = need - above), and the state update the level implies.  The
// graph's histogram row is cleared for the next level.  The graph stops refining once its
// bucket overshoots need by at most max(1024, need / 16) keys, or at the last level.
__global__ __launch_bounds__(1024) void k_pick_update(uint32_t *__restrict__ hist, int lv, int shift, int width,
                                                      int last, SelState S)
{
    __shared__ int64_t lds[1024 / GSS_WAVE + 1];
    __shared__ int64_t s_found[3];
    const int g = blockIdx.x;
    if (S.active[lv] == 0) return;
    const int64_t need = S.need[g];
    if (need <= 0) return;
    const int64_t target = need - S.above[g];
    uint32_t *h = hist + (int64_t)g * SEL_BINS;
    const int nb = 1 << width;
    const int per = (nb + 1023) / 1024;
    if (threadIdx.x == 0) s_found[0] = -1;
    int64_t sum = 0;
    for (int i = 0; i < per; i++) {
        const int r = threadIdx.x * per + i;
        if (r < nb) sum += h[nb - 1 - r];
    }
    int64_t tot;
    const int64_t before = block_exclusive_scan<int64_t>(sum, lds, &tot);  // synchronises
    if (before < target && before + sum >= target) {
        int64_t acc = before;
        for (int i = 0; i < per; i++) {
            const int r = threadIdx.x * per + i;
            if (r >= nb) break;
            const int64_t c = h[nb - 1 - r];
            if (acc + c >= target) {
                s_found[0] = nb - 1 - r;
                s_found[1] = acc;
                s_found[2] = c;
                break;
            }
            acc += c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
    if (threadIdx.x != 0) return;
    const int64_t d = s_found[0];
    if (d < 0) {  // fewer keys than wanted: take every eligible key
        S.thr[g] = 1;
        S.plen[g] = S.eligible[g];
        S.need[g] = 0;
        return;
    }
    const uint64_t dmask = ((uint64_t)1 << width) - 1;
    S.pmask[g] |= dmask << shift;
    const uint64_t pval = S.pval[g] | ((uint64_t)d << shift);
    S.pval[g] = pval;
    const int64_t above = S.above[g] + s_found[1];
    S.above[g] = above;
    const int64_t slack = max((int64_t)1024, need / 16);
    // the bucket's lowest key, never 0 (a zero key is an edge already recovered)
    S.thr[g] = pval > 1 ? pval : 1;
    S.plen[g] = above + s_found[2];
    if (above + s_found[2] - need <= slack || last) S.need[g] = 0;
    else atomicAdd(&S.active[lv + 1], 1);
}

// ------------------------------------------------------------------------------------
// 3. compaction of {key >= T[graph]} (id order, hence graph-major) and the radix sort
// ------------------------------------------------------------------------------------
// Prefix compaction {key >= thr[graph]}, in id order.  A tile of PX_TILE keys is read
// round-major (key base + i*256 + t), so every load is coalesced; the counting pass
// stores one count per tile, the writing pass keeps (round, wave, lane) = id order.
#define PX_ITEMS 16
#define PX_TILE (256 * PX_ITEMS)
__global__ __launch_bounds__(256) void k_prefix_count(const uint64_t *__restrict__ key, int64_t M,
                                                      const int32_t *__restrict__ off_g,
                                                      const uint64_t *__restrict__ thr, int32_t *__restrict__ cnt)
{
    __shared__ int32_t s_c[256 / GSS_WAVE];
    const int64_t base = (int64_t)blockIdx.x * PX_TILE;
    uint64_t kv[PX_ITEMS];
    int32_t gv[PX_ITEMS];
#pragma unroll
    for (int i = 0; i < PX_ITEMS; i++) {
        const int64_t j = base + (int64_t)i * 256 + threadIdx.x;
        kv[i] = j < M ? key[j] : 0;
        gv[i] = (off_g && j < M) ? off_g[j] : 0;
    }
    int32_t c = 0;
#pragma unroll
    for (int i = 0; i < PX_ITEMS; i++) {
        const int64_t j = base + (int64_t)i * 256 + threadIdx.x;
        if (j < M && kv[i] >= thr[gv[i]]) c++;
    }
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, GSS_WAVE);
    if (lane_id() == 0) s_c[threadIdx.x / GSS_WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / GSS_WAVE; w++) c += s_c[w];
        cnt[blockIdx.x] = c;
    }
}

// Batches: before[g] = prefix edges with an off-tree index below obase[g] (graphs are
// contiguous in that index), from the scanned tile counts plus a count inside the tile
// holding the boundary.  One workgroup per boundary; no shared counters.
__global__ __launch_bounds__(256) void k_prefix_before(const uint64_t *__restrict__ key, int64_t M,
                                                       const int32_t *__restrict__ off_g,
                                                       const uint64_t *__restrict__ thr,
                                                       const int64_t *__restrict__ obase,
                                                       const int32_t *__restrict__ tile_off, int64_t P,
                                                       int64_t *__restrict__ before)
{
    __shared__ int32_t s_c[256 / GSS_WAVE];
    const int64_t b = obase[blockIdx.x];
    if (b >= M) {
        if (threadIdx.x == 0) before[blockIdx.x] = P;
        return;
    }
    const int64_t tile = b / PX_TILE, t0 = tile * PX_TILE;
    int32_t c = 0;
    for (int64_t j = t0 + threadIdx.x; j < b; j += 256) c += key[j] >= thr[off_g ? off_g[j] : 0] ? 1 : 0;
    for (int d = 32; d > 0; d >>= 1) c += __shfl_xor(c, d, GSS_WAVE);
    if (lane_id() == 0) s_c[threadIdx.x / GSS_WAVE] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / GSS_WAVE; w++) c += s_c[w];
        before[blockIdx.x] = (int64_t)tile_off[tile] + c;
    }
}
__global__ __launch_bounds__(256) void k_prefix_write(const uint64_t *__restrict__ key, int64_t M,
                                                      const int32_t *__restrict__ off_g,
                                                      const uint64_t *__restrict__ thr, const int32_t *__restrict__ off,
                                                      int64_t cap, int32_t *__restrict__ pj, uint64_t *__restrict__ pk)
{
    constexpr int NW = 256 / GSS_WAVE;
    __shared__ int32_t s_w[PX_ITEMS][NW];
    const int lane = lane_id(), wid = threadIdx.x / GSS_WAVE;
    const int64_t base = (int64_t)blockIdx.x * PX_TILE;
    uint64_t kv[PX_ITEMS];
    uint64_t keepm[PX_ITEMS];
#pragma unroll
    for (int i = 0; i < PX_ITEMS; i++) {
        const int64_t j = base + (int64_t)i * 256 + threadIdx.x;
        kv[i] = j < M ? key[j] : 0;
    }
#pragma unroll
    for (int i = 0; i < PX_ITEMS; i++) {
        const int64_t j = base + (int64_t)i * 256 + threadIdx.x;
        keepm[i] = __ballot(j < M && kv[i] >= thr[off_g ? off_g[j] : 0]);
        if (lane == 0) s_w[i][wid] = __popcll(keepm[i]);
    }
    __syncthreads();
    int64_t q = off[blockIdx.x];
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < PX_ITEMS; i++) {
        int64_t o = q;
        for (int w = 0; w < NW; w++) {
            if (w < wid) o += s_w[i][w];
            q += s_w[i][w];
        }
        if ((keepm[i] >> lane) & 1ull) {
            o += __popcll(keepm[i] & lt);
            if (o < cap) {  // cap = the length the host sized the prefix for
                pj[o] = (int32_t)(base + (int64_t)i * 256 + threadIdx.x);
                pk[o] = ~kv[i];  // ascending order of ~key = descending stretch
            }
        }
    }
}

// slots [*total, cap) of a prefix sized from the selection, should the scan find fewer
// keys: a valid index and the largest sort key (the host compares the lengths at its
// next read-back and fails the call on a difference)
__global__ void k_prefix_pad(const int64_t *__restrict__ total, int64_t cap, int32_t *__restrict__ pj,
                             uint64_t *__restrict__ pk, int64_t *__restrict__ pstart)
{
    if (threadIdx.x == 0) {  // the one graph's rank range [0, cap)
        pstart[0] = 0;
        pstart[1] = cap;
    }
    for (int64_t i = *total + threadIdx.x; i < cap; i += blockDim.x) {
        pj[i] = 0;
        pk[i] = ~0ull;
    }
}

// graph id of each compacted edge, as a sort key
__global__ void k_graph_key(int64_t P, const int32_t *__restrict__ pj, const int32_t *__restrict__ off_g,
                            uint64_t *__restrict__ gk)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) gk[p] = (uint64_t)(uint32_t)off_g[pj[p]];
}

// ------------------------------------------------------------------------------------
// stable LSD radix sort of (64-bit key, int32 value) pairs, 8-bit digits: one histogram
// pass over the keys for all digit positions, then one scatter kernel per varying
// digit, whose tiles learn their per-digit output bases by decoupled look-back
// ------------------------------------------------------------------------------------
#define RS_BLOCK 256
#ifndef RS_ITEMS
#define RS_ITEMS 8
#endif
#define RS_TILE (RS_BLOCK * RS_ITEMS)

// the pairs to sort: the first n, or the first *dn of them when a device count is given
__device__ __forceinline__ int64_t rs_count(int64_t n, const int64_t *dn)
{
    if (!dn) return n;
    const int64_t d = *dn;
    return d < 0 ? 0 : (d < n ? d : n);
}

// global digit counts of all eight byte positions: ghist[pos * 256 + digit] (zeroed)
__global__ __launch_bounds__(RS_BLOCK) void k_rs_ghist(const uint64_t *__restrict__ k, int64_t n_,
                                                       const int64_t *__restrict__ dn, int npos,
                                                       int32_t *__restrict__ ghist)
{
    const int64_t n = rs_count(n_, dn);
    __shared__ int32_t sh[8][256];
#pragma unroll
    for (int p = 0; p < 8; p++) sh[p][threadIdx.x] = 0;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * RS_BLOCK + threadIdx.x; i < n; i += (int64_t)gridDim.x * RS_BLOCK) {
        const uint64_t kk = k[i];
#pragma unroll
        for (int p = 0; p < 8; p++)
            if (p < npos) atomicAdd(&sh[p][(uint32_t)(kk >> (8 * p)) & 255u], 1);
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 8; p++) {
        const int32_t c = p < npos ? sh[p][threadIdx.x] : 0;
        if (c) atomicAdd(&ghist[p * 256 + threadIdx.x], c);
    }
}

// One pass.  Wavefront w of a tile owns the RS_ITEMS * 64 consecutive keys starting at
// tile offset w * RS_ITEMS * 64 and ranks them round by round (64 consecutive keys per
// round) with wave-private digit counters, so the only workgroup barriers are around the
// per-digit totals; tile order = (wave, round, lane) = index order.  The tile's base for
// digit d is the global start of d plus the count of d in all earlier tiles (look-back
// over status[tile][256]).  A digit position on which every key agrees needs no
// scatter: the pass then copies its tile in place (so the ping-pong buffers stay in
// step) and neither publishes nor reads look-back status.
__global__ __launch_bounds__(RS_BLOCK) void k_rs_onesweep(const uint64_t *__restrict__ kin,
                                                          const int32_t *__restrict__ vin, int64_t n_,
                                                          const int64_t *__restrict__ dn, int shift,
                                                          int64_t ntiles, const int32_t *__restrict__ ghist,
                                                          uint64_t *__restrict__ status, uint32_t epoch,
                                                          unsigned long long *ticket, uint64_t *__restrict__ kout,
                                                          int32_t *__restrict__ vout)
{
    constexpr int NW = RS_BLOCK / GSS_WAVE;
    __shared__ int32_t s_cnt[NW][256];  // per wavefront: digit counts so far
    __shared__ int32_t s_base[NW][256];  // per wavefront: output base of each digit
    __shared__ int32_t s_scan[NW + 1];
    __shared__ int64_t s_tile;
    __shared__ int s_const;
    const int t = threadIdx.x, wid = t / GSS_WAVE, lane = lane_id();
    const int64_t n = rs_count(n_, dn);
    if (t == 0) {
        s_tile = lb_ticket(ticket, ntiles);
        s_const = 0;
    }
#pragma unroll
    for (int w = 0; w < NW; w++) s_cnt[w][t] = 0;
    const int32_t gh = ghist[t];
    int32_t gtot;
    const int32_t gstart = block_exclusive_scan<int32_t>(gh, s_scan, &gtot);  // synchronises
    if ((int64_t)gh == n) s_const = 1;  // one digit holds every key
    __syncthreads();
    const int64_t tile = s_tile;
    // tiles past a device count hold nothing; no tile before them waits on them
    if (tile > 0 && tile * RS_TILE >= n) return;
    const int64_t wbase = tile * RS_TILE + (int64_t)wid * (RS_ITEMS * GSS_WAVE);
    if (s_const) {
#pragma unroll
        for (int i = 0; i < RS_ITEMS; i++) {
            const int64_t idx = wbase + i * GSS_WAVE + lane;
            if (idx < n) {
                kout[idx] = kin[idx];
                vout[idx] = vin[idx];
            }
        }
        return;
    }
    uint64_t kk[RS_ITEMS];
    int32_t vv[RS_ITEMS], pos[RS_ITEMS];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const int64_t idx = wbase + i * GSS_WAVE + lane;
        const bool valid = idx < n;
        kk[i] = valid ? kin[idx] : 0;
        vv[i] = valid ? vin[idx] : 0;
    }
    int32_t *cnt = s_cnt[wid];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        const bool valid = wbase + i * GSS_WAVE + lane < n;
        const uint32_t d = (uint32_t)(kk[i] >> shift) & 255u;
        // lanes of this wavefront holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const int leader = peers ? __ffsll((long long)peers) - 1 : lane;
        int32_t old = 0;
        if (valid && lane == leader) {
            old = cnt[d];
            cnt[d] = old + __popcll(peers);
        }
        old = __shfl(old, leader, GSS_WAVE);
        pos[i] = old + __popcll(peers & lanemask_lt());
    }
    __syncthreads();
    // thread t resolves digit t: wave offsets inside the tile, then the tile's base
    int32_t tc = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        s_base[w][t] = tc;
        tc += s_cnt[w][t];
    }
    int64_t excl = 0;
    if (tile == 0) {
        lb_store(status + t, lb_word(LB_INC, epoch, (uint64_t)tc));
    } else {
        lb_store(status + tile * 256 + t, lb_word(LB_AGG, epoch, (uint64_t)tc));
        excl = lb_lookback_thread<16>(status, 256, t, tile, epoch);
        lb_store(status + tile * 256 + t, lb_word(LB_INC, epoch, (uint64_t)(excl + tc)));
    }
#pragma unroll
    for (int w = 0; w < NW; w++) s_base[w][t] += gstart + (int32_t)excl;
    __syncthreads();
    const int32_t *base = s_base[wid];
#pragma unroll
    for (int i = 0; i < RS_ITEMS; i++) {
        if (wbase + i * GSS_WAVE + lane < n) {
            const int32_t o = base[(uint32_t)(kk[i] >> shift) & 255u] + pos[i];
            kout[o] = kk[i];
            vout[o] = vv[i];
        }
    }
}

// ------------------------------------------------------------------------------------
// per-rank gather and the anchor hash join
// ------------------------------------------------------------------------------------

__global__ void k_rank_gather(int64_t P, const int32_t *__restrict__ sj, const int32_t *__restrict__ off_id,
                              const int32_t *__restrict__ off_u, const int32_t *__restrict__ off_v,
                              const uint8_t *__restrict__ bst, const int32_t *__restrict__ lca,
                              const VRec *__restrict__ vrec, const int32_t *__restrict__ parent, int32_t c,
                              int32_t *__restrict__ rid,
                              uint8_t *__restrict__ rb, int32_t *__restrict__ ru, int32_t *__restrict__ rv,
                              int32_t *__restrict__ rdu, int32_t *__restrict__ rdv, int32_t *__restrict__ rl,
                              uint64_t *__restrict__ lkey, int32_t *__restrict__ lval,
                              int32_t *__restrict__ ancU, int32_t *__restrict__ ancV)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    int32_t j = sj[p];
    rid[p] = off_id[j];
    rb[p] = bst[j];
    int32_t a = off_u[j], b = off_v[j];
    ru[p] = a;
    rv[p] = b;
    int32_t l = lca[j];
    rl[p] = l;
    lkey[p] = (uint64_t)(uint32_t)l;
    lval[p] = (int32_t)p;
    VRec ra = vrec[a], rbv = vrec[b];
    rdu[p] = ra.depth;
    rdv[p] = rbv.depth;
    ancU[p] = a;
    ancV[p] = b;
    // the ancestor chains walk the 4-byte parent array (vrec[x].parent == parent[x]), not
    // the 32-byte vertex records
    int32_t pa = ra.parent, pb = rbv.parent;
    for (int i = 1; i <= c; i++) {
        ancU[(int64_t)i * P + p] = pa;
        ancV[(int64_t)i * P + p] = pb;
        if (i == c) break;
        pa = (pa >= 0) ? parent[pa] : -1;
        pb = (pb >= 0) ? parent[pb] : -1;
    }
}

// ------------------------------------------------------------------------------------
// Anchor join, partitioned.  Marker p = (u,v) with beta* b marks a later edge t = (x,y)
// of its subtask when x is within b tree hops of u and y within b of v (or x of v and y
// of u).  Within b hops means a common ancestor anc_i(x) = anc_j(u) with i + j <= b, so
// every edge emits records keyed by an ancestor pair:
//   build  (t): (anc_i(x), anc_k(y)) and (anc_i(y), anc_k(x)) for i, k <= c,
//   probe  (p): (anc_j(u), anc_l(v)) for j, l <= b,
// and a probe record matches a build record of equal key with i <= b - j, k <= b - l
// and t later than p.  Records are scattered into 2^bits partitions by a hash of the
// key (per-block histograms, a scan, then a scatter with LDS cursors: no global
// atomics), and every partition is joined in LDS by one workgroup.
// ------------------------------------------------------------------------------------
#define JP_BITS_MIN 11                   // 2048 partitions ...
#define JP_BITS_MAX 14                   // ... up to 16384, about 1024 records each
#define JP_BLOCK 256
#define JP_CAP 2048                      // records of a partition held in LDS at once
#define JP_TAB (2 * JP_CAP)              // LDS hash slots
#define JP_PROBE (1u << 31)

struct JRec {
    unsigned long long ab;  // (A << 32) | B
    int32_t p;              // rank of the edge
    uint32_t meta;          // build: (i << 8) | k; probe: JP_PROBE | (j << 16) | (l << 8) | beta*
};

__device__ __forceinline__ uint64_t jp_hash(uint64_t ab) { return mix64(ab * 0x9E3779B97F4A7C15ull + 1); }
__device__ __forceinline__ uint32_t jp_part(uint64_t ab, int bits) { return (uint32_t)(jp_hash(ab) >> (64 - bits)); }

// Every listed edge is handled by one thread, which loads the edge's ancestor chains once
// and emits all its records: build records for both orientations and every i, k <= c,
// probe records for j, l <= beta* (none when beta* = 0: such an edge marks nothing).
// A record whose key holds a missing ancestor (above the root) is not emitted.  The
// count and scatter passes give each workgroup the same edges, so the per-workgroup
// partition counts of the first pass are exactly the records the second one writes.
template <int C, bool WRITE>
__device__ __forceinline__ void jp_emit_edge(int32_t p, int beta, const int32_t (&au)[C + 1],
                                             const int32_t (&av)[C + 1], int bits, int32_t *sh,
                                             JRec *__restrict__ recs)
{
    auto emit = [&](int32_t A, int32_t B, uint32_t meta) {
        if (A < 0 || B < 0) return;
        const unsigned long long ab = ((unsigned long long)(uint32_t)A << 32) | (uint32_t)B;
        const uint32_t part = jp_part(ab, bits);
        if (WRITE) {
            JRec r;
            r.ab = ab;
            r.p = p;
            r.meta = meta;
            recs[atomicAdd(&sh[part], 1)] = r;
        } else {
            atomicAdd(&sh[part], 1);
        }
    };
#pragma unroll
    for (int i = 0; i <= C; i++)
#pragma unroll
        for (int k = 0; k <= C; k++) {
            emit(au[i], av[k], ((uint32_t)i << 8) | (uint32_t)k);
            emit(av[i], au[k], ((uint32_t)i << 8) | (uint32_t)k);
        }
    if (beta > 0) {
#pragma unroll
        for (int j = 0; j <= C; j++)
#pragma unroll
            for (int l = 0; l <= C; l++)
                if (j <= beta && l <= beta)
                    emit(au[j], av[l], JP_PROBE | ((uint32_t)j << 16) | ((uint32_t)l << 8) | (uint32_t)beta);
    }
}

// pass 1 (WRITE = false): per-workgroup partition histogram, stored partition-major:
// hist[part * nblk + block].  Pass 2 (WRITE = true): the same records, written at their
// partition offsets off[part * nblk + block] (order inside a partition is immaterial).
// Workgroup b owns listed edges [b * JP_BLOCK * ept, (b + 1) * JP_BLOCK * ept).
template <int C, bool WRITE>
__global__ __launch_bounds__(JP_BLOCK) void k_jp_records(int64_t ng, const int32_t *__restrict__ glist, int64_t P,
                                                          const uint8_t *__restrict__ rb,
                                                          const int32_t *__restrict__ ancU,
                                                          const int32_t *__restrict__ ancV, int bits, int ept,
                                                          int32_t nblk, int32_t *__restrict__ hist,
                                                          JRec *__restrict__ recs)
{
    extern __shared__ int32_t sh[];  // one counter (or output cursor) per partition
    const int nparts = 1 << bits;
    for (int b = threadIdx.x; b < nparts; b += JP_BLOCK)
        sh[b] = WRITE ? hist[(int64_t)b * nblk + blockIdx.x] : 0;
    __syncthreads();
    const int64_t g0 = (int64_t)blockIdx.x * JP_BLOCK * ept;
    for (int it = 0; it < ept; it++) {
        const int64_t g = g0 + (int64_t)it * JP_BLOCK + threadIdx.x;
        if (g >= ng) break;
        const int32_t p = glist[g];
        const int beta = rb[p];
        int32_t au[C + 1], av[C + 1];
#pragma unroll
        for (int i = 0; i <= C; i++) {
            au[i] = ancU[(int64_t)i * P + p];
            av[i] = ancV[(int64_t)i * P + p];
        }
        jp_emit_edge<C, WRITE>(p, beta, au, av, bits, sh, recs);
    }
    if (!WRITE) {
        __syncthreads();
        for (int b = threadIdx.x; b < nparts; b += JP_BLOCK) hist[(int64_t)b * nblk + blockIdx.x] = sh[b];
    }
}

static void launch_jp_records(gss_ctx ctx, int C, bool write, int64_t ng, const int32_t *glist, int64_t P,
                              const uint8_t *rb, const int32_t *ancU, const int32_t *ancV, int bits, int ept,
                              int32_t nblk, int32_t *hist, JRec *recs)
{
    hipStream_t st = ctx->stream;
    const size_t lds = sizeof(int32_t) << bits;
    // per listed edge: rank, beta* and 2(c+1) ancestors read; with WRITE, 16 B per
    // record written
    const int64_t rd = ng * (5 + 8 * (int64_t)(C + 1));
    const int64_t wr = write ? 16 * ng * 3 * (int64_t)(C + 1) * (C + 1) : 0;
    switch (C) {
#define CASE(k)                                                                                            \
    case k: {                                                                                              \
        auto k_jp_count = &k_jp_records<k, false>;                                                         \
        auto k_jp_scatter = &k_jp_records<k, true>;                                                        \
        if (write)                                                                                         \
            GSS_LAUNCH_B(rd + wr, k_jp_scatter, dim3(nblk), dim3(JP_BLOCK), lds, st, ng, glist, P, rb, ancU, \
                         ancV, bits, ept, nblk, hist, recs);                                               \
        else                                                                                               \
            GSS_LAUNCH_B(rd, k_jp_count, dim3(nblk), dim3(JP_BLOCK), lds, st, ng, glist, P, rb, ancU, ancV,  \
                         bits, ept, nblk, hist, recs);                                                     \
    } break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: throw gss_error{GSS_ERR_ARG, "beta out of range"};
    }
    HIP_OK(hipGetLastError());
}

// pass 3: one workgroup per partition.  Build records of a chunk of JP_CAP records go
// into an LDS hash table; every probe record of the partition then looks up its key.
// arcs found by a workgroup are staged in LDS (the first JP_ARC_LDS) and stored in its
// partition's own slice of the arc buffer (no global counter to contend on)
#define JP_ARC_LDS 1024
__device__ __forceinline__ void jp_probe(const JRec &r, bool active, const unsigned long long *s_ab,
                                         const int32_t *s_p, const uint32_t *s_meta, const int32_t *s_tab,
                                         int2 *s_arc, int32_t *s_narc, int32_t arc_slot, int2 *arc_slice,
                                         int32_t *__restrict__ indeg)
{
    const int j = (r.meta >> 16) & 255, l = (r.meta >> 8) & 255, beta = r.meta & 255;
    uint32_t h = (uint32_t)jp_hash(r.ab) & (JP_TAB - 1);
    while (__ballot(active)) {
        bool hit = false;
        int32_t t = 0;
        if (active) {
            const int li = s_tab[h];
            if (li < 0) {
                active = false;
            } else {
                if (s_ab[li] == r.ab) {
                    const uint32_t mk = s_meta[li];
                    t = s_p[li];
                    hit = (int)(mk >> 8) <= beta - j && (int)(mk & 255) <= beta - l && t > r.p;
                }
                h = (h + 1) & (JP_TAB - 1);
            }
        }
        if (hit) {
            const int32_t a = atomicAdd(s_narc, 1);
            if (a < JP_ARC_LDS) s_arc[a] = make_int2(r.p, t);
            else if (a < arc_slot) arc_slice[a] = make_int2(r.p, t);
            if (indeg) atomicAdd(&indeg[t], 1);
        }
    }
}

__global__ __launch_bounds__(JP_BLOCK) void k_jp_join(const JRec *__restrict__ recs, const int32_t *__restrict__ off,
                                                       int32_t nblk, int32_t nparts, const int64_t *__restrict__ total,
                                                       int32_t arc_slot, int2 *__restrict__ arc_buf,
                                                       int32_t *__restrict__ arc_cnt, int32_t *__restrict__ indeg,
                                                       const int32_t *__restrict__ parts)
{
    constexpr int PER = JP_CAP / JP_BLOCK;
    __shared__ unsigned long long s_ab[JP_CAP];
    __shared__ int32_t s_p[JP_CAP];
    __shared__ uint32_t s_meta[JP_CAP];
    __shared__ int32_t s_tab[JP_TAB];
    __shared__ int2 s_arc[JP_ARC_LDS];
    __shared__ int32_t s_narc;
    // parts == null: every partition, arc slices indexed by partition, in-degrees counted.
    // Otherwise a second run over the listed partitions whose arcs overflowed their slice:
    // slices indexed by list position, in-degrees already counted by the first run.
    const int64_t part = parts ? parts[blockIdx.x] : blockIdx.x;
    if (parts) indeg = nullptr;
    const int64_t start = off[part * nblk];
    const int64_t end = (part + 1 < nparts) ? off[(part + 1) * nblk] : *total;
    int2 *arc_slice = arc_buf + (int64_t)blockIdx.x * arc_slot;
    if (threadIdx.x == 0) s_narc = 0;
    JRec zero;
    zero.ab = 0;
    zero.p = 0;
    zero.meta = 0;
    for (int64_t c0 = start; c0 < end; c0 += JP_CAP) {
        const int64_t c1 = (end - c0 < JP_CAP) ? end : c0 + JP_CAP;
        // this chunk's records: all loads in flight together
        JRec rr[PER];
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int64_t q = c0 + k * JP_BLOCK + threadIdx.x;
            rr[k] = q < c1 ? recs[q] : zero;
        }
        for (int h = threadIdx.x; h < JP_TAB; h += JP_BLOCK) s_tab[h] = -1;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int li = k * JP_BLOCK + threadIdx.x;
            if (c0 + li < c1) {
                s_ab[li] = rr[k].ab;
                s_p[li] = rr[k].p;
                s_meta[li] = rr[k].meta;
                if (!(rr[k].meta & JP_PROBE)) {
                    uint32_t h = (uint32_t)jp_hash(rr[k].ab) & (JP_TAB - 1);
                    while (atomicCAS(&s_tab[h], -1, li) != -1) h = (h + 1) & (JP_TAB - 1);
                }
            }
        }
        __syncthreads();
        if (c0 == start && c1 == end) {
            // the whole partition is this chunk: its probe records are already in registers
#pragma unroll
            for (int k = 0; k < PER; k++) {
                const bool act = c0 + k * JP_BLOCK + threadIdx.x < c1 && (rr[k].meta & JP_PROBE);
                jp_probe(rr[k], act, s_ab, s_p, s_meta, s_tab, s_arc, &s_narc, arc_slot, arc_slice, indeg);
            }
        } else {
            for (int64_t q0 = start; q0 < end; q0 += JP_BLOCK) {
                const int64_t q = q0 + threadIdx.x;
                const JRec r = q < end ? recs[q] : zero;
                jp_probe(r, q < end && (r.meta & JP_PROBE), s_ab, s_p, s_meta, s_tab, s_arc, &s_narc, arc_slot,
                         arc_slice, indeg);
            }
        }
        __syncthreads();
    }
    const int32_t na = s_narc;
    if (threadIdx.x == 0) arc_cnt[part] = na;  // the true count: above arc_slot the host retries
    for (int a = threadIdx.x; a < na && a < arc_slot && a < JP_ARC_LDS; a += JP_BLOCK) arc_slice[a] = s_arc[a];
}

// arc_off = exclusive scan of the partitions' arc counts, total[0] = their sum and
// total[3] = the largest count (one workgroup; nparts a multiple of 1024, at most 16384)
__global__ __launch_bounds__(1024) void k_jp_offsets(const int32_t *__restrict__ cnt, int32_t nparts,
                                                    int32_t *__restrict__ arc_off, int64_t *total)
{
    __shared__ int32_t s_sum[1024 / GSS_WAVE + 1];
    __shared__ int32_t s_max[1024 / GSS_WAVE];
    const int per = nparts / 1024;
    const int32_t b0 = threadIdx.x * per;
    int32_t sum = 0, mx = 0;
    for (int k = 0; k < per; k++) {
        sum += cnt[b0 + k];
        mx = max(mx, cnt[b0 + k]);
    }
    int32_t tot;
    int32_t ex = block_exclusive_scan<int32_t>(sum, s_sum, &tot);
    for (int k = 0; k < per; k++) {
        arc_off[b0 + k] = ex;
        ex += cnt[b0 + k];
    }
    for (int d = 32; d > 0; d >>= 1) mx = max(mx, __shfl_xor(mx, d, GSS_WAVE));
    if (lane_id() == 0) s_max[threadIdx.x / GSS_WAVE] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 1024 / GSS_WAVE; w++) mx = max(mx, s_max[w]);
        total[0] = tot;
        total[3] = mx;
    }
}
// the partitions' arcs, packed (arc_cnt scanned to offsets)
// packs every partition's arcs (arc_cnt scanned to offsets); partitions that overflowed
// their first slice read from the second run's buffer (ov_slot[part] >= 0)
__global__ void k_jp_pack(const int2 *__restrict__ arc_buf, const int32_t *__restrict__ arc_cnt,
                          const int32_t *__restrict__ arc_off, int32_t arc_slot, const int32_t *__restrict__ ov_slot,
                          const int2 *__restrict__ ov_buf, int32_t ov_size, int2 *__restrict__ arcs)
{
    const int64_t part = blockIdx.x;
    const int32_t n = arc_cnt[part], o = arc_off[part];
    const int32_t os = ov_slot ? ov_slot[part] : -1;
    const int2 *src = os >= 0 ? ov_buf + (int64_t)os * ov_size : arc_buf + part * (int64_t)arc_slot;
    for (int a = threadIdx.x; a < n; a += blockDim.x) arcs[o + a] = src[a];
}

__global__ void k_state_init(int64_t NG, const int32_t *__restrict__ glist, const int32_t *__restrict__ indeg,
                             uint8_t *__restrict__ state)
{
    int64_t gi = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gi < NG) {
        const int32_t p = glist[gi];
        state[p] = indeg[p] == 0 ? ST_CAND : ST_UNDEC;
    }
}

// Every edge without in-arcs is recovered (k_state_init), so every target of such an edge
// is marked; one pass over all arcs settles those, and only arcs into still-undecided
// targets go on to the rounds.
__global__ void k_arc_settle(int64_t A, const int2 *__restrict__ arcs, const int32_t *__restrict__ indeg,
                             uint8_t *__restrict__ state)
{
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= A) return;
    int2 e = arcs[a];
    if (indeg[e.x] == 0) state[e.y] = ST_MARK;  // the source has no in-arcs: recovered
}

__global__ void k_arc_compact(int64_t A, const int2 *__restrict__ arcs, const uint8_t *__restrict__ state,
                              int2 *__restrict__ out, unsigned long long *count)
{
    int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool keep = false;
    int2 e = make_int2(0, 0);
    if (a < A) {
        e = arcs[a];
        keep = state[e.y] == ST_UNDEC;
    }
    uint64_t m = __ballot(keep);
    if (!m) return;
    unsigned long long base = 0;
    int leader = __ffsll((long long)m) - 1;
    if (lane_id() == leader) base = atomicAdd(count, (unsigned long long)__popcll(m));
    base = __shfl(base, leader, GSS_WAVE);
    if (keep) out[base + __popcll(m & lanemask_lt())] = e;
}

// Dependency rounds over the compacted arcs (x -> y: y is strictly similar to the earlier
// x).  A round marks every undecided target with a recovered source, counts for each
// undecided target its marked sources, and recovers the targets whose sources are all
// marked.  Arcs always point forward in the order, so the rounds end.
//
// Many arcs: each phase is a grid-wide kernel over the arcs and a round is three
// launches; the first phase of round r also resets the counts of undecided targets and
// records whether any target is still undecided (flag[r]); once a round finds none,
// every later launch returns at once.  The rounds are queued without host waits, and a
// single-workgroup kernel finishes whatever they left (usually nothing).
// rf: [0] done, [1] rounds completed by the grid-wide kernels, [2 + r] flag[r]
#define RES_GRID_ROUNDS 4
#define RES_GRID_MIN 65536  // arcs (before settling) from which the grid-wide rounds pay
__global__ void k_round_mark(const unsigned long long *A, const int2 *__restrict__ arcs, uint8_t *state,
                             int32_t *mcnt, int32_t *rf, int r)
{
    if (rf[0]) return;
    const int64_t n = (int64_t)*A;
    bool und = false;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
        const int2 e = arcs[a];
        if (state[e.y] == ST_UNDEC) {
            und = true;
            mcnt[e.y] = 0;
            if (state[e.x] == ST_CAND) state[e.y] = ST_MARK;
        }
    }
    if (__syncthreads_or(und) && threadIdx.x == 0) rf[2 + r] = 1;
}
__global__ void k_round_count(const unsigned long long *A, const int2 *__restrict__ arcs,
                              const uint8_t *__restrict__ state, int32_t *mcnt, int32_t *rf, int r)
{
    if (rf[0]) return;
    if (!rf[2 + r]) {  // nothing was undecided when round r began: r rounds settled it
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            rf[0] = 1;
            rf[1] = r;
        }
        return;
    }
    const int64_t n = (int64_t)*A;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
        const int2 e = arcs[a];
        if (state[e.y] == ST_UNDEC && state[e.x] == ST_MARK) atomicAdd(&mcnt[e.y], 1);
    }
}
__global__ void k_round_settle(const unsigned long long *A, const int2 *__restrict__ arcs,
                               const int32_t *__restrict__ indeg, uint8_t *state, const int32_t *__restrict__ mcnt,
                               int32_t *rf, int r)
{
    if (rf[0]) return;
    const int64_t n = (int64_t)*A;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < n; a += (int64_t)gridDim.x * blockDim.x) {
        const int2 e = arcs[a];
        if (state[e.y] == ST_UNDEC && mcnt[e.y] == indeg[e.y]) state[e.y] = ST_CAND;
    }
    if (r == RES_GRID_ROUNDS - 1 && blockIdx.x == 0 && threadIdx.x == 0) rf[1] = RES_GRID_ROUNDS;
}

// single workgroup: the remaining rounds (all of them when rf is null); rounds_out gets
// the total number of rounds
__global__ __launch_bounds__(1024) void k_resolve_dev(const unsigned long long *A, const int2 *__restrict__ arcs,
                                                      const int32_t *__restrict__ indeg, uint8_t *state, int32_t *mcnt,
                                                      const int32_t *rf, int64_t *rounds_out)
{
    const int64_t n = (int64_t)*A;
    int64_t rounds = rf ? rf[1] : 0;
    if (rf && rf[0]) {
        if (threadIdx.x == 0) *rounds_out = rounds;
        return;
    }
    if (rf) {  // counts left by the grid-wide rounds; stop if nothing is undecided
        int undec = 0;
        for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
            const int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC) {
                mcnt[e.y] = 0;
                undec = 1;
            }
        }
        if (!__syncthreads_or(undec)) {
            if (threadIdx.x == 0) *rounds_out = rounds;
            return;
        }
    }
    while (n > 0) {
        for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
            int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC && state[e.x] == ST_CAND) state[e.y] = ST_MARK;
        }
        __syncthreads();
        for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
            int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC && state[e.x] == ST_MARK) atomicAdd(&mcnt[e.y], 1);
        }
        __syncthreads();
        for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
            int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC && mcnt[e.y] == indeg[e.y]) state[e.y] = ST_CAND;
        }
        __syncthreads();
        int undec = 0;
        for (int64_t a = threadIdx.x; a < n; a += blockDim.x) {
            int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC) {
                mcnt[e.y] = 0;
                undec = 1;
            }
        }
        rounds++;
        if (!__syncthreads_or(undec)) break;
    }
    if (threadIdx.x == 0) *rounds_out = rounds;
}

// ------------------------------------------------------------------------------------
// 6. selection of the first `need` recovered edges in rank order
// ------------------------------------------------------------------------------------
// candidate flags (1 = recovered) per rank, scanned into ranks among candidates
__global__ void k_cand_flags(int64_t P, const uint8_t *__restrict__ state, int32_t *__restrict__ flag)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) flag[p] = state[p] == ST_CAND ? 1 : 0;
    if (p == P) flag[p] = 0;
}

// per graph: candidates in its rank range [pstart[g], pstart[g+1]); out[G]: the flags word
// (read back with the counts)
__global__ void k_cand_per_graph(int32_t G, const int64_t *__restrict__ pstart, const int32_t *__restrict__ candq,
                                 const uint32_t *__restrict__ flags, int64_t *__restrict__ out)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G) out[g] = (int64_t)candq[pstart[g + 1]] - (int64_t)candq[pstart[g]];
    if (g == G) out[G] = (int64_t)*flags;
}

struct GraphOut {
    int32_t *order;      // may be null
    uint8_t *mask;
    int64_t ebase;       // union edge id of the graph's first edge
    int64_t nrec;        // edges already recovered (earlier passes)
    int64_t need;        // edges still wanted (0: the graph takes nothing in this round)
    int64_t pstart;      // first rank of the graph in the prefix
    int32_t full;        // the prefix holds every eligible edge of the graph
};

// Writes the candidates a graph takes in this prefix round, decided on the device from
// its candidate count cand[g] by the rule of the pass: the first `need` candidates when
// there are that many, all of them when the prefix held every eligible edge (a pass
// that ends short), otherwise none (a longer prefix follows).  A stretch that was not a
// finite double (F_RANGE) fails the call: nothing is written then.
// go: one record per graph (device), or null for one graph whose record is go1
__global__ void k_cand_write(int64_t P, const uint8_t *__restrict__ state, const int32_t *__restrict__ candq,
                             const int32_t *__restrict__ rg, const GraphOut *__restrict__ go, GraphOut go1,
                             const int64_t *__restrict__ cand, const int32_t *__restrict__ rid,
                             const int32_t *__restrict__ sj, uint64_t *__restrict__ key,
                             const uint32_t *__restrict__ flags)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || state[p] != ST_CAND || (*flags & F_RANGE)) return;
    const int32_t g = rg ? rg[p] : 0;
    const GraphOut o = go ? go[g] : go1;
    const int64_t c = cand[g];
    const int64_t take = (c >= o.need || o.full) ? (c < o.need ? c : o.need) : 0;
    int64_t r = (int64_t)candq[p] - (int64_t)candq[o.pstart];
    if (r >= take) return;
    int32_t local = (int32_t)(rid[p] - o.ebase);
    if (o.order) o.order[o.nrec + r] = local;
    o.mask[local] = 1;
    key[sj[p]] = 0;  // recovered: leaves the pool of later passes
}

__global__ void k_fill_i32_r(int32_t *p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_mask_tree(const int32_t *__restrict__ tree_eid, int32_t x0, int32_t x1, int64_t ebase,
                            uint8_t *__restrict__ mask)
{
    int32_t x = x0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (x < x1 && tree_eid[x] >= 0) mask[tree_eid[x] - ebase] = 1;
}

// subtask statistics of one graph (block) over its vertex range
__global__ __launch_bounds__(RB) void k_lca_stats_g(const int32_t *__restrict__ lcacnt,
                                                    const int32_t *__restrict__ vbase, int64_t *__restrict__ out)
{
    __shared__ int64_t snz[RB], smx[RB];
    int32_t g = blockIdx.x;
    int64_t nz = 0, mx = 0;
    for (int32_t x = vbase[g] + threadIdx.x; x < vbase[g + 1]; x += RB) {
        int32_t c = lcacnt[x];
        nz += c > 0;
        mx = c > mx ? c : mx;
    }
    snz[threadIdx.x] = nz;
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int h = RB / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            snz[threadIdx.x] += snz[threadIdx.x + h];
            smx[threadIdx.x] = max(smx[threadIdx.x], smx[threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * g] = snz[0];
        out[2 * g + 1] = smx[0];
    }
}

__global__ void k_edge_lca_out(int64_t M, const int32_t *__restrict__ off_id, const int32_t *__restrict__ lca,
                               const uint8_t *__restrict__ bst, int32_t *__restrict__ lca_out,
                               int32_t *__restrict__ b_out)
{
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= M) return;
    int32_t id = off_id[j];
    if (lca_out) lca_out[id] = lca[j];
    if (b_out) b_out[id] = bst[j];
}

// ------------------------------------------------------------------------------------
// host
// ------------------------------------------------------------------------------------
static RmqView rmq_view(gss_tree t)
{
    RmqView q;
    q.epk = t->epk;
    q.pmask = t->pmask;
    q.ppre = t->ppre;
    q.psuf = t->psuf;
    q.bmin = t->bmin;
    q.bmask = t->bmask;
    q.bpre = t->bpre;
    q.bsuf = t->bsuf;
    q.sbst = t->sbst;
    q.nsb = t->nsb;
    return q;
}

// reads counter words [0, nwords) back; `used` names the words the caller uses
static void read_counters(gss_ctx ctx, int nwords, uint64_t used)
{
    ctx->readback(ctx->h_counters, ctx->d_counters, sizeof(int64_t) * nwords, used);
}

// Stable LSD radix sort of (key, val) pairs by key ascending, with no host round trip.
// With key_bytes = 0 all eight digit positions run (a position where every key agrees
// is a plain copy); with key_bytes > 0 (keys known to be below 2^(8 key_bytes)) only the
// low key_bytes positions run.  With a device count dn only the first min(n, *dn) pairs
// are sorted (the rest of the output is undefined).
static void radix_sort_pairs(gss_ctx ctx, uint64_t *&k, int32_t *&v, uint64_t *&k2, int32_t *&v2, int64_t n,
                             int key_bytes = 0, const int64_t *dn = nullptr)
{
    if (n <= 1) return;
    hipStream_t st = ctx->stream;
    const int64_t ntiles = (n + RS_TILE - 1) / RS_TILE;
    int32_t *ghist = ctx->alloc<int32_t>(8 * 256);
    fill_bytes(ctx, ghist, 0, sizeof(int32_t) * 8 * 256);
    const int npos = key_bytes > 0 ? key_bytes : 8;
    GSS_LAUNCH_B(8 * n, k_rs_ghist, dim3((unsigned)std::min<int64_t>(ntiles, 512)), dim3(RS_BLOCK), 0, st, k, n, dn,
                 npos, ghist);
    for (int p = 0; p < npos; p++) {
        uint32_t epoch = 0;
        uint64_t *status = lb_begin(ctx, ntiles * 256, &epoch);
        GSS_LAUNCH_B(24 * n, k_rs_onesweep, dim3((unsigned)ntiles), dim3(RS_BLOCK), 0, st, k, v, n, dn, 8 * p, ntiles,
                     ghist + p * 256, status, epoch, lb_ticket_ptr(ctx), k2, v2);
        HIP_OK(hipGetLastError());
        std::swap(k, k2);
        std::swap(v, v2);
    }
    ctx->free(ghist);
}

// Sort of (key, value) pairs with distinct values by (key, value): the sample sort for
// the short sorts of a prefix (a few launches whatever the key width), the radix sort
// (stable, so the same order) above its size limit.  dn: a device count of the pairs
// that matter (the rest hold the largest key and stay last); only the radix sort uses it.
static void sort_pairs(gss_ctx ctx, uint64_t *&k, int32_t *&v, uint64_t *&k2, int32_t *&v2, int64_t n,
                       int key_bytes = 0, const int64_t *dn = nullptr)
{
    // one-byte keys take one radix pass (two launches), fewer than the sample sort's four
    if (n <= sample_sort_max() && !ctx->sort_radix && key_bytes != 1) sample_sort_pairs(ctx, k, v, k2, v2, n);
    else radix_sort_pairs(ctx, k, v, k2, v2, n, key_bytes, dn);
}

static int bytes_for(uint64_t maxkey)
{
    int b = 1;
    while (b < 8 && (maxkey >> (8 * b)) != 0) b++;
    return b;
}

struct PrefixResult {
    int64_t P = 0, arcs = 0, rounds = 0, nsub = 0, nlocal = 0, njoin = 0;
    bool rounds_pending = false;  // rounds is in h_counters[12] after the next synchronisation
    std::vector<int64_t> Pg, cand;  // per graph (cand after finish_candidates)
    int64_t *dcand = nullptr;       // per graph candidate counts on the device (and the flags)
    uint32_t flags = 0;             // the flags word read with the counts
};

struct PrefixBufs {
    int32_t *sj = nullptr, *rid = nullptr, *ancU = nullptr, *ancV = nullptr, *indeg = nullptr, *mcnt = nullptr;
    int32_t *ru = nullptr, *rv = nullptr, *rdu = nullptr, *rdv = nullptr, *rl = nullptr, *rg = nullptr;
    int32_t *grp = nullptr, *sub_ptr = nullptr, *sub_lca = nullptr, *candq = nullptr;
    int64_t *pstart = nullptr;
    uint8_t *rb = nullptr, *state = nullptr;
    int32_t *glist = nullptr;
    void release(gss_ctx ctx)
    {
        void *ps[] = {sj, rid, ancU,    ancV,    indeg, mcnt,  ru,        rv,    rdu,   rdv,
                      rl, rg,  grp,     sub_ptr, sub_lca, candq, pstart, rb,    state, glist};
        for (void *p : ps) ctx->free(p);
        *this = PrefixBufs();
    }
};

__global__ void k_rank_graph(int64_t P, const int32_t *__restrict__ sj, const int32_t *__restrict__ off_g,
                             int32_t *__restrict__ rg)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P) rg[p] = off_g[sj[p]];
}

// Candidates per graph (ranks among the recovered edges), counted on the device into
// res.dcand without waiting: the outputs are written from the device counts, and
// finish_candidates reads them back afterwards.
static void count_candidates(gss_ctx ctx, int32_t G, int64_t P, PrefixBufs &B, PrefixResult &res)
{
    hipStream_t st = ctx->stream;
    B.candq = ctx->alloc<int32_t>(P + 2);
    GSS_LAUNCH(k_cand_flags, dim3(grid_for(P + 1, RB)), dim3(RB), 0, st, P, B.state, B.candq);
    scan_exclusive_i32(ctx, B.candq, P + 1, false);
    res.dcand = ctx->alloc<int64_t>(G + 1);
    GSS_LAUNCH(k_cand_per_graph, dim3(grid_for(G + 1, RB)), dim3(RB), 0, st, G, B.pstart, B.candq, ctx->d_flags,
               res.dcand);
}

// res.cand, the flags word (res.flags) and the pending round count from the device;
// synchronises
static void finish_candidates(gss_ctx ctx, int32_t G, PrefixResult &res)
{
    res.cand.assign(G + 1, 0);
    ctx->readback(res.cand.data(), res.dcand, sizeof(int64_t) * (G + 1));
    res.flags = (uint32_t)res.cand[G];
    res.cand.resize(G);
    if (res.rounds_pending) res.rounds = ctx->h_counters[12];
    ctx->free(res.dcand);
    res.dcand = nullptr;
}

// Resolves, for every graph g, the prefix {key >= thr[g]} of its criticality order.
// One graph: the prefix's per-tile counts {key >= thr} scanned in place (pc, one word per
// PX_TILE keys and one more); the total goes to counter word 13
static void prefix_tile_counts(gss_ctx ctx, gss_tree t, const uint64_t *key, const uint64_t *thr, int32_t *pc)
{
    const int64_t M = t->M;
    const int64_t nthr = (M + PX_TILE - 1) / PX_TILE;
    GSS_LAUNCH_B(8 * M, k_prefix_count, dim3((unsigned)std::max<int64_t>(nthr, 1)), dim3(256), 0, ctx->stream, key, M,
                 (const int32_t *)nullptr, thr, pc);
    scan_exclusive_i32_dev(ctx, pc, nthr, ctx->d_counters + 13);
}

// pc_ready (one graph): the scanned tile counts, already computed by prefix_tile_counts
// (ownership passes here)
static PrefixResult resolve_prefix(gss_ctx ctx, gss_tree t, int32_t c, const uint64_t *key, const uint8_t *bst,
                                   const int32_t *lca, const uint64_t *thr, const std::vector<int64_t> &plen,
                                   PrefixBufs &B, const gss_params *prm, int32_t *pc_ready = nullptr)
{
    hipStream_t st = ctx->stream;
    const int64_t M = t->M;
    const int32_t G = t->G;
    const int32_t *off_g = (G > 1) ? t->off_g : nullptr;
    PrefixResult res;
    std::vector<void *> scratch;
    // compaction (id order: graph-major)
    int64_t nthr = (M + PX_TILE - 1) / PX_TILE;  // tiles
    // a single graph's prefix length is known from the selection; the scan's total is
    // compared with it at the next read-back instead of being waited for here
    const bool p_known = G == 1;
    int32_t *pc = pc_ready;
    if (!pc) {
        pc = ctx->alloc<int32_t>(nthr + 1);
        if (p_known) {
            prefix_tile_counts(ctx, t, key, thr, pc);
        } else {
            GSS_LAUNCH_B(8 * M, k_prefix_count, dim3((unsigned)std::max<int64_t>(nthr, 1)), dim3(256), 0, st, key, M,
                         off_g, thr, pc);
        }
    }
    int64_t P;
    if (p_known) {
        P = plen[0];
    } else {
        P = scan_exclusive_i32(ctx, pc, nthr, true);
    }
    res.P = P;
    res.Pg.assign(G, 0);
    if (G > 1) {
        int64_t *before = ctx->alloc<int64_t>(G + 1);
        GSS_LAUNCH(k_prefix_before, dim3(G + 1), dim3(256), 0, st, key, M, off_g, thr, t->d_obase, pc, P, before);
        std::vector<int64_t> hb(G + 1);
        ctx->readback(hb.data(), before, sizeof(int64_t) * (G + 1));
        for (int32_t g = 0; g < G; g++) res.Pg[g] = hb[g + 1] - hb[g];
        ctx->free(before);
    } else {
        res.Pg[0] = P;
    }
    B.pstart = ctx->alloc<int64_t>(G + 1);
    uint64_t *k1 = ctx->alloc<uint64_t>(P + 1), *k2 = ctx->alloc<uint64_t>(P + 1);
    int32_t *v1 = ctx->alloc<int32_t>(P + 1), *v2 = ctx->alloc<int32_t>(P + 1);
    GSS_LAUNCH_B(8 * M + 12 * P, k_prefix_write, dim3((unsigned)std::max<int64_t>(nthr, 1)), dim3(256), 0, st, key, M,
                 off_g, thr, pc, P, v1, k1);
    if (p_known) GSS_LAUNCH(k_prefix_pad, dim3(1), dim3(256), 0, st, ctx->d_counters + 13, P, v1, k1, B.pstart);
    ctx->free(pc);
    sort_pairs(ctx, k1, v1, k2, v2, P);  // stretch descending, id ascending
    if (G > 1) {  // stable by graph: each graph's prefix becomes contiguous, in rank order
        GSS_LAUNCH(k_graph_key, dim3(grid_for(P, RB)), dim3(RB), 0, st, P, v1, t->off_g, k1);
        radix_sort_pairs(ctx, k1, v1, k2, v2, P, bytes_for((uint64_t)(G - 1)));
    }
    B.sj = v1;
    if (!p_known) {  // one graph: written by k_prefix_pad
        std::vector<int64_t> ps(G + 1, 0);
        for (int32_t g = 0; g < G; g++) ps[g + 1] = ps[g] + res.Pg[g];
        ctx->h2d(B.pstart, ps.data(), sizeof(int64_t) * (G + 1));
    }
    if (G > 1) {
        B.rg = ctx->alloc<int32_t>(P + 1);
        GSS_LAUNCH(k_rank_graph, dim3(grid_for(P, RB)), dim3(RB), 0, st, P, B.sj, t->off_g, B.rg);
    }
    // per-rank data, and (lca, rank) pairs for the grouping
    B.rid = ctx->alloc<int32_t>(P + 1);
    B.rb = ctx->alloc<uint8_t>(P + 1);
    B.ru = ctx->alloc<int32_t>(P + 1);
    B.rv = ctx->alloc<int32_t>(P + 1);
    B.rdu = ctx->alloc<int32_t>(P + 1);
    B.rdv = ctx->alloc<int32_t>(P + 1);
    B.rl = ctx->alloc<int32_t>(P + 1);
    B.ancU = ctx->alloc<int32_t>((int64_t)(c + 1) * P + 1);
    B.ancV = ctx->alloc<int32_t>((int64_t)(c + 1) * P + 1);
    uint64_t *lkey = k1, *lkey2 = k2;
    int32_t *lval = v2, *lval2 = ctx->alloc<int32_t>(P + 1);
    // per prefix edge: id, endpoints, beta*, LCA and 2(c+1) ancestors read; the rank
    // record, the (LCA, rank) pair and the ancestor columns written
    GSS_LAUNCH_B((58 + 16 * (int64_t)(c + 1)) * P, k_rank_gather, dim3(grid_for(P, RB)), dim3(RB), 0, st, P, B.sj,
                 t->off_id, t->off_u, t->off_v, bst,
               lca, t->vrec, t->parent, c, B.rid, B.rb, B.ru, B.rv, B.rdu, B.rdv, B.rl, lkey, lval, B.ancU, B.ancV);

    if (prm->flags & GSS_F_LOOSE) {
        // feGRASS's loose condition (Def. "Similar edge (Loose)"): loosely similar edges
        // need not share their LCA, so there are no subtasks; the whole prefix is decided
        // by rounds over tree-ancestor cells, with the constant radius c for every edge
        ctx->free(lkey);
        ctx->free(lkey2);
        ctx->free(lval);
        ctx->free(lval2);
        B.state = ctx->alloc<uint8_t>(P + 1);
        res.rounds = loose_greedy(ctx, t->n, t->virt_root, P, c, B.ancU, B.ancV, B.state);
        count_candidates(ctx, G, P, B, res);
        return res;
    }

    // LCA subtasks (Alg. 1 Step 3): stable sort of the rank-ordered prefix by LCA.  LCAs
    // of different graphs of a batch are different vertices, so subtasks never mix graphs.
    sort_pairs(ctx, lkey, lval, lkey2, lval2, P, bytes_for((uint64_t)(t->n - 1)));  // LCA < n
    B.grp = lval;
    scratch.push_back(lkey2);
    scratch.push_back(lval2);
    const uint64_t *glca = lkey;
    scratch.push_back(lkey);
    int32_t *hid = ctx->alloc<int32_t>(P + 1);
    scratch.push_back(hid);
    launch_grouping_kernels(ctx, P, glca, hid);
    // the subtask count stays on the device until the queue split is read back below;
    // everything sized by it takes the bound P instead
    int64_t *d_nsub = ctx->d_counters + 14;
    if (P > 0) scan_exclusive_i32_dev(ctx, hid, P, d_nsub);
    else fill_bytes(ctx, d_nsub, 0, sizeof(int64_t));
    const int32_t cap = (int32_t)P;  // nsub <= P
    B.sub_ptr = ctx->alloc<int32_t>(P + 1);
    B.sub_lca = ctx->alloc<int32_t>(P + 1);
    launch_group_ptr(ctx, P, glca, hid, B.sub_ptr, B.sub_lca);

    // work queue: local subtasks first, heaviest predicted cost first
    const int32_t local_max = std::min<int32_t>(ctx->local_max, GSS_LOCAL_CAP);
    float *feat = nullptr, *pred = nullptr;
    const bool want_feat = (prm->sched == GSS_SCHED_LEARNED && ctx->model_ready) || ctx->record;
    if (want_feat && P > 0) {
        feat = ctx->alloc<float>(P * GSS_NFEAT + 1);
        scratch.push_back(feat);
        launch_subtask_features(ctx, d_nsub, cap, B.sub_ptr, B.sub_lca, B.grp, B.rdu, B.rdv, B.rb, B.ru, B.rv,
                                t->vrec, P, local_max, feat);
        if (prm->sched == GSS_SCHED_LEARNED && ctx->model_ready) {
            pred = ctx->alloc<float>(P + 1);
            scratch.push_back(pred);
            costmodel_predict(ctx, feat, P, d_nsub, pred);
        }
    }
    uint64_t *qk = ctx->alloc<uint64_t>(P + 1), *qk2 = ctx->alloc<uint64_t>(P + 1);
    int32_t *qv = ctx->alloc<int32_t>(P + 1), *qv2 = ctx->alloc<int32_t>(P + 1);
    int32_t *is_local = ctx->alloc<int32_t>(P + 1);
    fill_bytes(ctx, ctx->d_counters + 4, 0, 4 * sizeof(int64_t));
    // queue keys: cost in the low cost_bits (sizes are at most P; predicted costs are float
    // bits), the on-join-path flag above them
    // (the edge-count order uses the dense key of k_subtask_keys: cost_bits = 0)
    int cost_bits = 0;
    if (pred) cost_bits = 32;
    // counters: queued subtasks in the low half of word 4, the lane-sized ones among them
    // in its high half, join-path edges in word 6
    launch_subtask_keys(ctx, d_nsub, cap, B.sub_ptr, local_max, pred, cost_bits, qk, qv, is_local,
                        (int32_t *)(ctx->d_counters + 4), (int32_t *)(ctx->d_counters + 4) + 1,
                        (unsigned long long *)(ctx->d_counters + 6));
    // only the nsub queued entries are read, so the radix sort orders just those
    sort_pairs(ctx, qk, qv, qk2, qv2, P,
               bytes_for(cost_bits == 0 ? 3 * ((uint64_t)local_max + 1) - 1 : ((uint64_t)3 << cost_bits) - 1), d_nsub);
    // words 4 and 6: the queue split; 14: the subtask count; 13: the prefix length (one graph).
    // The join list (ranks of the edges on the join path, in grouped order; at most P of
    // them) needs only device data: it is built while the host waits, and left unused when
    // no subtask goes to the join.
    ctx->readback_early(ctx->h_counters, ctx->d_counters, sizeof(int64_t) * 15,
                        (1ull << 4) | (1ull << 6) | (1ull << 14) | (p_known ? 1ull << 13 : 0ull));
    B.glist = ctx->alloc<int32_t>(P + 1);
    launch_join_list(ctx, P, glca, hid, is_local, B.grp, B.glist);
    ctx->wait_early();
    if (p_known && ctx->h_counters[13] != P) {
        for (void *p : scratch) ctx->free(p);
        throw gss_error{GSS_ERR_HIP, "prefix length differs from the selection"};
    }
    const int64_t nsub = ctx->h_counters[14];
    res.nsub = nsub;
    const int32_t nlocal = (int32_t)(ctx->h_counters[4] & 0xffffffffll);
    const int32_t nsmall = (int32_t)((uint64_t)ctx->h_counters[4] >> 32);
    const int64_t nglobal_edges = ctx->h_counters[6];
    res.nlocal = nlocal;
    res.njoin = nglobal_edges;
    scratch.push_back(qk);
    scratch.push_back(qk2);
    scratch.push_back(qv);
    scratch.push_back(qv2);
    scratch.push_back(is_local);

    B.state = ctx->alloc<uint8_t>(P + 1);

    // Step 4, small and medium subtasks: persistent work-queue kernel
    // launched at once without a join, else between the join's read-back and the wait for
    // it (it touches neither the join's edges nor its counters), to cover the host round trip
    uint64_t *cycles = nullptr;
    bool local_launched = false;
    auto local_step = [&]() {
        if (local_launched || nlocal <= 0) return;
        local_launched = true;
        if (ctx->record) {
            cycles = ctx->alloc<uint64_t>(nsub + 1);
            scratch.push_back(cycles);
            fill_bytes(ctx, cycles, 0, sizeof(uint64_t) * (nsub + 1));
        }
        fill_bytes(ctx, ctx->d_counters + 5, 0, sizeof(int64_t));
        SubtaskArgs a;
        a.P = P;
        a.grp = B.grp;
        a.sub_ptr = B.sub_ptr;
        a.queue = qv;
        a.nqueue = nlocal;
        a.nbig = nlocal;  // set below once the grid is known
        a.local_max = local_max;
        a.queue_head = (unsigned int *)(ctx->d_counters + 5);  // two 32-bit heads, zeroed above
        a.ancU = B.ancU;
        a.ancV = B.ancV;
        a.rdu = B.rdu;
        a.rdv = B.rdv;
        a.rb = B.rb;
        a.state = B.state;
        a.cycles = cycles;
        int blocks = std::max(1, std::min<int>(ctx->local_blocks, (nlocal + 3) / 4));
        // candidate scratch: at most ~256 MB whatever the setting
        const size_t per_wave = (size_t)std::max<int32_t>(local_max, 1) * local_desc_bytes(c);
        blocks = (int)std::min<int64_t>(blocks, std::max<int64_t>(1, ((int64_t)256 << 20) / (4 * per_wave)));
        // small subtasks run one per lane when there are enough of them to give every
        // wavefront several full takes; otherwise whole wavefronts take them too
        a.nbig = (nsmall >= (int64_t)16 * blocks * 4) ? nlocal - nsmall : nlocal;
        // about 16 chunks per wavefront; one subtask per take while the queue is short
        // the heaviest 2 W queue entries are dealt to the W wavefronts (LPT bins)
        a.lpt_rounds = 2;
        a.chunk = ctx->local_chunk > 0 ? ctx->local_chunk
                                       : std::max<int32_t>(1, std::min<int32_t>(64, a.nbig / (blocks * 4 * 16)));
        void *scr = ctx->alloc<uint8_t>((size_t)blocks * 4 * per_wave + 64);
        scratch.push_back(scr);
        a.cand_scratch = scr;
        // per queued edge: rank, 2(c+1) ancestors, depths and beta* read, state written;
        // per subtask: queue entry and bounds
        if (ctx->prof) ctx->prof_bytes = (P - nglobal_edges) * (14 + 8 * (int64_t)(c + 1)) + 12 * (int64_t)nlocal;
        launch_local_recover(ctx, c, a, blocks);
    };
    if (nsub <= nlocal) local_step();
    // Step 4, large subtasks: hash join + dependency rounds over their edges
    B.indeg = ctx->alloc<int32_t>(P + 1);
    B.mcnt = ctx->alloc<int32_t>(P + 1);
    if (nsub > nlocal) {
        // partition the join records by key hash: about 1024 records per partition, so a
        // partition usually fits one LDS chunk of the join
        const int64_t nslots = nglobal_edges * 3 * (int64_t)(c + 1) * (c + 1);
        int bits = JP_BITS_MIN;
        while (bits < JP_BITS_MAX && nslots > ((int64_t)1024 << bits)) bits++;
        const int32_t nparts = 1 << bits;
        // edges per thread: about four records per partition counter in each workgroup,
        // which keeps the histogram matrix near nslots / 4 entries
        const int64_t per_edge = 3 * (int64_t)(c + 1) * (c + 1);
        const int ept = (int)std::max<int64_t>(1, std::min<int64_t>(64, (4 * (int64_t)nparts + JP_BLOCK * per_edge - 1) /
                                                                            (JP_BLOCK * per_edge)));
        const int32_t nblk = (int32_t)((nglobal_edges + (int64_t)JP_BLOCK * ept - 1) / ((int64_t)JP_BLOCK * ept));
        int32_t *jhist = ctx->alloc<int32_t>((int64_t)nparts * nblk + 1);
        JRec *recs = ctx->alloc<JRec>(nslots + 1);
        int64_t *d_total = ctx->d_counters + 8;
        launch_jp_records(ctx, c, false, nglobal_edges, B.glist, P, B.rb, B.ancU, B.ancV, bits, ept, nblk, jhist,
                          recs);
        scan_exclusive_i32_dev(ctx, jhist, (int64_t)nparts * nblk, d_total);
        launch_jp_records(ctx, c, true, nglobal_edges, B.glist, P, B.rb, B.ancU, B.ancV, bits, ept, nblk, jhist,
                          recs);
        const int32_t arc_slot = 128;
        int32_t *arc_cnt = ctx->alloc<int32_t>(nparts + 1);
        int32_t *arc_off = ctx->alloc<int32_t>(nparts + 1);
        {
            int2 *arc_buf = ctx->alloc<int2>((int64_t)nparts * arc_slot);
            fill_bytes(ctx, B.indeg, 0, sizeof(int32_t) * (P + 1));
            GSS_LAUNCH_B(16 * nslots, k_jp_join, dim3(nparts), dim3(JP_BLOCK), 0, st, recs, jhist, nblk, nparts, d_total,
                         arc_slot, arc_buf, arc_cnt, B.indeg, (const int32_t *)nullptr);
            GSS_LAUNCH(k_jp_offsets, dim3(1), dim3(1024), 0, st, arc_cnt, nparts, arc_off, ctx->d_counters);
            ctx->readback_early(ctx->h_counters, ctx->d_counters, sizeof(int64_t) * 4, (1ull << 0) | (1ull << 3));
            local_step();
            ctx->wait_early();
            const int64_t most = ctx->h_counters[3];
            const int64_t A = ctx->h_counters[0];
            // partitions with more arcs than their slice: joined again into a buffer of their own
            int32_t *ov_slot = nullptr, *ov_parts = nullptr;
            int2 *ov_buf = nullptr;
            int32_t ov_size = 0;
            if (most > arc_slot) {
                std::vector<int32_t> hc(nparts), slot(nparts, -1), list;
                ctx->readback(hc.data(), arc_cnt, sizeof(int32_t) * nparts);
                for (int32_t q = 0; q < nparts; q++)
                    if (hc[q] > arc_slot) {
                        slot[q] = (int32_t)list.size();
                        list.push_back(q);
                    }
                ov_size = (int32_t)most;
                ov_slot = ctx->alloc<int32_t>(nparts);
                ov_parts = ctx->alloc<int32_t>(list.size());
                ov_buf = ctx->alloc<int2>((int64_t)list.size() * ov_size);
                ctx->h2d(ov_slot, slot.data(), sizeof(int32_t) * nparts);
                ctx->h2d(ov_parts, list.data(), sizeof(int32_t) * list.size());
                GSS_LAUNCH(k_jp_join, dim3((unsigned)list.size()), dim3(JP_BLOCK), 0, st, recs, jhist, nblk, nparts,
                           d_total,
                           ov_size, ov_buf, arc_cnt, B.indeg, (const int32_t *)ov_parts);
            }
            int2 *arcs = ctx->alloc<int2>(A + 1);
            if (A > 0)
                GSS_LAUNCH(k_jp_pack, dim3(nparts), dim3(64), 0, st, arc_buf, arc_cnt, arc_off, arc_slot, ov_slot,
                           ov_buf, ov_size, arcs);
            ctx->free(arc_buf);
            ctx->free(ov_slot);
            ctx->free(ov_parts);
            ctx->free(ov_buf);
            res.arcs = A;
            fill_bytes(ctx, B.mcnt, 0, sizeof(int32_t) * (P + 1));
            GSS_LAUNCH(k_state_init, dim3(grid_for(nglobal_edges, RB)), dim3(RB), 0, st, nglobal_edges, B.glist,
                       B.indeg, B.state);
            if (A > 0) {
                int2 *arcs2 = ctx->alloc<int2>(A + 1);
                fill_bytes(ctx, ctx->d_counters + 2, 0, sizeof(int64_t));
                GSS_LAUNCH(k_arc_settle, dim3(grid_for(A, RB)), dim3(RB), 0, st, A, arcs, B.indeg, B.state);
                GSS_LAUNCH(k_arc_compact, dim3(grid_for(A, RB)), dim3(RB), 0, st, A, arcs, B.state, arcs2,
                           (unsigned long long *)(ctx->d_counters + 2));
                const unsigned long long *dA = (const unsigned long long *)(ctx->d_counters + 2);
                int32_t *rf = nullptr;
                if (A >= RES_GRID_MIN) {  // many arcs: grid-wide rounds first
                    rf = ctx->alloc<int32_t>(2 + RES_GRID_ROUNDS);
                    fill_bytes(ctx, rf, 0, sizeof(int32_t) * (2 + RES_GRID_ROUNDS));
                    const dim3 g((unsigned)std::min<int64_t>(grid_for(A, RB), 4096));
                    for (int r = 0; r < RES_GRID_ROUNDS; r++) {
                        GSS_LAUNCH(k_round_mark, g, dim3(RB), 0, st, dA, arcs2, B.state, B.mcnt, rf, r);
                        GSS_LAUNCH(k_round_count, g, dim3(RB), 0, st, dA, arcs2, B.state, B.mcnt, rf, r);
                        GSS_LAUNCH(k_round_settle, g, dim3(RB), 0, st, dA, arcs2, B.indeg, B.state, B.mcnt, rf, r);
                    }
                }
                GSS_LAUNCH(k_resolve_dev, dim3(1), dim3(1024), 0, st, dA, arcs2, B.indeg, B.state, B.mcnt,
                           (const int32_t *)rf, ctx->d_counters + 1);
                if (rf) ctx->free(rf);
                // rounds (for the info record) arrive with the next synchronisation
                ctx->readback_async(&ctx->h_counters[12], ctx->d_counters + 1, sizeof(int64_t));
                res.rounds_pending = true;
                ctx->free(arcs2);
            }
            ctx->free(arcs);
        }
        ctx->free(jhist);
        ctx->free(recs);
        ctx->free(arc_cnt);
        ctx->free(arc_off);
    }
    local_step();  // launched above when there was a join
    count_candidates(ctx, G, P, B, res);
    if (ctx->record && nsub > 0) trace_append(ctx, nsub, B.sub_ptr, B.sub_lca, P, feat, cycles, qv, nlocal);
    for (void *p : scratch) ctx->free(p);
    return res;
}

// Per graph, a key threshold T such that {key >= T} holds at least want[g] eligible edges
// (and not many more).  want[g] <= 0: graph not selected (threshold above every key).
// The digit levels run on the device, each graph's state updated by the pick kernel,
// without a host round trip between levels; dthr points at the thresholds (device, G) in the
// state block state_out, which the caller frees.
//
// plen[g] receives the number of keys >= thr[g]: the keys above the chosen bucket plus the
// bucket's own (every key of the bucket is at least its lowest key, every key below it is
// smaller), all eligible keys when the threshold is 1, none when the graph is not selected.
// overlap (may be null) is called with the device thresholds after each read-back of the
// state is enqueued and before it is waited for: work that needs only the thresholds runs
// during the host round trip (it is called again after a later level, whose thresholds
// then replace the earlier ones)
static void select_thresholds(gss_ctx ctx, gss_tree t, const uint64_t *key, uint32_t *hist, bool hist_ready,
                              const std::vector<int64_t> &want, const std::vector<int64_t> &eligible,
                              std::vector<int64_t> &plen, const uint64_t *&dthr, void *&state_out,
                              const std::function<void(const uint64_t *)> *overlap = nullptr)
{
    hipStream_t st = ctx->stream;
    const int32_t G = t->G;
    const int32_t *off_g = (G > 1) ? t->off_g : nullptr;
    constexpr int LEVELS = 6;
    const int shifts[LEVELS] = {51, 39, 27, 15, 3, 0};
    const int widths[LEVELS] = {12, 12, 12, 12, 12, 3};
    // initial state, packed in int64 words: need, above, plen, eligible, pmask, pval, thr
    // (G each), then the per-level active counts (int32, LEVELS + 1)
    const size_t words = 7 * (size_t)G + (LEVELS + 2) / 2;
    std::vector<int64_t> init(words, 0);
    int64_t *h_need = init.data(), *h_plen = h_need + 2 * G, *h_elig = h_need + 3 * G;
    uint64_t *h_thr = (uint64_t *)(h_need + 6 * G);
    int32_t *h_active = (int32_t *)(h_need + 7 * G);
    int32_t refining = 0;
    plen.assign(G, 0);
    for (int32_t g = 0; g < G; g++) {
        h_elig[g] = eligible[g];
        h_thr[g] = ~0ull;  // not selected: above every key
        if (want[g] <= 0) continue;
        if (want[g] >= eligible[g]) {
            h_thr[g] = 1;  // every eligible key is >= 1
            h_plen[g] = eligible[g];
        } else {
            h_need[g] = want[g];
            refining++;
        }
    }
    h_active[0] = refining;
    int64_t *dstate = ctx->alloc<int64_t>((int64_t)words);
    ctx->h2d(dstate, init.data(), sizeof(int64_t) * words);
    SelState S;
    S.need = dstate;
    S.above = dstate + G;
    S.plen = dstate + 2 * G;
    S.eligible = dstate + 3 * G;
    S.pmask = (uint64_t *)(dstate + 4 * G);
    S.pval = (uint64_t *)(dstate + 5 * G);
    S.thr = (uint64_t *)(dstate + 6 * G);
    S.active = (int32_t *)(dstate + 7 * G);
    // the first two levels settle most selections; the state read back after them says
    // whether the remaining levels are needed (one more read-back if so)
    int lv = 0;
    for (int upto : {2, LEVELS}) {
        if (refining > 0) {
            if (lv == 0 && (!hist_ready || G > 1)) fill_bytes(ctx, hist, 0, sizeof(uint32_t) * SEL_BINS * G);
            for (; lv < upto; lv++) {
                if (lv > 0 || !hist_ready || G > 1)
                    GSS_LAUNCH(k_key_hist, dim3(std::min<int64_t>(grid_for(t->M, RB), 2048)), dim3(RB), 0, st, key,
                               t->M, off_g, shifts[lv], widths[lv], S.pmask, S.pval, S.need, hist, S.active + lv);
                GSS_LAUNCH(k_pick_update, dim3(G), dim3(1024), 0, st, hist, lv, shifts[lv], widths[lv],
                           lv == LEVELS - 1 ? 1 : 0, S);
            }
        }
        if (overlap) {
            ctx->readback_early(init.data(), dstate, sizeof(int64_t) * words);
            (*overlap)(S.thr);
            ctx->wait_early();
        } else {
            ctx->readback(init.data(), dstate, sizeof(int64_t) * words);
        }
        refining = lv < LEVELS ? h_active[lv] : 0;
        if (refining == 0) break;
    }
    memcpy(plen.data(), h_plen, sizeof(int64_t) * G);
    // the thresholds stay in the state block, which the caller frees after using them
    dthr = S.thr;
    state_out = dstate;
}

// Recovery of every graph of a tree (a single graph, or a batch).
gss_status recover_impl(gss_ctx ctx, gss_tree t, const gss_params *prms, uint8_t *const *masks,
                        int32_t *const *orders, double *stretch, gss_info *infos)
{
    hipStream_t st = ctx->stream;
    const int32_t n = t->n, G = t->G;
    const int64_t M = t->M;
    const int32_t c = prms[0].beta;
    const int key_rt = (prms[0].flags & GSS_F_KEY_RT) ? 1 : 0;
    for (int32_t g = 1; g < G; g++)
        if (prms[g].beta != c || prms[g].sched != prms[0].sched ||
            ((prms[g].flags & GSS_F_KEY_RT) ? 1 : 0) != key_rt ||
            ((prms[g].flags ^ prms[0].flags) & GSS_F_LOOSE))
            throw gss_error{GSS_ERR_ARG,
                            "all graphs of a batch need the same beta, schedule, sort key and similarity condition"};
    std::vector<int64_t> K(G), nrec(G, 0), eligible(G), want(G), mg(G);
    std::vector<int32_t> passes(G, 0);
    std::vector<int64_t> lastP(G, 0), nsubg(G, 0), largest(G, 0);
    std::vector<bool> active(G);
    for (int32_t g = 0; g < G; g++) {
        K[g] = target_count(t, g, &prms[g]);
        mg[g] = t->ebase[g + 1] - t->ebase[g];
        eligible[g] = t->Mg[g];
        fill_bytes(ctx, masks[g], 0, (size_t)mg[g]);
        if (prms[g].flags & GSS_F_MASK_TREE) {
            int32_t x0 = (int32_t)t->vbase[g], x1 = (int32_t)t->vbase[g + 1];
            GSS_LAUNCH(k_mask_tree, dim3(grid_for(x1 - x0, RB)), dim3(RB), 0, st, t->tree_eid, x0, x1, t->ebase[g],
                       masks[g]);
        }
    }
    if (stretch) fill_bytes(ctx, stretch, 0, sizeof(double) * (size_t)t->m);
    fill_bytes(ctx, ctx->d_flags, 0, sizeof(uint32_t));

    uint64_t *key = ctx->alloc<uint64_t>(M + 1);
    int32_t *lca = ctx->alloc<int32_t>(M + 1);
    uint8_t *bst = ctx->alloc<uint8_t>(M + 1);
    uint32_t *hist = ctx->alloc<uint32_t>((int64_t)SEL_BINS * G);
    // per-LCA edge counts: subtask statistics, and two of the cost model's features
    const bool need_lca_counts = (prms[0].flags & GSS_F_STATS) != 0;
    int32_t *lcacnt = need_lca_counts ? ctx->alloc<int32_t>(n) : nullptr;
    fill_bytes(ctx, hist, 0, sizeof(uint32_t) * SEL_BINS);
    if (lcacnt) fill_bytes(ctx, lcacnt, 0, sizeof(int32_t) * n);
    // per off-tree edge: u, v, w (16 B); first, depth and D of u and v and D of the LCA
    // (56 B); the two LCA-sequence entries that answer the range minimum (16 B); key, LCA and
    // beta* written (13 B); optional stretch (8 B)
    if (M > 0) {
        if (STRETCH_HIST && G == 1)
            GSS_LAUNCH_B((101 + (stretch ? 8 : 0)) * M, k_edge_stretch<true>,
                         dim3((unsigned)std::min<int64_t>(grid_for(M, RB * EDGE_ITEMS), EDGE_GRID)), dim3(RB), 0, st,
                         M, t->off_id, t->off_u, t->off_v, t->off_w, t->vrec, rmq_view(t), t->scale, c, key, lca, bst,
                         stretch, hist, lcacnt, ctx->d_flags, key_rt);
        else
            GSS_LAUNCH_B((101 + (stretch ? 8 : 0)) * M, k_edge_stretch<false>,
                         dim3((unsigned)std::min<int64_t>(grid_for(M, RB * EDGE_ITEMS), EDGE_GRID)), dim3(RB), 0, st,
                         M, t->off_id, t->off_u, t->off_v, t->off_w, t->vrec, rmq_view(t), t->scale, c, key, lca, bst,
                         stretch, (uint32_t *)nullptr, lcacnt, ctx->d_flags, key_rt);
    }
    HIP_OK(hipGetLastError());
    if (!lcacnt) {
        for (int32_t g = 0; g < G; g++) nsubg[g] = largest[g] = -1;
    } else if (G == 1) {
        int64_t init2[2] = {0, 0};
        ctx->h2d(ctx->d_counters + 2, init2, sizeof init2);
        GSS_LAUNCH(k_lca_stats, dim3(std::min<int64_t>(grid_for(n, RB), 1024)), dim3(RB), 0, st, lcacnt, n,
                   ctx->d_counters + 2);
        read_counters(ctx, 4, (1ull << 2) | (1ull << 3));
        nsubg[0] = ctx->h_counters[2];
        largest[0] = ctx->h_counters[3];
    } else {
        int64_t *dst = ctx->alloc<int64_t>(2 * G);
        std::vector<int64_t> hs(2 * G);
        GSS_LAUNCH(k_lca_stats_g, dim3(G), dim3(RB), 0, st, lcacnt, t->d_vbase, dst);
        ctx->readback(hs.data(), dst, sizeof(int64_t) * 2 * G);
        ctx->free(dst);
        for (int32_t g = 0; g < G; g++) {
            nsubg[g] = hs[2 * g];
            largest[g] = hs[2 * g + 1];
        }
    }
    // the range flag comes back with the first prefix round's candidate counts (k_cand_write
    // writes nothing while it is set), or, when no round runs, by itself at the end
    bool flags_checked = false;
    auto cleanup = [&]() {
        ctx->free(key);
        ctx->free(lca);
        ctx->free(bst);
        ctx->free(hist);
        ctx->free(lcacnt);
    };

    auto first_want = [&](int32_t g) {
        int64_t need = K[g] - nrec[g];
        return std::min<int64_t>(eligible[g], need + need / 4 + 1024);
    };
    int any_active = 0;
    for (int32_t g = 0; g < G; g++) {
        active[g] = K[g] > 0 && eligible[g] > 0;
        want[g] = active[g] ? first_want(g) : 0;
        any_active |= active[g];
    }
    bool hist_ready = STRETCH_HIST && G == 1;
    int64_t arcs = 0, rounds = 0, njoin = 0;
    GraphOut *dgo = ctx->alloc<GraphOut>(G);
    std::vector<GraphOut> go(G);
    if (!any_active) ctx->readback_async(&ctx->h_counters[15], ctx->d_flags, sizeof(uint32_t));
    while (any_active) {
        const size_t amark = ctx->arena_mark();  // allocation-free calls: rounds reuse the scratch
        std::vector<int64_t> plen;
        const uint64_t *dthr = nullptr;
        void *sel_state = nullptr;
        // one graph: the prefix's tile counts run while the host waits for the selection
        int32_t *pc = nullptr;
        std::function<void(const uint64_t *)> tile_counts;
        if (G == 1) {
            pc = ctx->alloc<int32_t>((t->M + PX_TILE - 1) / PX_TILE + 1);
            tile_counts = [&](const uint64_t *thr) { prefix_tile_counts(ctx, t, key, thr, pc); };
        }
        select_thresholds(ctx, t, key, hist, hist_ready, want, eligible, plen, dthr, sel_state,
                          pc ? &tile_counts : nullptr);
        hist_ready = false;
        PrefixBufs B;
        PrefixResult r = resolve_prefix(ctx, t, c, key, bst, lca, dthr, plen, B, &prms[0], pc);
        ctx->free(sel_state);
        // the outputs are written before the candidate counts come back: k_cand_write
        // applies the pass rule below to the device counts (and writes nothing on F_RANGE)
        int64_t pst = 0;
        for (int32_t g = 0; g < G; g++) {
            go[g].order = orders ? orders[g] : nullptr;
            go[g].mask = masks[g];
            go[g].ebase = t->ebase[g];
            go[g].nrec = nrec[g];
            go[g].need = active[g] ? K[g] - nrec[g] : 0;
            go[g].full = r.Pg[g] >= eligible[g] ? 1 : 0;
            go[g].pstart = pst;
            pst += r.Pg[g];
            if (active[g]) lastP[g] = r.Pg[g];
        }
        if (r.P > 0) {
            if (G > 1) ctx->h2d(dgo, go.data(), sizeof(GraphOut) * G);  // one graph: a kernel argument
            GSS_LAUNCH(k_cand_write, dim3(grid_for(r.P, RB)), dim3(RB), 0, st, r.P, B.state, B.candq, B.rg,
                       G > 1 ? (const GraphOut *)dgo : (const GraphOut *)nullptr, go[0], r.dcand, B.rid, B.sj,
                       key, ctx->d_flags);
            HIP_OK(hipGetLastError());
        }
        finish_candidates(ctx, G, r);  // synchronises: also delivers the range flag
        if (!flags_checked) {
            const uint32_t f = r.flags;
            flags_checked = true;
            if (f & F_RANGE) {
                B.release(ctx);
                ctx->free(dgo);
                cleanup();
                throw gss_error{GSS_ERR_RANGE, "a stretch is not a finite double"};
            }
        }
        arcs = r.arcs;
        rounds = r.rounds;
        njoin = r.njoin;
        any_active = 0;
        for (int32_t g = 0; g < G; g++) {
            if (!active[g]) continue;
            const int64_t need = K[g] - nrec[g];
            if (r.cand[g] >= need) {  // done: the first `need` candidates are final
                nrec[g] += need;
                eligible[g] -= need;
                if (need > 0) passes[g]++;
                active[g] = false;
            } else if (r.Pg[g] >= eligible[g]) {  // the pass ended short: next pass
                const int64_t take = r.cand[g];
                nrec[g] += take;
                eligible[g] -= take;
                if (take > 0) passes[g]++;
                active[g] = take > 0 && eligible[g] > 0 && nrec[g] < K[g];
                if (active[g]) want[g] = first_want(g);
            } else {  // the prefix held too few candidates: a longer one is needed
                double ratio = (double)need / (double)std::max<int64_t>(r.cand[g], 1);
                int64_t next = (int64_t)((double)r.Pg[g] * ratio * 1.15) + 1024;
                want[g] = std::min<int64_t>(eligible[g], std::max<int64_t>(next, r.Pg[g] + 1024));
            }
            if (!active[g]) want[g] = 0;
            any_active |= active[g];
        }
        B.release(ctx);
        ctx->arena_reset(amark);
    }
    ctx->sync();
    if (!flags_checked) {
        uint32_t f = 0;
        memcpy(&f, &ctx->h_counters[15], sizeof f);  // the synchronisation above delivered it
        if (f & F_RANGE) {
            ctx->free(dgo);
            cleanup();
            throw gss_error{GSS_ERR_RANGE, "a stretch is not a finite double"};
        }
    }
    ctx->free(dgo);
    cleanup();
    bool short_any = false;
    for (int32_t g = 0; g < G; g++) {
        short_any |= nrec[g] < K[g];
        if (!infos) continue;
        gss_info &info = infos[g];
        info.m = mg[g];
        info.n_offtree = t->Mg[g];
        info.k = K[g];
        info.n_recovered = nrec[g];
        info.n_subtasks = nsubg[g];
        info.largest_subtask = largest[g];
        info.prefix_len = lastP[g];
        info.n_arcs = arcs;
        info.n_join = njoin;
        info.passes = passes[g];
        info.rounds = (int32_t)rounds;
        info.sched = (prms[0].sched == GSS_SCHED_LEARNED && ctx->model_ready) ? GSS_SCHED_LEARNED
                                                                               : GSS_SCHED_EDGECOUNT;
    }
    return short_any ? GSS_SHORT : GSS_OK;
}

void edge_lca_impl(gss_ctx ctx, gss_tree t, int32_t beta, int32_t *lca_out, int32_t *b_out)
{
    hipStream_t st = ctx->stream;
    const int64_t M = t->M, m = t->m;
    if (lca_out) {
        GSS_LAUNCH(k_fill_i32_r, dim3(grid_for(m, RB)), dim3(RB), 0, st, lca_out, m, -1);
    }
    if (b_out) fill_bytes(ctx, b_out, 0, sizeof(int32_t) * (size_t)m);
    uint64_t *key = ctx->alloc<uint64_t>(M + 1);
    int32_t *lca = ctx->alloc<int32_t>(M + 1);
    uint8_t *bst = ctx->alloc<uint8_t>(M + 1);
    uint32_t *hist = ctx->alloc<uint32_t>(SEL_BINS);
    fill_bytes(ctx, hist, 0, sizeof(uint32_t) * SEL_BINS);
    if (M > 0) {
        GSS_LAUNCH(k_edge_stretch<false>, dim3((unsigned)std::min<int64_t>(grid_for(M, RB * EDGE_ITEMS), EDGE_GRID)),
                   dim3(RB), 0, st, M, t->off_id, t->off_u, t->off_v, t->off_w, t->vrec, rmq_view(t), t->scale, beta,
                   key, lca, bst, (double *)nullptr, (uint32_t *)nullptr, (int32_t *)nullptr, ctx->d_flags, 0);
        GSS_LAUNCH(k_edge_lca_out, dim3(grid_for(M, RB)), dim3(RB), 0, st, M, t->off_id, lca, bst,
                           lca_out, b_out);
    }
    HIP_OK(hipGetLastError());
    ctx->sync();
    ctx->free(key);
    ctx->free(lca);
    ctx->free(bst);
    ctx->free(hist);
}
