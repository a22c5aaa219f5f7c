// gss_recover.hip -- off-tree edge recovery on gfx950.
//
// Paper: Alg. 1 (Steps 1-4), eq. RT, eq. beta-new, Def. "Similar edge (Strict)",
// Lemma "strictly similar edges share their LCA".
//
// Path of one pass:
//  1. k_edge_stretch  every off-tree edge: LCA by RMQ over the Euler tour, exact
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

#include "gss_impl.h"
#include "gss_subtask.h"

#define RB 256
#define SEL_BITS 12
#define SEL_BINS (1 << SEL_BITS)
#define CHUNK 16

enum : uint8_t { ST_UNDEC = 0, ST_CAND = 1, ST_MARK = 2 };

struct RmqView {
    const uint64_t *epk, *pmask, *ppre, *psuf, *bmin, *bmask, *bpre, *bsuf, *sbst;
    int32_t nsb;
};

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int ctz64(uint64_t x) { return __ffsll((long long)x) - 1; }

// minimum packed (depth<<32|vertex) over block minima b0..b1 (inclusive, b0 <= b1)
__device__ __forceinline__ uint64_t rmq_blocks(const RmqView &q, int32_t b0, int32_t b1)
{
    int32_t s0 = b0 >> 6, s1 = b1 >> 6;
    if (s0 == s1) {
        uint64_t m = q.bmask[b1] & (~0ull << (b0 & 63));
        return q.bmin[(s0 << 6) + ctz64(m)];
    }
    uint64_t best = umin64(q.bsuf[b0], q.bpre[b1]);
    int32_t a = s0 + 1, c = s1 - 1;
    if (a <= c) {
        int32_t len = c - a + 1;
        int k = 31 - __clz(len);
        const uint64_t *lv = q.sbst + (int64_t)k * q.nsb;
        best = umin64(best, umin64(lv[a], lv[c - (1 << k) + 1]));
    }
    return best;
}

// minimum packed value over Euler positions i..j (i <= j)
__device__ __forceinline__ uint64_t rmq(const RmqView &q, int32_t i, int32_t j)
{
    int32_t bi = i >> 6, bj = j >> 6;
    if (bi == bj) {
        uint64_t m = q.pmask[j] & (~0ull << (i & 63));
        return q.epk[(bi << 6) + ctz64(m)];
    }
    uint64_t best = umin64(q.psuf[i], q.ppre[j]);
    if (bi + 1 <= bj - 1) best = umin64(best, rmq_blocks(q, bi + 1, bj - 1));
    return best;
}

// ------------------------------------------------------------------------------------
// 1. per-edge LCA / resistance / stretch / beta*
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(RB) void k_edge_stretch(
    int64_t M, const int32_t *__restrict__ off_id, const int32_t *__restrict__ off_u,
    const int32_t *__restrict__ off_v, const double *__restrict__ off_w,
    const VRec *__restrict__ vrec, RmqView q, int32_t scale, int32_t c, uint64_t *__restrict__ key, int32_t *__restrict__ lca,
    uint8_t *__restrict__ bst, double *__restrict__ stretch_out, uint32_t *__restrict__ hist,
    int32_t *__restrict__ lcacnt, uint32_t *flags)
{
    __shared__ uint32_t sh[SEL_BINS];
    for (int i = threadIdx.x; i < SEL_BINS; i += RB) sh[i] = 0;
    __syncthreads();
    int64_t j = (int64_t)blockIdx.x * RB + threadIdx.x;
    int32_t l = -1;
    if (j < M) {
        int32_t u = off_u[j], v = off_v[j];
        VRec ru = vrec[u], rv = vrec[v];
        int32_t fu = ru.first, fv = rv.first;
        uint64_t pk = (fu <= fv) ? rmq(q, fu, fv) : rmq(q, fv, fu);
        l = (int32_t)(uint32_t)pk;
        int32_t dl = (int32_t)(pk >> 32);
        int32_t du = ru.depth - dl, dv = rv.depth - dl;
        u128 Dl = vrec[l].D;
        u128 R = add128(sub128(ru.D, Dl), sub128(rv.D, Dl));
        double r;
        bool ok = u128_to_double_rne(R, scale, &r);
        double s = off_w[j] * r;
        uint64_t bits = (uint64_t)__double_as_longlong(s);
        if (!ok || ((bits >> 52) & 0x7ff) == 0x7ff) {
            atomicOr(flags, F_RANGE);
            bits = 1;
        }
        int32_t b = du < dv ? du : dv;
        if (c < b) b = c;
        key[j] = bits;
        lca[j] = l;
        bst[j] = (uint8_t)b;
        if (stretch_out) stretch_out[off_id[j]] = s;
        atomicAdd(&sh[(uint32_t)(bits >> 51) & (SEL_BINS - 1)], 1u);
    }
    // subtask sizes: lanes sharing the first lane's LCA add once (skewed graphs put most
    // edges on a few LCAs), the others add individually
    if (lcacnt) {
        uint64_t active = __ballot(l >= 0);
        if (active) {
            int leader = ctz64(active);
            int32_t lv = __shfl(l, leader, GSS_WAVE);
            uint64_t same = __ballot(l == lv) & active;
            if (lane_id() == leader) atomicAdd(&lcacnt[lv], __popcll(same));
            else if (l >= 0 && l != lv) atomicAdd(&lcacnt[l], 1);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SEL_BINS; i += RB)
        if (sh[i]) atomicAdd(&hist[i], sh[i]);
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
// 2. radix select of the prefix threshold
// ------------------------------------------------------------------------------------
// histogram of key digit [shift, shift+width) over eligible keys matching the prefix
__global__ __launch_bounds__(RB) void k_key_hist(const uint64_t *__restrict__ key, int64_t M, int shift,
                                                 int width, uint64_t pmask, uint64_t pval,
                                                 uint32_t *__restrict__ hist)
{
    __shared__ uint32_t sh[SEL_BINS];
    for (int i = threadIdx.x; i < SEL_BINS; i += RB) sh[i] = 0;
    __syncthreads();
    uint32_t dmask = (1u << width) - 1;
    for (int64_t j = (int64_t)blockIdx.x * RB + threadIdx.x; j < M; j += (int64_t)gridDim.x * RB) {
        uint64_t k = key[j];
        if (k != 0 && (k & pmask) == pval) atomicAdd(&sh[(uint32_t)(k >> shift) & dmask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SEL_BINS; i += RB)
        if (sh[i]) atomicAdd(&hist[i], sh[i]);
}

// digit holding the need-th largest element; writes {digit, count above it, its count}
__global__ __launch_bounds__(1024) void k_pick_bucket(const uint32_t *__restrict__ hist, int width,
                                                      int64_t need, int64_t *out)
{
    __shared__ int64_t lds[1024 / GSS_WAVE + 1];
    const int nb = 1 << width;
    const int per = (nb + 1023) / 1024;
    // thread t owns digits (from the top) [t*per, t*per+per)
    int64_t s = 0;
    for (int i = 0; i < per; i++) {
        int r = threadIdx.x * per + i;
        if (r < nb) s += hist[nb - 1 - r];
    }
    int64_t tot;
    int64_t before = block_exclusive_scan<int64_t>(s, lds, &tot);
    if (before < need && before + s >= need) {
        int64_t acc = before;
        for (int i = 0; i < per; i++) {
            int r = threadIdx.x * per + i;
            if (r >= nb) break;
            int64_t h = hist[nb - 1 - r];
            if (acc + h >= need) {
                out[0] = nb - 1 - r;
                out[1] = acc;
                out[2] = h;
                break;
            }
            acc += h;
        }
    }
    if (threadIdx.x == 0 && tot < need) {
        out[0] = -1;
        out[1] = tot;
        out[2] = 0;
    }
}

// ------------------------------------------------------------------------------------
// 3. compaction of {key >= T} (id order) and the stable radix sort
// ------------------------------------------------------------------------------------
__global__ void k_prefix_count(const uint64_t *__restrict__ key, int64_t M, uint64_t T,
                               int32_t *__restrict__ cnt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t j0 = t * CHUNK;
    if (j0 >= M) return;
    int32_t c = 0;
    for (int i = 0; i < CHUNK; i++) {
        int64_t j = j0 + i;
        if (j < M && key[j] >= T) c++;
    }
    cnt[t] = c;
}

__global__ void k_prefix_write(const uint64_t *__restrict__ key, int64_t M, uint64_t T,
                               const int32_t *__restrict__ off, int32_t *__restrict__ pj,
                               uint64_t *__restrict__ pk)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t j0 = t * CHUNK;
    if (j0 >= M) return;
    int32_t q = off[t];
    for (int i = 0; i < CHUNK; i++) {
        int64_t j = j0 + i;
        if (j < M) {
            uint64_t k = key[j];
            if (k >= T) {
                pj[q] = (int32_t)j;
                pk[q] = ~k;  // ascending order of ~key = descending stretch
                q++;
            }
        }
    }
}

__global__ __launch_bounds__(1024) void k_key_varying(const uint64_t *__restrict__ k, int64_t n,
                                                      uint64_t *out)
{
    __shared__ uint64_t so[1024], sa[1024];
    uint64_t o = 0, a = ~0ull;
    for (int64_t i = threadIdx.x; i < n; i += 1024) {
        o |= k[i];
        a &= k[i];
    }
    so[threadIdx.x] = o;
    sa[threadIdx.x] = a;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            so[threadIdx.x] |= so[threadIdx.x + h];
            sa[threadIdx.x] &= sa[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = so[0] ^ sa[0];
}

#define RS_BLOCK 256
#define RS_ITEMS 16
#define RS_TILE (RS_BLOCK * RS_ITEMS)

// per-tile digit counts, stored digit-major: cnt[d * ntiles + tile]
__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint64_t *__restrict__ k, int64_t n, int shift,
                                                      int32_t ntiles, int32_t *__restrict__ cnt)
{
    __shared__ int32_t sh[256];
    sh[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_ITEMS; i++) {
        int64_t idx = base + (int64_t)i * RS_BLOCK + threadIdx.x;
        if (idx < n) atomicAdd(&sh[(uint32_t)(k[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    cnt[(int64_t)threadIdx.x * ntiles + blockIdx.x] = sh[threadIdx.x];
}

// stable scatter: items are ranked in (round, thread) order, which is index order
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                         const int32_t *__restrict__ vin, int64_t n,
                                                         int shift, int32_t ntiles,
                                                         const int32_t *__restrict__ off,
                                                         uint64_t *__restrict__ kout,
                                                         int32_t *__restrict__ vout)
{
    __shared__ int32_t run[256];
    __shared__ int32_t wc[RS_BLOCK / GSS_WAVE][256];
    const int wid = threadIdx.x / GSS_WAVE;
    run[threadIdx.x] = off[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    for (int w = 0; w < RS_BLOCK / GSS_WAVE; w++) wc[w][threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int i = 0; i < RS_ITEMS; i++) {
        int64_t idx = base + (int64_t)i * RS_BLOCK + threadIdx.x;
        bool valid = idx < n;
        uint64_t kk = valid ? kin[idx] : 0;
        int32_t vv = valid ? vin[idx] : 0;
        uint32_t d = (uint32_t)(kk >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        int rank = __popcll(peers & lanemask_lt());
        if (valid && rank == 0) wc[wid][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t o = run[d] + rank;
            for (int w = 0; w < wid; w++) o += wc[w][d];
            kout[o] = kk;
            vout[o] = vv;
        }
        __syncthreads();
        {
            int32_t s = 0;
            for (int w = 0; w < RS_BLOCK / GSS_WAVE; w++) {
                s += wc[w][threadIdx.x];
                wc[w][threadIdx.x] = 0;
            }
            run[threadIdx.x] += s;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// per-rank gather and the anchor hash join
// ------------------------------------------------------------------------------------
struct Slot {
    unsigned long long ab;  // (A << 32) | B, all ones = empty
    int32_t p;              // rank of the inserted edge
    int32_t ik;             // (i << 8) | k
};
#define SLOT_EMPTY 0xffffffffffffffffull

__global__ void k_rank_gather(int64_t P, const int32_t *__restrict__ sj, const int32_t *__restrict__ off_id,
                              const int32_t *__restrict__ off_u, const int32_t *__restrict__ off_v,
                              const uint8_t *__restrict__ bst, const int32_t *__restrict__ lca,
                              const VRec *__restrict__ vrec, int32_t c, int32_t *__restrict__ rid,
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
    int32_t pa = ra.parent, pb = rbv.parent;
    for (int i = 1; i <= c; i++) {
        ancU[(int64_t)i * P + p] = pa;
        ancV[(int64_t)i * P + p] = pb;
        pa = (pa >= 0) ? vrec[pa].parent : -1;
        pb = (pb >= 0) ? vrec[pb].parent : -1;
    }
}

__device__ __forceinline__ uint64_t slot_hash(uint64_t ab) { return mix64(ab * 0x9E3779B97F4A7C15ull + 1); }

__device__ __forceinline__ void join_insert(Slot *tab, uint64_t cap_mask, int32_t A, int32_t B, int32_t p,
                                            int ik)
{
    unsigned long long ab = ((unsigned long long)(uint32_t)A << 32) | (uint32_t)B;
    uint64_t h = slot_hash(ab) & cap_mask;
    for (;;) {
        unsigned long long old = atomicCAS(&tab[h].ab, SLOT_EMPTY, ab);
        if (old == SLOT_EMPTY) {
            tab[h].p = p;
            tab[h].ik = ik;
            return;
        }
        h = (h + 1) & cap_mask;
    }
}

__global__ void k_join_build(int64_t P, int32_t c, const int32_t *__restrict__ ancU,
                             const int32_t *__restrict__ ancV, const uint8_t *__restrict__ is_global, Slot *tab,
                             uint64_t cap_mask)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || !is_global[p]) return;
    for (int orient = 0; orient < 2; orient++) {
        const int32_t *X = orient ? ancV : ancU;
        const int32_t *Y = orient ? ancU : ancV;
        for (int i = 0; i <= c; i++) {
            int32_t A = X[(int64_t)i * P + p];
            if (A < 0) break;
            for (int k = 0; k <= c; k++) {
                int32_t B = Y[(int64_t)k * P + p];
                if (B < 0) break;
                join_insert(tab, cap_mask, A, B, (int32_t)p, (i << 8) | k);
            }
        }
    }
}

__global__ void k_join_probe(int64_t P, const uint8_t *__restrict__ rb, const int32_t *__restrict__ ancU,
                             const int32_t *__restrict__ ancV, const uint8_t *__restrict__ is_global,
                             const Slot *__restrict__ tab, uint64_t cap_mask, int2 *__restrict__ arcs,
                             int64_t arc_cap, unsigned long long *arc_count, int32_t *__restrict__ indeg,
                             uint32_t *flags)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || !is_global[p]) return;
    int beta = rb[p];
    if (beta == 0) return;  // S_u = {u}, S_v = {v}: only the edge itself is similar
    for (int j = 0; j <= beta; j++) {
        int32_t A = ancU[(int64_t)j * P + p];
        if (A < 0) break;
        for (int l = 0; l <= beta; l++) {
            int32_t B = ancV[(int64_t)l * P + p];
            if (B < 0) break;
            unsigned long long ab = ((unsigned long long)(uint32_t)A << 32) | (uint32_t)B;
            uint64_t h = slot_hash(ab) & cap_mask;
            for (;;) {
                unsigned long long s = tab[h].ab;
                if (s == SLOT_EMPTY) break;
                if (s == ab) {
                    int ik = tab[h].ik;
                    int32_t t = tab[h].p;
                    if ((ik >> 8) <= beta - j && (ik & 255) <= beta - l && t > p) {
                        unsigned long long a = atomicAdd(arc_count, 1ull);
                        if ((int64_t)a < arc_cap) {
                            arcs[a] = make_int2((int32_t)p, t);
                            atomicAdd(&indeg[t], 1);
                        } else {
                            atomicOr(flags, F_OVERFLOW);
                        }
                    }
                }
                h = (h + 1) & cap_mask;
            }
        }
    }
}

// ------------------------------------------------------------------------------------
// 5. dependency rounds (one workgroup)
// ------------------------------------------------------------------------------------
__global__ void k_state_init(int64_t P, const int32_t *__restrict__ indeg, const uint8_t *__restrict__ is_global,
                             uint8_t *__restrict__ state)
{
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < P && is_global[p]) state[p] = indeg[p] == 0 ? ST_CAND : ST_UNDEC;
}

__global__ __launch_bounds__(1024) void k_resolve(int64_t A, const int2 *__restrict__ arcs,
                                                  const int32_t *__restrict__ indeg, uint8_t *state,
                                                  int32_t *mcnt, int64_t *rounds_out)
{
    int64_t rounds = 0;
    for (;;) {
        for (int64_t a = threadIdx.x; a < A; a += blockDim.x) {
            int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC && state[e.x] == ST_CAND) state[e.y] = ST_MARK;
        }
        __syncthreads();
        for (int64_t a = threadIdx.x; a < A; a += blockDim.x) {
            int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC && state[e.x] == ST_MARK) atomicAdd(&mcnt[e.y], 1);
        }
        __syncthreads();
        for (int64_t a = threadIdx.x; a < A; a += blockDim.x) {
            int2 e = arcs[a];
            if (state[e.y] == ST_UNDEC && mcnt[e.y] == indeg[e.y]) state[e.y] = ST_CAND;
        }
        __syncthreads();
        int undec = 0;
        for (int64_t a = threadIdx.x; a < A; a += blockDim.x) {
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
__global__ void k_cand_count(int64_t P, const uint8_t *__restrict__ state, int32_t *__restrict__ cnt)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p0 = t * CHUNK;
    if (p0 >= P) return;
    int32_t c = 0;
    for (int i = 0; i < CHUNK; i++) {
        int64_t p = p0 + i;
        if (p < P && state[p] == ST_CAND) c++;
    }
    cnt[t] = c;
}

__global__ void k_cand_write(int64_t P, const uint8_t *__restrict__ state, const int32_t *__restrict__ off,
                             int64_t need, const int32_t *__restrict__ rid, const int32_t *__restrict__ sj,
                             int32_t *__restrict__ order, int64_t order_base, uint8_t *__restrict__ mask,
                             uint64_t *__restrict__ key)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t p0 = t * CHUNK;
    if (p0 >= P) return;
    int64_t q = off[t];
    for (int i = 0; i < CHUNK; i++) {
        int64_t p = p0 + i;
        if (p < P && state[p] == ST_CAND) {
            if (q < need) {
                int32_t id = rid[p];
                if (order) order[order_base + q] = id;
                mask[id] = 1;
                key[sj[p]] = 0;  // recovered: leaves the pool of later passes
            }
            q++;
        }
    }
}

__global__ void k_fill_i32_r(int32_t *p, int64_t n, int32_t v)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_mask_tree(const int32_t *__restrict__ tree_eid, int32_t n, uint8_t *__restrict__ mask)
{
    int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n && tree_eid[x] >= 0) mask[tree_eid[x]] = 1;
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

static void read_counters(gss_ctx ctx, int nwords)
{
    HIP_OK(hipMemcpyAsync(ctx->h_counters, ctx->d_counters, sizeof(int64_t) * nwords, hipMemcpyDeviceToHost,
                          ctx->stream));
    ctx->sync();
}

// stable LSD radix sort of (key, val) pairs by key ascending, only over varying digits
static void radix_sort_pairs(gss_ctx ctx, uint64_t *&k, int32_t *&v, uint64_t *&k2, int32_t *&v2, int64_t n)
{
    if (n <= 1) return;
    hipStream_t st = ctx->stream;
    GSS_LAUNCH(k_key_varying, dim3(1), dim3(1024), 0, st, k, n, (uint64_t *)ctx->d_counters);
    read_counters(ctx, 1);
    uint64_t varying = (uint64_t)ctx->h_counters[0];
    int32_t ntiles = (int32_t)((n + RS_TILE - 1) / RS_TILE);
    int64_t cn = (int64_t)ntiles * 256;
    int32_t *cnt = ctx->alloc<int32_t>(cn + 1);
    for (int shift = 0; shift < 64; shift += 8) {
        if (((varying >> shift) & 255ull) == 0) continue;
        GSS_LAUNCH(k_rs_hist, dim3(ntiles), dim3(RS_BLOCK), 0, st, k, n, shift, ntiles, cnt);
        scan_exclusive_i32(ctx, cnt, cn, false);
        GSS_LAUNCH(k_rs_scatter, dim3(ntiles), dim3(RS_BLOCK), 0, st, k, v, n, shift, ntiles, cnt, k2,
                           v2);
        HIP_OK(hipGetLastError());
        std::swap(k, k2);
        std::swap(v, v2);
    }
    ctx->free(cnt);
}

struct PrefixResult {
    int64_t P = 0, cand = 0, arcs = 0, rounds = 0, nsub = 0, nlocal = 0;
};

// resolves the prefix {key >= T}; leaves state/rid/sj for the caller to select from
struct PrefixBufs {
    int32_t *sj = nullptr, *rid = nullptr, *ancU = nullptr, *ancV = nullptr, *indeg = nullptr, *mcnt = nullptr;
    int32_t *ccnt = nullptr, *ru = nullptr, *rv = nullptr, *rdu = nullptr, *rdv = nullptr, *rl = nullptr;
    int32_t *grp = nullptr, *sub_ptr = nullptr, *sub_lca = nullptr;
    uint8_t *rb = nullptr, *state = nullptr, *is_global = nullptr;
    void release(gss_ctx ctx)
    {
        void *ps[] = {sj, rid, ancU, ancV, indeg, mcnt, ccnt, ru, rv, rdu, rdv, rl, grp, sub_ptr, sub_lca, rb, state,
                      is_global};
        for (void *p : ps) ctx->free(p);
        *this = PrefixBufs();
    }
};

static PrefixResult resolve_prefix(gss_ctx ctx, gss_tree t, int32_t c, const uint64_t *key, const uint8_t *bst,
                                   const int32_t *lca, const int32_t *lcacnt, uint64_t T, PrefixBufs &B,
                                   const gss_params *prm)
{
    hipStream_t st = ctx->stream;
    const int64_t M = t->M;
    PrefixResult res;
    std::vector<void *> scratch;
    // compaction (id order)
    int64_t nthr = (M + CHUNK - 1) / CHUNK;
    int32_t *pc = ctx->alloc<int32_t>(nthr + 1);
    GSS_LAUNCH(k_prefix_count, dim3(grid_for(nthr, RB)), dim3(RB), 0, st, key, M, T, pc);
    int64_t P = scan_exclusive_i32(ctx, pc, nthr, true);
    res.P = P;
    uint64_t *k1 = ctx->alloc<uint64_t>(P + 1), *k2 = ctx->alloc<uint64_t>(P + 1);
    int32_t *v1 = ctx->alloc<int32_t>(P + 1), *v2 = ctx->alloc<int32_t>(P + 1);
    GSS_LAUNCH(k_prefix_write, dim3(grid_for(nthr, RB)), dim3(RB), 0, st, key, M, T, pc, v1, k1);
    ctx->free(pc);
    radix_sort_pairs(ctx, k1, v1, k2, v2, P);  // rank order: v1[p] = off-tree index of rank p
    B.sj = v1;
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
    GSS_LAUNCH(k_rank_gather, dim3(grid_for(P, RB)), dim3(RB), 0, st, P, B.sj, t->off_id, t->off_u, t->off_v, bst,
               lca, t->vrec, c, B.rid, B.rb, B.ru, B.rv, B.rdu, B.rdv, B.rl, lkey, lval, B.ancU, B.ancV);

    // LCA subtasks (Alg. 1 Step 3): stable sort of the rank-ordered prefix by LCA
    radix_sort_pairs(ctx, lkey, lval, lkey2, lval2, P);
    B.grp = lval;
    scratch.push_back(lkey2);
    scratch.push_back(lval2);
    const uint64_t *glca = lkey;
    scratch.push_back(lkey);
    int32_t *hid = ctx->alloc<int32_t>(P + 1);
    scratch.push_back(hid);
    launch_grouping_kernels(ctx, P, glca, hid);
    int64_t nsub = scan_exclusive_i32(ctx, hid, P, true);
    res.nsub = nsub;
    B.sub_ptr = ctx->alloc<int32_t>(nsub + 1);
    B.sub_lca = ctx->alloc<int32_t>(nsub + 1);
    launch_group_ptr(ctx, P, glca, hid, B.sub_ptr, B.sub_lca, (int32_t)nsub);

    // work queue: local subtasks first, heaviest predicted cost first
    const int32_t local_max = std::min<int32_t>(ctx->local_max, GSS_LOCAL_CAP);
    float *feat = nullptr, *pred = nullptr;
    const bool want_feat = (prm->sched == GSS_SCHED_LEARNED && ctx->model_ready) || ctx->record;
    if (want_feat && nsub > 0) {
        feat = ctx->alloc<float>(nsub * GSS_NFEAT + 1);
        scratch.push_back(feat);
        launch_subtask_features(ctx, (int32_t)nsub, B.sub_ptr, B.sub_lca, B.grp, B.rdu, B.rdv, B.rb, B.ru, B.rv,
                                t->vrec, lcacnt, feat);
        if (prm->sched == GSS_SCHED_LEARNED && ctx->model_ready) {
            pred = ctx->alloc<float>(nsub + 1);
            scratch.push_back(pred);
            costmodel_predict(ctx, feat, nsub, pred);
        }
    }
    uint64_t *qk = ctx->alloc<uint64_t>(nsub + 1), *qk2 = ctx->alloc<uint64_t>(nsub + 1);
    int32_t *qv = ctx->alloc<int32_t>(nsub + 1), *qv2 = ctx->alloc<int32_t>(nsub + 1);
    int32_t *is_local = ctx->alloc<int32_t>(nsub + 1);
    HIP_OK(hipMemsetAsync(ctx->d_counters + 4, 0, sizeof(int64_t), st));
    launch_subtask_keys(ctx, (int32_t)nsub, B.sub_ptr, local_max, pred, qk, qv, is_local,
                        (int32_t *)(ctx->d_counters + 4));
    radix_sort_pairs(ctx, qk, qv, qk2, qv2, nsub);
    read_counters(ctx, 5);
    const int32_t nlocal = (int32_t)ctx->h_counters[4];
    res.nlocal = nlocal;
    scratch.push_back(qk);
    scratch.push_back(qk2);
    scratch.push_back(qv);
    scratch.push_back(qv2);
    scratch.push_back(is_local);

    B.state = ctx->alloc<uint8_t>(P + 1);
    B.is_global = ctx->alloc<uint8_t>(P + 1);
    HIP_OK(hipMemsetAsync(B.is_global, 0, P + 1, st));
    if (nsub > nlocal) launch_mark_global(ctx, (int32_t)nsub, B.sub_ptr, is_local, B.grp, B.is_global);

    // Step 4, small and medium subtasks: persistent work-queue kernel
    uint64_t *cycles = nullptr;
    if (nlocal > 0) {
        if (ctx->record) {
            cycles = ctx->alloc<uint64_t>(nsub + 1);
            scratch.push_back(cycles);
            HIP_OK(hipMemsetAsync(cycles, 0, sizeof(uint64_t) * (nsub + 1), st));
        }
        HIP_OK(hipMemsetAsync(ctx->d_counters + 5, 0, sizeof(int64_t), st));
        SubtaskArgs a;
        a.P = P;
        a.grp = B.grp;
        a.sub_ptr = B.sub_ptr;
        a.queue = qv;
        a.nqueue = nlocal;
        a.local_max = local_max;
        a.queue_head = (unsigned int *)(ctx->d_counters + 5);
        a.ancU = B.ancU;
        a.ancV = B.ancV;
        a.rdu = B.rdu;
        a.rdv = B.rdv;
        a.rb = B.rb;
        a.state = B.state;
        a.cycles = cycles;
        int blocks = std::max(1, std::min<int>(ctx->local_blocks, (nlocal + 3) / 4));
        launch_local_recover(ctx, c, a, blocks);
    }
    // Step 4, large subtasks: hash join + dependency rounds over their edges
    B.indeg = ctx->alloc<int32_t>(P + 1);
    B.mcnt = ctx->alloc<int32_t>(P + 1);
    if (nsub > nlocal) {
        int64_t entries = 2 * (int64_t)(c + 1) * (c + 1) * P;
        uint64_t cap = 1024;
        while (cap < 2 * (uint64_t)entries) cap <<= 1;
        Slot *tab = ctx->alloc<Slot>(cap);
        HIP_OK(hipMemsetAsync(tab, 0xff, sizeof(Slot) * cap, st));
        GSS_LAUNCH(k_join_build, dim3(grid_for(P, RB)), dim3(RB), 0, st, P, c, B.ancU, B.ancV, B.is_global, tab,
                   cap - 1);
        int64_t arc_cap = std::max<int64_t>(4 * P, 1 << 16);
        for (;;) {
            int2 *arcs = ctx->alloc<int2>(arc_cap);
            HIP_OK(hipMemsetAsync(B.indeg, 0, sizeof(int32_t) * (P + 1), st));
            HIP_OK(hipMemsetAsync(ctx->d_counters, 0, sizeof(int64_t) * 2, st));
            GSS_LAUNCH(k_join_probe, dim3(grid_for(P, RB)), dim3(RB), 0, st, P, B.rb, B.ancU, B.ancV, B.is_global,
                       tab, cap - 1, arcs, arc_cap, (unsigned long long *)ctx->d_counters, B.indeg, ctx->d_flags);
            read_counters(ctx, 1);
            int64_t A = ctx->h_counters[0];
            if (A > arc_cap) {
                ctx->free(arcs);
                arc_cap = A + A / 4 + 1024;
                continue;
            }
            res.arcs = A;
            HIP_OK(hipMemsetAsync(B.mcnt, 0, sizeof(int32_t) * (P + 1), st));
            GSS_LAUNCH(k_state_init, dim3(grid_for(P, RB)), dim3(RB), 0, st, P, B.indeg, B.is_global, B.state);
            if (A > 0)
                GSS_LAUNCH(k_resolve, dim3(1), dim3(1024), 0, st, A, arcs, B.indeg, B.state, B.mcnt,
                           ctx->d_counters + 1);
            read_counters(ctx, 2);
            res.rounds = A > 0 ? ctx->h_counters[1] : 0;
            ctx->free(arcs);
            break;
        }
        ctx->free(tab);
    }
    int64_t nthr2 = (P + CHUNK - 1) / CHUNK;
    B.ccnt = ctx->alloc<int32_t>(nthr2 + 1);
    GSS_LAUNCH(k_cand_count, dim3(grid_for(nthr2, RB)), dim3(RB), 0, st, P, B.state, B.ccnt);
    res.cand = scan_exclusive_i32(ctx, B.ccnt, nthr2, true);
    if (ctx->record && nsub > 0) trace_append(ctx, nsub, B.sub_ptr, feat, cycles, qv, nlocal);
    for (void *p : scratch) ctx->free(p);
    return res;
}

// threshold T such that {key >= T} holds at least `want` eligible edges (and not many more)
static uint64_t select_threshold(gss_ctx ctx, gss_tree t, const uint64_t *key, uint32_t *hist, bool hist_ready,
                                 int64_t want, int64_t eligible)
{
    hipStream_t st = ctx->stream;
    if (want >= eligible) return 1;  // every eligible key is >= 1
    const int shifts[6] = {51, 39, 27, 15, 3, 0};
    const int widths[6] = {12, 12, 12, 12, 12, 3};
    uint64_t pmask = 0, pval = 0;
    int64_t above = 0;
    const int64_t slack = std::max<int64_t>(1024, want / 16);
    for (int lv = 0; lv < 6; lv++) {
        if (lv > 0 || !hist_ready) {
            HIP_OK(hipMemsetAsync(hist, 0, sizeof(uint32_t) * SEL_BINS, st));
            GSS_LAUNCH(k_key_hist, dim3(std::min<int64_t>(grid_for(t->M, RB), 2048)), dim3(RB), 0, st, key,
                               t->M, shifts[lv], widths[lv], pmask, pval, hist);
        }
        GSS_LAUNCH(k_pick_bucket, dim3(1), dim3(1024), 0, st, hist, widths[lv], want - above,
                           ctx->d_counters);
        HIP_OK(hipGetLastError());
        read_counters(ctx, 3);
        int64_t d = ctx->h_counters[0], cum = ctx->h_counters[1], cnt = ctx->h_counters[2];
        if (d < 0) return 1;  // fewer than `want` keys: take everything
        uint64_t dmask = ((1ull << widths[lv]) - 1) << shifts[lv];
        pmask |= dmask;
        pval |= (uint64_t)d << shifts[lv];
        above += cum;
        if (above + cnt - want <= slack || lv == 5) return pval;  // lowest key of the bucket
    }
    return pval;
}

gss_status recover_impl(gss_ctx ctx, gss_tree t, const gss_params *prm, uint8_t *mask, int32_t *order,
                        double *stretch, gss_info *info)
{
    hipStream_t st = ctx->stream;
    const int32_t n = t->n;
    const int64_t M = t->M, m = t->m;
    const int32_t c = prm->beta;
    const int64_t K = prm->k_override >= 0 ? prm->k_override : (int64_t)std::floor(prm->alpha * (double)n);

    HIP_OK(hipMemsetAsync(mask, 0, (size_t)m, st));
    if (stretch) HIP_OK(hipMemsetAsync(stretch, 0, sizeof(double) * (size_t)m, st));
    if (prm->flags & GSS_F_MASK_TREE)
        GSS_LAUNCH(k_mask_tree, dim3(grid_for(n, RB)), dim3(RB), 0, st, t->tree_eid, n, mask);
    HIP_OK(hipMemsetAsync(ctx->d_flags, 0, sizeof(uint32_t), st));

    uint64_t *key = ctx->alloc<uint64_t>(M + 1);
    int32_t *lca = ctx->alloc<int32_t>(M + 1);
    uint8_t *bst = ctx->alloc<uint8_t>(M + 1);
    uint32_t *hist = ctx->alloc<uint32_t>(SEL_BINS);
    int32_t *lcacnt = ctx->alloc<int32_t>(n);
    HIP_OK(hipMemsetAsync(hist, 0, sizeof(uint32_t) * SEL_BINS, st));
    HIP_OK(hipMemsetAsync(lcacnt, 0, sizeof(int32_t) * n, st));
    if (M > 0)
        GSS_LAUNCH(k_edge_stretch, dim3(grid_for(M, RB)), dim3(RB), 0, st, M, t->off_id, t->off_u,
                           t->off_v, t->off_w, t->vrec, rmq_view(t), t->scale, c, key, lca, bst,
                           stretch, hist, lcacnt, ctx->d_flags);
    HIP_OK(hipGetLastError());
    int64_t init2[2] = {0, 0};
    memcpy(ctx->h_counters + 2, init2, sizeof init2);
    HIP_OK(hipMemcpyAsync(ctx->d_counters + 2, ctx->h_counters + 2, sizeof init2, hipMemcpyHostToDevice, st));
    GSS_LAUNCH(k_lca_stats, dim3(std::min<int64_t>(grid_for(n, RB), 1024)), dim3(RB), 0, st, lcacnt, n,
               ctx->d_counters + 2);
    read_counters(ctx, 4);
    int64_t nsub = ctx->h_counters[2], largest = ctx->h_counters[3];
    uint32_t f = read_flags(ctx);
    auto cleanup = [&]() {
        ctx->free(key);
        ctx->free(lca);
        ctx->free(bst);
        ctx->free(hist);
        ctx->free(lcacnt);
    };
    if (f & F_RANGE) {
        cleanup();
        throw gss_error{GSS_ERR_RANGE, "a stretch is not a finite double"};
    }

    int64_t nrec = 0, eligible = M, last_P = 0, last_arcs = 0, last_rounds = 0;
    int32_t passes = 0;
    bool hist_ready = true;
    while (nrec < K && eligible > 0) {
        int64_t need = K - nrec;
        int64_t want = std::min<int64_t>(eligible, need + need / 4 + 1024);
        PrefixBufs B;
        PrefixResult r;
        for (;;) {
            uint64_t T = select_threshold(ctx, t, key, hist, hist_ready, want, eligible);
            hist_ready = false;
            r = resolve_prefix(ctx, t, c, key, bst, lca, lcacnt, T, B, prm);
            if (r.cand >= need || r.P >= eligible) break;
            // not enough recovered edges in this prefix: a longer one is needed
            double ratio = (double)need / (double)std::max<int64_t>(r.cand, 1);
            int64_t next = (int64_t)((double)r.P * ratio * 1.15) + 1024;
            want = std::min<int64_t>(eligible, std::max<int64_t>(next, r.P + 1024));
            B.release(ctx);
        }
        int64_t take = std::min<int64_t>(r.cand, need);
        int64_t nthr2 = (r.P + CHUNK - 1) / CHUNK;
        GSS_LAUNCH(k_cand_write, dim3(grid_for(nthr2, RB)), dim3(RB), 0, st, r.P, B.state, B.ccnt, take,
                           B.rid, B.sj, order, nrec, mask, key);
        HIP_OK(hipGetLastError());
        B.release(ctx);
        last_P = r.P;
        last_arcs = r.arcs;
        last_rounds = r.rounds;
        nrec += take;
        eligible -= take;
        if (take > 0) passes++;
        if (take == 0) break;
    }
    ctx->sync();
    cleanup();
    if (info) {
        info->m = m;
        info->n_offtree = M;
        info->k = K;
        info->n_recovered = nrec;
        info->n_subtasks = nsub;
        info->largest_subtask = largest;
        info->prefix_len = last_P;
        info->n_arcs = last_arcs;
        info->passes = passes;
        info->rounds = (int32_t)last_rounds;
    }
    return nrec < K ? GSS_SHORT : GSS_OK;
}

void edge_lca_impl(gss_ctx ctx, gss_tree t, int32_t beta, int32_t *lca_out, int32_t *b_out)
{
    hipStream_t st = ctx->stream;
    const int64_t M = t->M, m = t->m;
    if (lca_out) {
        GSS_LAUNCH(k_fill_i32_r, dim3(grid_for(m, RB)), dim3(RB), 0, st, lca_out, m, -1);
    }
    if (b_out) HIP_OK(hipMemsetAsync(b_out, 0, sizeof(int32_t) * (size_t)m, st));
    uint64_t *key = ctx->alloc<uint64_t>(M + 1);
    int32_t *lca = ctx->alloc<int32_t>(M + 1);
    uint8_t *bst = ctx->alloc<uint8_t>(M + 1);
    uint32_t *hist = ctx->alloc<uint32_t>(SEL_BINS);
    HIP_OK(hipMemsetAsync(hist, 0, sizeof(uint32_t) * SEL_BINS, st));
    if (M > 0) {
        GSS_LAUNCH(k_edge_stretch, dim3(grid_for(M, RB)), dim3(RB), 0, st, M, t->off_id, t->off_u,
                           t->off_v, t->off_w, t->vrec, rmq_view(t), t->scale, beta, key, lca, bst,
                           (double *)nullptr, hist, (int32_t *)nullptr, ctx->d_flags);
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
