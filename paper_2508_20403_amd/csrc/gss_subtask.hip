// gss_subtask.hip -- LCA subtasks of the resolved prefix (paper: Lemmas "strictly similar
// edges share their LCA" and "contraposition", Alg. 1 Steps 3-4).
//
// The prefix edges, already in rank order, are grouped by LCA (stable, so each subtask
// keeps rank order).  Subtasks up to a size limit are drained by a persistent kernel: each
// wavefront pops the next subtask from a device work queue and runs the serial greedy of
// that subtask with wavefront ballots, 64 edges at a time:
//   * lanes hold consecutive edges of the subtask; each lane first tests its edge against
//     the candidates recovered in earlier chunks (their descriptors are kept in a
//     per-wavefront scratch that stays in cache);
//   * the unmarked lanes are then resolved in rank order: the lowest pending lane is a
//     candidate, its descriptor is broadcast, lanes after it test strict similarity and
//     the ballot of hits removes them.
// Subtasks of at most GSS_LANE_MAX edges (most of them on uniform graphs) are queued
// after the others and run one per lane: the lane walks its few edges in rank order and
// tests each against the earlier candidates of its subtask, so a wavefront finishes 64
// of them in the time one would take with the whole wavefront.
// Strict similarity is tested with ancestor chains: x is in the beta-ball of u iff
// anc_i(x) = anc_j(u) for some i + j <= beta; with depths known, for each i only
// j = depth(u) - depth(x) + i can match.  Larger subtasks go to the global hash-join path.
// Each wavefront records the cycles it spent on every subtask (the cost model's targets).
#include "gss_subtask.h"

namespace {

template <int C>
struct Desc {
    int32_t au[C + 1];  // u, parent(u), ...   (-1 above the root)
    int32_t av[C + 1];
    int32_t du, dv;     // depths of u and v
    int32_t beta;       // beta* of the edge
};

template <int C>
__device__ __forceinline__ void load_desc(Desc<C> &d, int64_t P, int32_t p, const int32_t *__restrict__ ancU,
                                          const int32_t *__restrict__ ancV, const int32_t *__restrict__ rdu,
                                          const int32_t *__restrict__ rdv, const uint8_t *__restrict__ rb)
{
#pragma unroll
    for (int i = 0; i <= C; i++) {
        d.au[i] = ancU[(int64_t)i * P + p];
        d.av[i] = ancV[(int64_t)i * P + p];
    }
    d.du = rdu[p];
    d.dv = rdv[p];
    d.beta = rb[p];
}

// is vertex x (chain ax, depth dx) within `beta` tree hops of vertex u (chain au, depth du)?
// anc_i(x) = anc_j(u) can hold only for j - i = du - dx; every (i, j) pair is tested with
// constant indices, so the chains stay in registers (a chain indexed by a computed j would
// have to live in private memory)
template <int C>
__device__ __forceinline__ bool in_ball(const int32_t *ax, int32_t dx, const int32_t *au, int32_t du, int beta)
{
    const int d = du - dx;
    bool hit = false;
#pragma unroll
    for (int i = 0; i <= C; i++)
#pragma unroll
        for (int j = 0; j <= C; j++)
            hit |= (j - i == d) & (i + j <= beta) & (ax[i] == au[j]) & (ax[i] >= 0);
    return hit;
}

// is edge t strictly similar to marker m under m's beta*?
template <int C>
__device__ __forceinline__ bool strictly_similar(const Desc<C> &t, const Desc<C> &m)
{
    const int b = m.beta;
    if (b == 0) return false;  // the balls are {u} and {v}: only the edge itself
    bool o1 = in_ball<C>(t.au, t.du, m.au, m.du, b) && in_ball<C>(t.av, t.dv, m.av, m.dv, b);
    bool o2 = in_ball<C>(t.au, t.du, m.av, m.dv, b) && in_ball<C>(t.av, t.dv, m.au, m.du, b);
    return o1 || o2;
}

// field-by-field copies to and from the candidate scratch (a whole-struct copy of a
// global Desc went through private memory)
template <int C>
__device__ __forceinline__ void read_desc(Desc<C> &d, const Desc<C> *__restrict__ src)
{
#pragma unroll
    for (int i = 0; i <= C; i++) {
        d.au[i] = src->au[i];
        d.av[i] = src->av[i];
    }
    d.du = src->du;
    d.dv = src->dv;
    d.beta = src->beta;
}

template <int C>
__device__ __forceinline__ void write_desc(Desc<C> *__restrict__ dst, const Desc<C> &d)
{
#pragma unroll
    for (int i = 0; i <= C; i++) {
        dst->au[i] = d.au[i];
        dst->av[i] = d.av[i];
    }
    dst->du = d.du;
    dst->dv = d.dv;
    dst->beta = d.beta;
}

template <int C>
__device__ __forceinline__ Desc<C> shfl_desc(const Desc<C> &d, int src)
{
    Desc<C> r;
#pragma unroll
    for (int i = 0; i <= C; i++) {
        r.au[i] = __shfl(d.au[i], src, GSS_WAVE);
        r.av[i] = __shfl(d.av[i], src, GSS_WAVE);
    }
    r.du = __shfl(d.du, src, GSS_WAVE);
    r.dv = __shfl(d.dv, src, GSS_WAVE);
    r.beta = __shfl(d.beta, src, GSS_WAVE);
    return r;
}

// serial greedy of one small subtask [g0, g1) by one lane: each edge is tested against
// the candidates found before it (their descriptors are loaded again: they were just
// read by this lane and sit in the cache)
template <int C>
__device__ __forceinline__ void lane_subtask(const SubtaskArgs &a, int32_t g0, int32_t g1)
{
    uint32_t cand = 0;
    for (int32_t j = 0; j < g1 - g0; j++) {
        const int32_t pj = a.grp[g0 + j];
        Desc<C> dj;
        load_desc<C>(dj, a.P, pj, a.ancU, a.ancV, a.rdu, a.rdv, a.rb);
        bool marked = false;
        for (int32_t i = 0; i < j && !marked; i++) {
            if (!((cand >> i) & 1u)) continue;
            Desc<C> di;
            load_desc<C>(di, a.P, a.grp[g0 + i], a.ancU, a.ancV, a.rdu, a.rdv, a.rb);
            marked = strictly_similar<C>(dj, di);
        }
        if (!marked) cand |= 1u << j;
        a.state[pj] = marked ? ST_MARK_ : ST_CAND_;
    }
}

// greedy of one wavefront-sized subtask (queue entry qi) by one wavefront
template <int C>
__device__ __forceinline__ void wave_subtask(const SubtaskArgs &a, int32_t qi, Desc<C> *cand)
{
    const int lane = lane_id();
    const int32_t s = a.queue[qi];
    const uint64_t t0 = clock64();
    const int32_t g0 = a.sub_ptr[s], g1 = a.sub_ptr[s + 1];
    int32_t ncand = 0;
    for (int32_t c0 = g0; c0 < g1; c0 += GSS_WAVE) {
        const int32_t gi = c0 + lane;
        const bool valid = gi < g1;
        const int32_t p = valid ? a.grp[gi] : 0;
        Desc<C> me;  // loaded for every lane (p = 0 on idle lanes, any valid rank)
        load_desc<C>(me, a.P, p, a.ancU, a.ancV, a.rdu, a.rdv, a.rb);
        // against candidates of earlier chunks
        bool marked = false;
        for (int32_t k = 0; k < ncand; k++) {
            Desc<C> m;
            read_desc<C>(m, cand + k);
            marked |= valid && strictly_similar<C>(me, m);
        }
        // in-chunk greedy in rank order
        uint64_t pending = __ballot(valid && !marked);
        uint64_t recovered = 0;
        while (pending) {
            const int i = __ffsll((long long)pending) - 1;
            Desc<C> m = shfl_desc<C>(me, i);
            const bool hit = valid && lane > i && strictly_similar<C>(me, m);
            const uint64_t hits = __ballot(hit);
            recovered |= 1ull << i;
            pending &= ~((1ull << i) | hits);
        }
        const bool is_cand = (recovered >> lane) & 1ull;
        if (valid) a.state[p] = is_cand ? ST_CAND_ : ST_MARK_;
        // append this chunk's candidates (rank order) to the candidate list
        const int before = __popcll(recovered & lanemask_lt());
        if (is_cand && ncand + before < a.local_max) write_desc<C>(cand + ncand + before, me);
        ncand += __popcll(recovered);
        __threadfence_block();
    }
    const uint64_t t1 = clock64();
    if (lane == 0 && a.cycles) a.cycles[s] = t1 - t0;
}

// persistent kernel: first the larger subtasks, one wavefront each, then the small ones,
// one per lane.  The queue is ordered by predicted cost, largest first.  Its first
// lpt_rounds * W entries (W = wavefronts of the grid) are dealt to the wavefronts in
// boustrophedon order before any is pulled: round r gives entry r W + w to wavefront w
// on even rounds and entry (r + 1) W - 1 - w on odd ones, so every wavefront starts with
// a balanced share of the heaviest subtasks (longest-processing-time bins) without
// touching the shared head; the rest is pulled from the head, `chunk` entries at a time.
template <int C>
__global__ __launch_bounds__(256) void k_local_recover(SubtaskArgs a)
{
    // descriptors of the candidates recovered so far in the current subtask, per wavefront,
    // in global scratch: written by the lanes, read back with wave-uniform vector loads
    // that stay in this CU's caches
    const int lane = lane_id();
    const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / GSS_WAVE;
    const int64_t W = (int64_t)gridDim.x * blockDim.x / GSS_WAVE;
    Desc<C> *cand = (Desc<C> *)a.cand_scratch + gw * a.local_max;
    for (int r = 0; r < a.lpt_rounds; r++) {
        const int64_t qi = (r & 1) ? (int64_t)(r + 1) * W - 1 - gw : (int64_t)r * W + gw;
        if (qi < a.nbig) wave_subtask<C>(a, (int32_t)qi, cand);
    }
    const int64_t dealt = (int64_t)a.lpt_rounds * W;
    // queue entries are taken `chunk` at a time, so the shared head sees one atomic per
    // chunk rather than one per subtask
    for (;;) {
        int64_t q0 = 0;
        if (lane == 0) q0 = dealt + (int64_t)atomicAdd(&a.queue_head[0], (unsigned)a.chunk);
        q0 = __shfl(q0, 0, GSS_WAVE);
        if (q0 >= a.nbig) break;
        const int64_t q1 = (q0 + a.chunk < a.nbig) ? q0 + a.chunk : a.nbig;
        for (int64_t qi = q0; qi < q1; qi++) wave_subtask<C>(a, (int32_t)qi, cand);
    }
    // small subtasks: 64 queue entries per take, one per lane
    for (;;) {
        int32_t q0 = 0;
        if (lane == 0) q0 = a.nbig + (int32_t)atomicAdd(&a.queue_head[1], (unsigned)GSS_WAVE);
        q0 = __shfl(q0, 0, GSS_WAVE);
        if (q0 >= a.nqueue) break;
        const int32_t qi = q0 + lane;
        if (qi < a.nqueue) {
            const int32_t s = a.queue[qi];
            const uint64_t t0 = clock64();
            lane_subtask<C>(a, a.sub_ptr[s], a.sub_ptr[s + 1]);
            const uint64_t t1 = clock64();
            if (a.cycles) a.cycles[s] = t1 - t0;
        }
    }
}

}  // namespace

size_t local_desc_bytes(int C)
{
    switch (C) {
#define CASE(k) \
    case k: return sizeof(Desc<k>);
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: throw gss_error{GSS_ERR_ARG, "beta out of range"};
    }
}

void launch_local_recover(gss_ctx ctx, int C, const SubtaskArgs &a, int blocks)
{
    hipStream_t st = ctx->stream;
    switch (C) {
#define CASE(k) \
    case k: GSS_LAUNCH(k_local_recover<k>, dim3(blocks), dim3(256), 0, st, a); break;
        CASE(0) CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: throw gss_error{GSS_ERR_ARG, "beta out of range"};
    }
    HIP_OK(hipGetLastError());
}

// ------------------------------------------------------------------------------------
// grouping helpers
// ------------------------------------------------------------------------------------
// subtask boundaries of the LCA-grouped list: head flag where the LCA changes
__global__ void k_group_heads(int64_t P, const uint64_t *__restrict__ glca, int32_t *__restrict__ head)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) head[i] = (i == 0 || glca[i] != glca[i - 1]) ? 1 : 0;
}

// sub_ptr[id] = start of subtask id (head flags scanned exclusively give the ids)
// sub_ptr[id] = start of subtask id (head flags scanned exclusively give the ids), and
// sub_ptr[nsub] = P from the last position
__global__ void k_group_ptr(int64_t P, const uint64_t *__restrict__ glca, const int32_t *__restrict__ hid,
                            int32_t *__restrict__ sub_ptr, int32_t *__restrict__ sub_lca)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P) return;
    const bool head = i == 0 || glca[i] != glca[i - 1];
    if (head) {
        sub_ptr[hid[i]] = (int32_t)i;
        sub_lca[hid[i]] = (int32_t)glca[i];
    }
    if (i == P - 1) sub_ptr[hid[i] + (head ? 1 : 0)] = (int32_t)P;
}

// per subtask: queue key (descending cost first) and the local/global split.  The
// subtask count nsub is read on the device; the queue has cap >= nsub slots and the ones
// past nsub get the largest key, so a stable ascending sort leaves them last.  With
// cost_bits = 0 (the edge-count order) the key is dense: class * (local_max + 1) +
// (local_max - size), sizes of the join's subtasks clamped to local_max (their order is
// never used), so small limits give one-byte keys.
__global__ __launch_bounds__(256) void k_subtask_keys(const int64_t *__restrict__ nsubp, int32_t cap,
                                                      const int32_t *__restrict__ sub_ptr,
                                                      int32_t local_max, const float *__restrict__ pred,
                                                      int cost_bits, uint64_t *__restrict__ qkey,
                                                      int32_t *__restrict__ qval,
                                                      int32_t *__restrict__ is_local, int32_t *__restrict__ nlocal,
                                                      int32_t *__restrict__ nsmall,
                                                      unsigned long long *__restrict__ nglobal_edges)
{
    __shared__ unsigned long long s_ge[256 / GSS_WAVE];
    __shared__ int32_t s_nl[256 / GSS_WAVE], s_ns[256 / GSS_WAVE];
    const int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t nsub = (int32_t)*nsubp;
    int32_t size = 0;
    if (s < nsub) size = sub_ptr[s + 1] - sub_ptr[s];
    const bool loc = s < nsub && size <= local_max;
    const bool small = loc && size <= GSS_LANE_MAX;
    if (s < nsub) {
        is_local[s] = loc ? 1 : 0;
        uint64_t cost;
        if (pred) cost = (uint64_t)__float_as_uint(fmaxf(pred[s], 0.f));  // non-negative floats order as ints
        else cost = (uint64_t)size;
        // ascending sort of this key = queued subtasks for wavefronts, then those for
        // lanes, each by cost descending, then id (a stable sort of ids in order), then
        // the join's; cost < 2^cost_bits
        const uint64_t cls = loc ? (small ? 1 : 0) : 2;
        if (cost_bits == 0) {
            const uint64_t L = (uint64_t)local_max, c = cost < L ? cost : L;
            qkey[s] = cls * (L + 1) + (L - c);
        } else {
            const uint64_t cmask = ((uint64_t)1 << cost_bits) - 1;
            qkey[s] = (cls << cost_bits) | ((~cost) & cmask);
        }
        qval[s] = s;
    } else if (s < cap) {
        qkey[s] = cost_bits == 0 ? 3 * ((uint64_t)local_max + 1) - 1
                                 : ((uint64_t)2 << cost_bits) | (((uint64_t)1 << cost_bits) - 1);
        qval[s] = s;
    }
    // edges on the join path, queued and small subtasks: one atomic per workgroup each
    unsigned long long ge = (s < nsub && !loc) ? (unsigned long long)size : 0ull;
    int32_t nl = loc ? 1 : 0, ns = small ? 1 : 0;
    for (int d = 32; d > 0; d >>= 1) {
        ge += __shfl_xor(ge, d, GSS_WAVE);
        nl += __shfl_xor(nl, d, GSS_WAVE);
        ns += __shfl_xor(ns, d, GSS_WAVE);
    }
    if (lane_id() == 0) {
        s_ge[threadIdx.x / GSS_WAVE] = ge;
        s_nl[threadIdx.x / GSS_WAVE] = nl;
        s_ns[threadIdx.x / GSS_WAVE] = ns;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < 256 / GSS_WAVE; w++) {
            ge += s_ge[w];
            nl += s_nl[w];
            ns += s_ns[w];
        }
        if (ge) atomicAdd(nglobal_edges, ge);
        if (nl) atomicAdd(nlocal, nl);
        if (ns) atomicAdd(nsmall, ns);
    }
}

// global-path flag per rank (edges of subtasks above the local limit)
// Ranks of the edges in subtasks on the join path, in grouped order: a flag per grouped
// position (its subtask is not on the work queue), a scan, and a write pass.  The
// subtask of position g is hid[g] (heads scanned exclusively) less one unless g is a head.
__device__ __forceinline__ bool on_join_path(int64_t g, const uint64_t *__restrict__ glca,
                                             const int32_t *__restrict__ hid, const int32_t *__restrict__ is_local)
{
    const bool head = g == 0 || glca[g] != glca[g - 1];
    return !is_local[hid[g] - (head ? 0 : 1)];
}
__global__ void k_join_flags(int64_t P, const uint64_t *__restrict__ glca, const int32_t *__restrict__ hid,
                             const int32_t *__restrict__ is_local, int32_t *__restrict__ flag)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < P) flag[g] = on_join_path(g, glca, hid, is_local) ? 1 : 0;
}
__global__ void k_join_write(int64_t P, const uint64_t *__restrict__ glca, const int32_t *__restrict__ hid,
                             const int32_t *__restrict__ is_local, const int32_t *__restrict__ pos,
                             const int32_t *__restrict__ grp, int32_t *__restrict__ glist)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < P && on_join_path(g, glca, hid, is_local)) glist[pos[g]] = grp[g];
}

// 12 features per subtask for the cost model.  They derive from integer sums over the
// subtask's edges (tree-path lengths below the LCA, beta*, endpoint tree degrees), which
// are exact and independent of the summation order.  Only queued subtasks (at most
// local_max edges) are scheduled by cost, so larger ones, which go to the join, get zero
// rows and no wave ever walks a hub subtask.
struct FeatSums {
    unsigned long long path, beta, nb0, deg;
    int32_t max_path, max_deg;
};

__device__ __forceinline__ void feat_edge(int32_t p, int32_t lca_depth, const int32_t *__restrict__ rdu,
                                          const int32_t *__restrict__ rdv, const uint8_t *__restrict__ rb,
                                          const int32_t *__restrict__ ru, const int32_t *__restrict__ rv,
                                          const VRec *__restrict__ vrec, FeatSums &a)
{
    const int32_t path = rdu[p] - lca_depth + rdv[p] - lca_depth;
    const int32_t b = rb[p];
    const VRec xu = vrec[ru[p]], xv = vrec[rv[p]];
    const int32_t deg = xu.pad + (xu.parent >= 0) + xv.pad + (xv.parent >= 0);  // deg_T(u) + deg_T(v)
    a.path += (unsigned long long)path;
    a.max_path = max(a.max_path, path);
    a.beta += (unsigned long long)b;
    a.nb0 += b == 0 ? 1ull : 0ull;
    a.deg += (unsigned long long)deg;
    a.max_deg = max(a.max_deg, deg);
}

__device__ __forceinline__ void feat_wave_reduce(FeatSums &a)
{
    for (int d = GSS_WAVE / 2; d > 0; d >>= 1) {
        a.path += __shfl_xor(a.path, d, GSS_WAVE);
        a.beta += __shfl_xor(a.beta, d, GSS_WAVE);
        a.nb0 += __shfl_xor(a.nb0, d, GSS_WAVE);
        a.deg += __shfl_xor(a.deg, d, GSS_WAVE);
        a.max_path = max(a.max_path, __shfl_xor(a.max_path, d, GSS_WAVE));
        a.max_deg = max(a.max_deg, __shfl_xor(a.max_deg, d, GSS_WAVE));
    }
}

__device__ __forceinline__ void feat_write(float *__restrict__ f, int32_t size, const FeatSums &a, const VRec &rl,
                                           int64_t P)
{
    const float S = (float)size;
    f[0] = log2f(1.f + S);
    f[1] = (float)((double)a.path / size);  // mean tree-path length below the LCA
    f[2] = (float)a.max_path;
    f[3] = (float)((double)a.beta / size);  // mean beta*
    f[4] = (float)((double)a.nb0 / size);   // share of edges with beta* = 0
    f[5] = (float)((double)a.deg / size);   // mean endpoint tree-degree sum
    f[6] = (float)a.max_deg;
    f[7] = log2f(1.f + (float)(rl.pad + (rl.parent >= 0)));  // tree degree of the LCA
    f[8] = log2f(1.f + (float)rl.depth);    // depth of the LCA
    f[9] = S / fmaxf((float)P, 1.f);        // share of the resolved prefix
    f[10] = log2f(1.f + (float)a.path);     // total tree-path length
    f[11] = log2f(1.f + S * S);
}

// one wave per subtask (grid-stride; the subtask count is read on the device)
__global__ __launch_bounds__(256) void k_subtask_features(const int64_t *__restrict__ nsubp,
                                                          const int32_t *__restrict__ sub_ptr,
                                                          const int32_t *__restrict__ sub_lca,
                                                          const int32_t *__restrict__ grp,
                                                          const int32_t *__restrict__ rdu,
                                                          const int32_t *__restrict__ rdv,
                                                          const uint8_t *__restrict__ rb,
                                                          const int32_t *__restrict__ ru,
                                                          const int32_t *__restrict__ rv,
                                                          const VRec *__restrict__ vrec, int64_t P,
                                                          int32_t local_max, float *__restrict__ feat)
{
    const int lane = lane_id();
    const int32_t nsub = (int32_t)*nsubp;
    const int32_t waves = (int32_t)(gridDim.x * blockDim.x / GSS_WAVE);
    for (int32_t s = (int32_t)((blockIdx.x * blockDim.x + threadIdx.x) / GSS_WAVE); s < nsub; s += waves) {
        const int32_t g0 = sub_ptr[s], g1 = sub_ptr[s + 1];
        if (g1 - g0 > local_max) {
            if (lane < GSS_NFEAT) feat[(int64_t)s * GSS_NFEAT + lane] = 0.f;
            continue;
        }
        const VRec rl = vrec[sub_lca[s]];
        FeatSums a = {0, 0, 0, 0, 0, 0};
        for (int32_t g = g0 + lane; g < g1; g += GSS_WAVE)
            feat_edge(grp[g], rl.depth, rdu, rdv, rb, ru, rv, vrec, a);
        feat_wave_reduce(a);
        if (lane == 0) feat_write(feat + (int64_t)s * GSS_NFEAT, g1 - g0, a, rl, P);
    }
}

void launch_grouping_kernels(gss_ctx ctx, int64_t P, const uint64_t *glca, int32_t *head)
{
    GSS_LAUNCH(k_group_heads, dim3(grid_for(P, 256)), dim3(256), 0, ctx->stream, P, glca, head);
}

void launch_group_ptr(gss_ctx ctx, int64_t P, const uint64_t *glca, const int32_t *hid, int32_t *sub_ptr,
                      int32_t *sub_lca)
{
    GSS_LAUNCH(k_group_ptr, dim3(grid_for(P, 256)), dim3(256), 0, ctx->stream, P, glca, hid, sub_ptr, sub_lca);
}

void launch_subtask_keys(gss_ctx ctx, const int64_t *nsubp, int32_t cap, const int32_t *sub_ptr, int32_t local_max,
                         const float *pred, int cost_bits, uint64_t *qkey, int32_t *qval, int32_t *is_local,
                         int32_t *nlocal, int32_t *nsmall, unsigned long long *nglobal_edges)
{
    GSS_LAUNCH(k_subtask_keys, dim3(grid_for(cap, 256)), dim3(256), 0, ctx->stream, nsubp, cap, sub_ptr, local_max,
               pred, cost_bits, qkey, qval, is_local, nlocal, nsmall, nglobal_edges);
}

void launch_join_list(gss_ctx ctx, int64_t P, const uint64_t *glca, const int32_t *hid, const int32_t *is_local,
                      const int32_t *grp, int32_t *glist)
{
    if (P <= 0) return;
    int32_t *flag = ctx->alloc<int32_t>(P + 1);
    GSS_LAUNCH_B(13 * P, k_join_flags, dim3(grid_for(P, 256)), dim3(256), 0, ctx->stream, P, glca, hid, is_local, flag);
    scan_exclusive_i32_dev(ctx, flag, P, ctx->d_counters + 7);
    GSS_LAUNCH_B(21 * P, k_join_write, dim3(grid_for(P, 256)), dim3(256), 0, ctx->stream, P, glca, hid, is_local,
                 flag, grp, glist);
    ctx->free(flag);
}

void launch_subtask_features(gss_ctx ctx, const int64_t *nsubp, int32_t cap, const int32_t *sub_ptr,
                             const int32_t *sub_lca, const int32_t *grp, const int32_t *rdu, const int32_t *rdv,
                             const uint8_t *rb, const int32_t *ru, const int32_t *rv, const VRec *vrec, int64_t P,
                             int32_t local_max, float *feat)
{
    const unsigned blocks = std::min<unsigned>(grid_for((int64_t)cap * GSS_WAVE, 256), 4096);
    GSS_LAUNCH(k_subtask_features, dim3(blocks), dim3(256), 0, ctx->stream, nsubp, sub_ptr, sub_lca, grp, rdu, rdv,
               rb, ru, rv, vrec, P, local_max, feat);
}
