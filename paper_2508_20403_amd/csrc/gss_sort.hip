// gss_sort.hip -- sample sort of (64-bit key, 32-bit value) pairs for the short sorts of
// the recovery: a prefix of the criticality order (Alg. 1 Step 2), its grouping by LCA
// (Step 3) and the subtask work queue.  These sorts hold a few hundred thousand pairs,
// too few for a radix sort to reach bandwidth: every radix pass is a launch bounded by
// its latency.  A sample sort needs five launches whatever the key width:
//   1. a stratified sample of the pairs is ranked by counting (every sample compared
//      with every other, spread over the grid) and nb - 1 evenly spaced ranks become
//      the splitters,
//   2. every tile counts its pairs per bucket (binary search over the splitters in LDS)
//      into a bucket-major count matrix,
//   3. an exclusive scan of that matrix gives every (bucket, tile) its output offset and
//      every bucket its start,
//   4. every tile scatters its pairs into their buckets,
//   5. one workgroup per bucket sorts it in registers when it holds at most eight times
//      the workgroup size, otherwise in place in global memory.
// Buckets hold about SS_MEAN pairs: the last launch takes as long as its largest bucket,
// whose bitonic network runs on one compute unit, so buckets are kept small and many.
// Pairs are ordered by (key, value); the callers' values are distinct, so the order is
// total and the result does not depend on the order in which a bucket is filled.
// The sorting network is the bitonic one in its one-direction form (the first step of
// every merge compares mirrored positions, so every comparison puts the smaller pair at
// the lower position).  In registers, thread t of the SS_BT holds positions r * SS_BT + t:
// partners closer than a wavefront are exchanged by lane shuffles, partners SS_BT or more
// apart sit in the same thread, and only the remaining steps go through LDS.
#include <algorithm>

#include "gss_impl.h"

#define SS_SAMPLES 4096  // largest sample (power of two)
#define SS_TT 256        // threads of the counting and scatter kernels
#define SS_TI 4          // pairs per thread there
#define SS_TILE (SS_TT * SS_TI)
#define SS_MAXB 2048     // largest bucket count
#ifndef SS_MEAN
#define SS_MEAN 384      // pairs per bucket on average
#endif
#ifndef SS_LBT
#define SS_LBT 9         // log2 of the bucket kernel's threads
#endif
#define SS_BT (1 << SS_LBT)
#define SS_CAP (SS_BT * 8)  // largest bucket sorted in registers (eight pairs per thread)

__device__ __forceinline__ bool ss_less(uint64_t ak, uint32_t av, uint64_t bk, uint32_t bv)
{
    return ak < bk || (ak == bk && av < bv);
}

// One-direction bitonic sort of keys/values [0, S) by all threads of the workgroup.
// K and V may be LDS or global memory (the same workgroup only: the barriers order the
// steps).  N2 = 2^lgN is the power of two at or above S; positions >= S act as +infinity
// and are never touched, since every comparison moves the smaller pair to the lower
// position.  Step (k = 2^lk, j = 2^lj): pair i joins a = (i >> lj) << (lj + 1) | (i & (j-1))
// with its mirror in the k-block (first step of a merge, lj = lk - 1) or with a + j.
template <typename KP, typename VP>
__device__ void ss_network(KP K, VP V, int S)
{
    int lgN = 0;
    while ((1 << lgN) < S) lgN++;
    const int half = (1 << lgN) >> 1;
    for (int lk = 1; lk <= lgN; lk++) {
        for (int lj = lk - 1; lj >= 0; lj--) {
            const int j = 1 << lj;
            for (int i = threadIdx.x; i < half; i += blockDim.x) {
                const int lo = i & (j - 1);
                const int a = ((i >> lj) << (lj + 1)) + lo;
                const int b = (lj == lk - 1) ? a - lo + (2 * j - 1 - lo) : a + j;
                if (b >= S) continue;
                const uint64_t ka = K[a], kb = K[b];
                const uint32_t va = V[a], vb = V[b];
                if (ss_less(kb, vb, ka, va)) {
                    K[a] = kb;
                    K[b] = ka;
                    V[a] = vb;
                    V[b] = va;
                }
            }
            __syncthreads();
        }
    }
}

// compare-exchange with a partner, without branches: the lower position keeps the smaller
// pair, the upper one the larger (equal pairs, the padding, need no exchange)
__device__ __forceinline__ void ss_keep(uint64_t &k, uint32_t &v, uint64_t pk, uint32_t pv, bool lower)
{
    const bool take = ss_less(pk, pv, k, v) == lower;
    k = take ? pk : k;
    v = take ? pv : v;
}

// the value of lane (lane ^ M) of the wavefront, M a constant below 64: quad permutes and
// the row mirrors of DPP where they express it, the bitmask swizzle within 32 lanes
// (source lane (lane & 31) ^ M) for the other masks below 32, a permute beyond
template <int M>
__device__ __forceinline__ uint32_t ss_lane_xor(uint32_t x)
{
    if constexpr (M == 1) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, true);  // [1,0,3,2]
    else if constexpr (M == 2) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, true);  // [2,3,0,1]
    else if constexpr (M == 3) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x1B, 0xF, 0xF, true);  // [3,2,1,0]
    else if constexpr (M == 7) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x141, 0xF, 0xF, true);  // half-row mirror
    else if constexpr (M == 15) return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x140, 0xF, 0xF, true);  // row mirror
    else if constexpr (M < 32) return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x1F | (M << 10));
    else return (uint32_t)__shfl_xor((int)x, M, GSS_WAVE);
}

// one step of the network: partner = position ^ M
template <int E, int M>
__device__ __forceinline__ void ss_step(uint64_t (&k)[E], uint32_t (&v)[E], uint64_t *ek, uint32_t *ev)
{
    const int t = threadIdx.x;
    if constexpr (M < GSS_WAVE) {  // partner in the same wavefront
        const bool lower = (t ^ M) > t;
#pragma unroll
        for (int r = 0; r < E; r++) {
            const uint32_t lo = ss_lane_xor<M>((uint32_t)k[r]), hi = ss_lane_xor<M>((uint32_t)(k[r] >> 32));
            const uint32_t pv = ss_lane_xor<M>(v[r]);
            ss_keep(k[r], v[r], ((uint64_t)hi << 32) | lo, pv, lower);
        }
    } else if constexpr ((M & (SS_BT - 1)) == 0) {  // same thread: registers r and r ^ (M / SS_BT)
        constexpr int RM = M >> SS_LBT;
#pragma unroll
        for (int r = 0; r < E; r++) {
            if (r & RM) continue;
            const int q = r ^ RM;  // q > r: position q * SS_BT + t is the higher one
            const bool lt = ss_less(k[q], v[q], k[r], v[r]);
            const uint64_t a = k[r], b = k[q];
            const uint32_t av = v[r], bv = v[q];
            k[r] = lt ? b : a;
            v[r] = lt ? bv : av;
            k[q] = lt ? a : b;
            v[q] = lt ? av : bv;
        }
    } else {  // through LDS
#pragma unroll
        for (int r = 0; r < E; r++) {
            ek[r * SS_BT + t] = k[r];
            ev[r * SS_BT + t] = v[r];
        }
        __syncthreads();
        uint64_t pk[E];
        uint32_t pv[E];
#pragma unroll
        for (int r = 0; r < E; r++) {
            const int q = (r * SS_BT + t) ^ M;
            pk[r] = ek[q];
            pv[r] = ev[q];
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < E; r++) ss_keep(k[r], v[r], pk[r], pv[r], (r * SS_BT + t) < ((r * SS_BT + t) ^ M));
    }
}

// the steps (LK, LJ) of the one-direction bitonic network in order, unrolled at compile
// time: merge size 2^LK from 1 to LG, distance 2^LJ from LK - 1 down to 0; the first
// step of every merge compares mirrored positions
template <int E, int LG, int LK, int LJ>
__device__ __forceinline__ void ss_steps(uint64_t (&k)[E], uint32_t (&v)[E], uint64_t *ek, uint32_t *ev)
{
    if constexpr (LK <= LG) {
        ss_step<E, (LJ == LK - 1) ? (2 << LJ) - 1 : (1 << LJ)>(k, v, ek, ev);
        if constexpr (LJ > 0) ss_steps<E, LG, LK, LJ - 1>(k, v, ek, ev);
        else ss_steps<E, LG, LK + 1, LK>(k, v, ek, ev);
    }
}

// Sorts the SS_BT * E pairs held in registers by a workgroup of SS_BT threads (thread t
// holds positions r * SS_BT + t).  ek/ev: LDS of SS_BT * E entries for the steps whose
// partners are in other wavefronts.
template <int E>
__device__ void ss_reg_sort(uint64_t (&k)[E], uint32_t (&v)[E], uint64_t *ek, uint32_t *ev)
{
    constexpr int LGE = E == 1 ? 0 : E == 2 ? 1 : E == 4 ? 2 : 3;
    ss_steps<E, SS_LBT + LGE, 1, 0>(k, v, ek, ev);
}

// loads S <= SS_BT E pairs (padded with the largest pair), sorts them in registers and
// stores them back
template <int E>
__device__ void ss_sort_run(uint64_t *__restrict__ k, int32_t *__restrict__ v, int S, uint64_t *ek, uint32_t *ev)
{
    uint64_t kk[E];
    uint32_t vv[E];
#pragma unroll
    for (int r = 0; r < E; r++) {
        const int p = r * SS_BT + (int)threadIdx.x;
        kk[r] = p < S ? k[p] : ~0ull;
        vv[r] = p < S ? (uint32_t)v[p] : ~0u;
    }
    ss_reg_sort<E>(kk, vv, ek, ev);
#pragma unroll
    for (int r = 0; r < E; r++) {
        const int p = r * SS_BT + (int)threadIdx.x;
        if (p < S) {
            k[p] = kk[r];
            v[p] = (int32_t)vv[r];
        }
    }
}

// bucket of (k, v): the number of splitters at or below it (splitters ascending)
__device__ __forceinline__ int ss_bucket(uint64_t k, uint32_t v, const uint64_t *spk, const uint32_t *spv,
                                         int nsp)
{
    int lo = 0, hi = nsp;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ss_less(k, v, spk[mid], spv[mid])) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// 1. the splitters: ns strata of equal length give one sample each, the pair at a hashed
// offset in the stratum.  Every block gathers all samples into LDS; SS_RT threads count
// the rank of one sample among them (each compares it with every SS_RT-th sample, then
// the counts are summed across those lanes).  Samples are distinct pairs, so the ranks
// are a permutation, and the sample of rank (b + 1) ns / nb becomes splitter b
// (b < nb - 1): no sort, and every step runs on the whole grid.
#define SS_RT 32   // threads ranking one sample (consecutive lanes)
#define SS_RB 256  // threads of the ranking kernel

// ns is a power of two (2^lgns <= n): stratum i is [i n / ns, (i + 1) n / ns), and the
// hashed offset in it is taken by a multiply-high (no 64-bit division on the device)
__device__ __forceinline__ int64_t ss_sample_pos(int i, int64_t n, int lgns)
{
    const int64_t lo = ((int64_t)i * n) >> lgns, hi = ((int64_t)(i + 1) * n) >> lgns;
    const uint64_t h = mix32(0x9E3779B9u * (uint32_t)(i + 1));
    const int64_t p = lo + (int64_t)((h * (uint64_t)(hi - lo)) >> 32);
    return p < n ? p : n - 1;
}

__global__ __launch_bounds__(SS_RB) void k_ss_splitters(const uint64_t *__restrict__ k, const int32_t *__restrict__ v,
                                                       int64_t n, int lgns, int nb, uint64_t *__restrict__ spk,
                                                       uint32_t *__restrict__ spv)
{
    __shared__ uint64_t sk[SS_SAMPLES];
    __shared__ uint32_t sv[SS_SAMPLES];
    const int ns = 1 << lgns;
    // the gathers of a thread are independent: all in flight before the LDS stores
#pragma unroll
    for (int r = 0; r < SS_SAMPLES / SS_RB; r++) {
        const int i = r * SS_RB + (int)threadIdx.x;
        if (i < ns) {
            const int64_t p = ss_sample_pos(i, n, lgns);
            sk[i] = k[p];
            sv[i] = (uint32_t)v[p];
        }
    }
    __syncthreads();
    const int t = blockIdx.x * SS_RB + (int)threadIdx.x;
    const int i = t / SS_RT, part = t % SS_RT;
    const bool valid = i < ns;
    const uint64_t mk = valid ? sk[i] : 0;
    const uint32_t mv = valid ? sv[i] : 0;
    int cnt = 0;
    if (valid)
        for (int j = part; j < ns; j += SS_RT) cnt += ss_less(sk[j], sv[j], mk, mv) ? 1 : 0;
#pragma unroll
    for (int d = SS_RT / 2; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d, GSS_WAVE);
    if (valid && part == 0) {
        // the one b + 1 that could select rank cnt: the least q with q ns / nb >= cnt
        const int64_t q = ((int64_t)cnt * nb + ns - 1) / ns;
        if (q >= 1 && q <= nb - 1 && (q * ns) / nb == cnt) {
            spk[q - 1] = mk;
            spv[q - 1] = mv;
        }
    }
}

__device__ __forceinline__ void ss_load_splitters(const uint64_t *__restrict__ spk, const uint32_t *__restrict__ spv,
                                                  int nsp, uint64_t *sk, uint32_t *sv)
{
    for (int i = threadIdx.x; i < nsp; i += blockDim.x) {
        sk[i] = spk[i];
        sv[i] = spv[i];
    }
}

// 2. per tile and bucket, bucket-major: hist[b * ntiles + tile]
__global__ __launch_bounds__(SS_TT) void k_ss_count(const uint64_t *__restrict__ k, const int32_t *__restrict__ v,
                                                   int64_t n, int nb, const uint64_t *__restrict__ spk,
                                                   const uint32_t *__restrict__ spv, int32_t *__restrict__ hist)
{
    __shared__ uint64_t sk[SS_MAXB];
    __shared__ uint32_t sv[SS_MAXB];
    __shared__ int32_t cnt[SS_MAXB];
    ss_load_splitters(spk, spv, nb - 1, sk, sv);
    for (int b = threadIdx.x; b < nb; b += SS_TT) cnt[b] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SS_TILE;
#pragma unroll
    for (int i = 0; i < SS_TI; i++) {
        const int64_t e = base + (int64_t)i * SS_TT + threadIdx.x;
        if (e < n) atomicAdd(&cnt[ss_bucket(k[e], (uint32_t)v[e], sk, sv, nb - 1)], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += SS_TT) hist[(int64_t)b * gridDim.x + blockIdx.x] = cnt[b];
}

// 4. scatter into buckets (slot order inside a bucket is arbitrary: step 5 sorts it)
__global__ __launch_bounds__(SS_TT) void k_ss_scatter(const uint64_t *__restrict__ k, const int32_t *__restrict__ v,
                                                     int64_t n, int nb, const uint64_t *__restrict__ spk,
                                                     const uint32_t *__restrict__ spv,
                                                     const int32_t *__restrict__ hist, uint64_t *__restrict__ ko,
                                                     int32_t *__restrict__ vo)
{
    __shared__ uint64_t sk[SS_MAXB];
    __shared__ uint32_t sv[SS_MAXB];
    __shared__ int32_t cur[SS_MAXB];
    ss_load_splitters(spk, spv, nb - 1, sk, sv);
    // the scanned counts: output position of this tile's first pair of bucket b
    for (int b = threadIdx.x; b < nb; b += SS_TT) cur[b] = hist[(int64_t)b * gridDim.x + blockIdx.x];
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SS_TILE;
#pragma unroll
    for (int i = 0; i < SS_TI; i++) {
        const int64_t e = base + (int64_t)i * SS_TT + threadIdx.x;
        if (e < n) {
            const uint64_t kk = k[e];
            const int32_t vv = v[e];
            const int32_t p = atomicAdd(&cur[ss_bucket(kk, (uint32_t)vv, sk, sv, nb - 1)], 1);
            ko[p] = kk;
            vo[p] = vv;
        }
    }
}

// 5. one workgroup per bucket: bucket b is [hist[b * ntiles], hist[(b + 1) * ntiles]) of
// the scanned counts (the last one ends at n)
__global__ __launch_bounds__(SS_BT) void k_ss_bucket(uint64_t *__restrict__ k, int32_t *__restrict__ v,
                                                    const int32_t *__restrict__ hist, int64_t ntiles, int nb,
                                                    int64_t n, int64_t cap)
{
    __shared__ uint64_t ek[SS_CAP];
    __shared__ uint32_t ev[SS_CAP];
    const int b = blockIdx.x;
    const int64_t s0 = hist[(int64_t)b * ntiles];
    const int64_t s1 = (b + 1 < nb) ? hist[(int64_t)(b + 1) * ntiles] : n;
    const int S = (int)(s1 - s0);
    if (S <= 1) return;
    if (S <= cap) {
        if (S <= SS_BT) ss_sort_run<1>(k + s0, v + s0, S, ek, ev);
        else if (S <= 2 * SS_BT) ss_sort_run<2>(k + s0, v + s0, S, ek, ev);
        else if (S <= 4 * SS_BT) ss_sort_run<4>(k + s0, v + s0, S, ek, ev);
        else ss_sort_run<8>(k + s0, v + s0, S, ek, ev);
    } else {  // a bucket far above its expected size: the LDS network in global memory
        ss_network(k + s0, (uint32_t *)(v + s0), S);
    }
}

// Sorts n pairs by (key, value).  The result is in (k, v) on return; (k2, v2) are
// scratch of the same length (the pointers are swapped, as by the radix sort).
void sample_sort_pairs(gss_ctx ctx, uint64_t *&k, int32_t *&v, uint64_t *&k2, int32_t *&v2, int64_t n)
{
    if (n <= 1) return;
    if (n > sample_sort_max()) throw gss_error{GSS_ERR_ARG, "sample sort: too many pairs"};
    hipStream_t st = ctx->stream;
    const int nb = (int)std::min<int64_t>(SS_MAXB, (n + SS_MEAN - 1) / SS_MEAN);  // about SS_MEAN pairs per bucket
    const int64_t ntiles = (n + SS_TILE - 1) / SS_TILE;
    // the register limit, or a smaller one set for tests (buckets above it take the global path)
    const int64_t cap = std::min<int64_t>(ctx->sort_cap > 0 ? ctx->sort_cap : SS_CAP, SS_CAP);
    int32_t *hist = ctx->alloc<int32_t>(ntiles * nb + 1);
    if (nb == 1) {  // one bucket: sort in place
        int32_t h = 0;
        ctx->h2d(hist, &h, sizeof h);
        GSS_LAUNCH_B(24 * n, k_ss_bucket, dim3(1), dim3(SS_BT), 0, st, k, v, hist, (int64_t)1, 1, n, cap);
        ctx->free(hist);
        return;
    }
    // at least 1024 samples and at most n; 2048 up to 1024 buckets (the ranking grows as the
    // square of the sample), 4096 beyond
    int lgns = nb <= 128 ? 10 : nb <= 1024 ? 11 : 12;
    while (((int64_t)1 << lgns) > n) lgns--;
    uint64_t *spk = ctx->alloc<uint64_t>(nb);
    uint32_t *spv = ctx->alloc<uint32_t>(nb);
    GSS_LAUNCH_B(12 * ((int64_t)1 << lgns), k_ss_splitters, dim3((unsigned)(((int64_t)SS_RT << lgns) / SS_RB)),
                 dim3(SS_RB), 0, st, k, v, n, lgns, nb, spk, spv);
    GSS_LAUNCH_B(12 * n, k_ss_count, dim3((unsigned)ntiles), dim3(SS_TT), 0, st, k, v, n, nb, spk, spv, hist);
    scan_exclusive_i32_dev(ctx, hist, ntiles * nb, ctx->d_counters + 11);
    GSS_LAUNCH_B(24 * n, k_ss_scatter, dim3((unsigned)ntiles), dim3(SS_TT), 0, st, k, v, n, nb, spk, spv, hist, k2,
                 v2);
    GSS_LAUNCH_B(24 * n, k_ss_bucket, dim3(nb), dim3(SS_BT), 0, st, k2, v2, hist, ntiles, nb, n, cap);
    HIP_OK(hipGetLastError());
    std::swap(k, k2);
    std::swap(v, v2);
    ctx->free(spk);
    ctx->free(spv);
    ctx->free(hist);
}

int64_t sample_sort_max() { return (int64_t)SS_MAXB * SS_MEAN; }

// ------------------------------------------------------------------------------------
// LSD radix sort of large (key, double) arrays: per 8-bit digit a counting pass (one
// LDS histogram per tile, stored digit-major), an exclusive scan of the digit-major
// counts (every digit's tiles in order, digits in order), and a scatter pass that ranks
// each tile's elements per digit in element order (wave-level peer ballots, then the
// waves in order) and adds the tile's scanned offset.  Stable; every pass is a stream
// over the arrays with no chain between tiles.  With run, the passes do nothing unless
// *run is nonzero (a choice made on the device).
// ------------------------------------------------------------------------------------
#define LSD_BLOCK 256
#define LSD_ITEMS 16
#define LSD_TILE (LSD_BLOCK * LSD_ITEMS)

__global__ __launch_bounds__(LSD_BLOCK) void k_lsd_count(const uint64_t *__restrict__ k, int64_t n, int shift,
                                                         int64_t ntiles, int32_t *__restrict__ hist,
                                                         const int64_t *__restrict__ run)
{
    if (run && *run == 0) return;
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * LSD_TILE;
#pragma unroll
    for (int i = 0; i < LSD_ITEMS; i++) {
        const int64_t idx = base + (int64_t)i * LSD_BLOCK + threadIdx.x;
        if (idx < n) atomicAdd(&h[(uint32_t)(k[idx] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// The scatter stages each tile in LDS in digit order first (local place = the digit's
// start in the tile + the earlier waves' count of it + the rank in the wave), then writes
// the staged keys, and after them the staged values, in order: consecutive threads write
// consecutive places of a digit's run, so the writes are coalesced instead of 256-way
// scattered.
__global__ __launch_bounds__(LSD_BLOCK) void k_lsd_scatter(const uint64_t *__restrict__ kin,
                                                           const double *__restrict__ win, int64_t n, int shift,
                                                           int64_t ntiles, const int32_t *__restrict__ off,
                                                           uint64_t *__restrict__ kout, double *__restrict__ wout,
                                                           const int64_t *__restrict__ run)
{
    if (run && *run == 0) return;
    constexpr int NW = LSD_BLOCK / GSS_WAVE;
    constexpr int PER = LSD_ITEMS;  // items per lane in the wave's contiguous chunk
    __shared__ int32_t s_cnt[NW][256];
    __shared__ int32_t s_scan[NW + 1];
    __shared__ int32_t s_dstart[256], s_goff[256];
    __shared__ uint64_t s_k[LSD_TILE];  // keys, then values, in digit order
    __shared__ uint8_t s_d[LSD_TILE];
    const int t = threadIdx.x, wid = t / GSS_WAVE, lane = lane_id();
#pragma unroll
    for (int w = 0; w < NW; w++) s_cnt[w][t] = 0;
    __syncthreads();
    // wave wid owns the contiguous chunk [wbase, wbase + PER * 64) of the tile
    const int64_t tbase = (int64_t)blockIdx.x * LSD_TILE;
    const int64_t wbase = tbase + (int64_t)wid * (PER * GSS_WAVE);
    uint64_t kk[PER];
    double ww[PER];
    int32_t pos[PER];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const int64_t idx = wbase + i * GSS_WAVE + lane;
        kk[i] = idx < n ? kin[idx] : 0;
        ww[i] = idx < n ? win[idx] : 0.0;
    }
    int32_t *cnt = s_cnt[wid];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        const bool valid = wbase + i * GSS_WAVE + lane < n;
        const uint32_t d = (uint32_t)(kk[i] >> shift) & 255u;
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
    // thread t = digit t: the earlier waves' counts of it, its start inside the tile and
    // its place in the output
    int32_t tot_t = 0;
#pragma unroll
    for (int w = 0; w < NW; w++) {
        const int32_t c = s_cnt[w][t];
        s_cnt[w][t] = tot_t;
        tot_t += c;
    }
    int32_t all;
    const int32_t dstart = block_exclusive_scan<int32_t>(tot_t, s_scan, &all);  // synchronises
    s_dstart[t] = dstart;
    s_goff[t] = off[(int64_t)t * ntiles + blockIdx.x];
    __syncthreads();
    int32_t lp[PER];
#pragma unroll
    for (int i = 0; i < PER; i++) {
        lp[i] = -1;
        if (wbase + i * GSS_WAVE + lane < n) {
            const uint32_t d = (uint32_t)(kk[i] >> shift) & 255u;
            lp[i] = s_dstart[d] + cnt[d] + pos[i];
            s_k[lp[i]] = kk[i];
            s_d[lp[i]] = (uint8_t)d;
        }
    }
    __syncthreads();
    const int nt = (int)(n - tbase < LSD_TILE ? n - tbase : LSD_TILE);
    for (int q = t; q < nt; q += LSD_BLOCK) {
        const int d = s_d[q];
        kout[s_goff[d] + (q - s_dstart[d])] = s_k[q];
    }
    __syncthreads();
    double *s_w = (double *)s_k;
#pragma unroll
    for (int i = 0; i < PER; i++)
        if (lp[i] >= 0) s_w[lp[i]] = ww[i];
    __syncthreads();
    for (int q = t; q < nt; q += LSD_BLOCK) {
        const int d = s_d[q];
        wout[s_goff[d] + (q - s_dstart[d])] = s_w[q];
    }
}

void lsd_sort_kw(gss_ctx ctx, uint64_t *&k, double *&w, uint64_t *&k2, double *&w2, int64_t n, int shift,
                 int passes, const int64_t *run)
{
    if (n <= 1) return;
    if (n >= ((int64_t)1 << 31)) throw gss_error{GSS_ERR_ARG, "radix sort: too many elements"};
    hipStream_t st = ctx->stream;
    const int64_t ntiles = (n + LSD_TILE - 1) / LSD_TILE;
    int32_t *hist = ctx->alloc<int32_t>(256 * ntiles + 1);
    for (int p = 0; p < passes; p++) {
        const int sh = shift + 8 * p;
        GSS_LAUNCH_B(8 * n, k_lsd_count, dim3((unsigned)ntiles), dim3(LSD_BLOCK), 0, ctx->stream, k, n, sh, ntiles,
                     hist, run);
        scan_exclusive_i32_dev(ctx, hist, 256 * ntiles, ctx->d_counters + 11);
        GSS_LAUNCH_B(32 * n, k_lsd_scatter, dim3((unsigned)ntiles), dim3(LSD_BLOCK), 0, ctx->stream, k, w, n, sh,
                     ntiles, hist, k2, w2, run);
        HIP_OK(hipGetLastError());
        std::swap(k, k2);
        std::swap(w, w2);
    }
    ctx->free(hist);
    (void)st;
}
