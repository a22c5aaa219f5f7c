// gss_sort.hip -- sample sort of (64-bit key, 32-bit value) pairs for the short sorts of
// the recovery: a prefix of the criticality order (Alg. 1 Step 2), its grouping by LCA
// (Step 3) and the subtask work queue.  These sorts hold a few hundred thousand pairs,
// too few for a radix sort to reach bandwidth: every radix pass is a launch bounded by
// its latency.  A sample sort needs five launches whatever the key width:
//   1. one workgroup sorts a stratified sample of the pairs in LDS and keeps nb - 1
//      evenly spaced splitters,
//   2. every tile counts its pairs per bucket (binary search over the splitters in LDS),
//   3. one workgroup turns the counts into bucket starts and per-tile output offsets,
//   4. every tile scatters its pairs into their buckets,
//   5. one workgroup per bucket sorts it: in LDS when it fits (eight times the mean
//      bucket size of about 1024 pairs), otherwise in place in global memory (same
//      network, slower).
// Pairs are ordered by (key, value); the callers' values are distinct, so the order is
// total and the result does not depend on the order in which a bucket is filled.
// The sorting network is the bitonic one in its one-direction form (the first step of
// every merge compares mirrored positions), so sizes need not be powers of two:
// comparisons that reach past the end are skipped.
#include <algorithm>

#include "gss_impl.h"

#define SS_SAMPLES 4096  // largest sample (power of two)
#define SS_TT 256        // threads of the counting and scatter kernels
#define SS_TI 16         // pairs per thread there
#define SS_TILE (SS_TT * SS_TI)
#define SS_MAXB 512      // largest bucket count
#define SS_BT 1024       // threads of the sample and bucket kernels
#define SS_CAP 8192      // largest bucket sorted in LDS

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

// 1. the sample: ns strata of equal length, one pair from each at a hashed offset;
// splitter b (b < nb - 1) is sample (b + 1) * ns / nb of the sorted sample
__global__ __launch_bounds__(SS_BT) void k_ss_sample(const uint64_t *__restrict__ k, const int32_t *__restrict__ v,
                                                    int64_t n, int ns, int nb, uint64_t *__restrict__ spk,
                                                    uint32_t *__restrict__ spv)
{
    __shared__ uint64_t sk[SS_SAMPLES];
    __shared__ uint32_t sv[SS_SAMPLES];
    for (int i = threadIdx.x; i < ns; i += SS_BT) {
        const int64_t lo = (int64_t)i * n / ns, hi = (int64_t)(i + 1) * n / ns;
        int64_t p = lo;
        if (hi > lo) p = lo + (int64_t)(mix64(0x9E3779B97F4A7C15ull * (uint64_t)(i + 1)) % (uint64_t)(hi - lo));
        if (p >= n) p = n - 1;
        sk[i] = k[p];
        sv[i] = (uint32_t)v[p];
    }
    __syncthreads();
    ss_network(sk, sv, ns);
    for (int b = threadIdx.x; b < nb - 1; b += SS_BT) {
        const int s = (int)((int64_t)(b + 1) * ns / nb);
        spk[b] = sk[s];
        spv[b] = sv[s];
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

// 2. per tile and bucket: hist[tile * nb + b]
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
    for (int b = threadIdx.x; b < nb; b += SS_TT) hist[(int64_t)blockIdx.x * nb + b] = cnt[b];
}

// 3. offsets: hist[t][b] becomes the output position of tile t's first pair of bucket b
// (bucket-major order); bptr[b] = start of bucket b, bptr[nb] = n.  One thread per bucket
// walks the tiles.
__global__ __launch_bounds__(SS_MAXB) void k_ss_offsets(int32_t *__restrict__ hist, int64_t ntiles, int nb,
                                                       int32_t *__restrict__ bptr)
{
    __shared__ int32_t lds[SS_MAXB / GSS_WAVE + 1];
    const int b = threadIdx.x;
    int32_t run = 0;
    if (b < nb) {
        for (int64_t t = 0; t < ntiles; t++) {
            const int32_t c = hist[t * nb + b];
            hist[t * nb + b] = run;
            run += c;
        }
    }
    int32_t total;
    const int32_t start = block_exclusive_scan<int32_t>(b < nb ? run : 0, lds, &total);
    if (b < nb) {
        bptr[b] = start;
        for (int64_t t = 0; t < ntiles; t++) hist[t * nb + b] += start;
    }
    if (b == 0) bptr[nb] = total;
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
    for (int b = threadIdx.x; b < nb; b += SS_TT) cur[b] = hist[(int64_t)blockIdx.x * nb + b];
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

// 5. one workgroup per bucket
__global__ __launch_bounds__(SS_BT) void k_ss_bucket(uint64_t *__restrict__ k, int32_t *__restrict__ v,
                                                    const int32_t *__restrict__ bptr, int64_t cap)
{
    __shared__ uint64_t sk[SS_CAP];
    __shared__ uint32_t sv[SS_CAP];
    const int64_t s0 = bptr[blockIdx.x];
    const int S = bptr[blockIdx.x + 1] - bptr[blockIdx.x];
    if (S <= 1) return;
    if (S <= cap) {
        for (int i = threadIdx.x; i < S; i += SS_BT) {
            sk[i] = k[s0 + i];
            sv[i] = (uint32_t)v[s0 + i];
        }
        __syncthreads();
        ss_network(sk, sv, S);
        for (int i = threadIdx.x; i < S; i += SS_BT) {
            k[s0 + i] = sk[i];
            v[s0 + i] = (int32_t)sv[i];
        }
    } else {  // a bucket far above its expected size: the same network in global memory
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
    const int nb = (int)std::min<int64_t>(SS_MAXB, (n + 1023) / 1024);  // about 1024 pairs per bucket
    const int64_t ntiles = (n + SS_TILE - 1) / SS_TILE;
    const int64_t cap = std::min<int64_t>(ctx->sort_cap > 0 ? ctx->sort_cap : SS_CAP, SS_CAP);
    int32_t *bptr = ctx->alloc<int32_t>(nb + 1);
    if (nb == 1) {
        // one bucket: sort in place
        int32_t h[2] = {0, (int32_t)n};
        ctx->h2d(bptr, h, sizeof h);
        GSS_LAUNCH_B(24 * n, k_ss_bucket, dim3(1), dim3(SS_BT), 0, st, k, v, bptr, cap);
        ctx->free(bptr);
        return;
    }
    int ns = 32;
    while (ns < 16 * nb && ns < SS_SAMPLES) ns <<= 1;
    uint64_t *spk = ctx->alloc<uint64_t>(nb);
    uint32_t *spv = ctx->alloc<uint32_t>(nb);
    int32_t *hist = ctx->alloc<int32_t>(ntiles * nb);
    GSS_LAUNCH_B(12 * (int64_t)ns, k_ss_sample, dim3(1), dim3(SS_BT), 0, st, k, v, n, ns, nb, spk, spv);
    GSS_LAUNCH_B(12 * n, k_ss_count, dim3((unsigned)ntiles), dim3(SS_TT), 0, st, k, v, n, nb, spk, spv, hist);
    GSS_LAUNCH(k_ss_offsets, dim3(1), dim3(SS_MAXB), 0, st, hist, ntiles, nb, bptr);
    GSS_LAUNCH_B(24 * n, k_ss_scatter, dim3((unsigned)ntiles), dim3(SS_TT), 0, st, k, v, n, nb, spk, spv, hist, k2,
                 v2);
    GSS_LAUNCH_B(24 * n, k_ss_bucket, dim3(nb), dim3(SS_BT), 0, st, k2, v2, bptr, cap);
    HIP_OK(hipGetLastError());
    std::swap(k, k2);
    std::swap(v, v2);
    ctx->free(spk);
    ctx->free(spv);
    ctx->free(hist);
    ctx->free(bptr);
}

int64_t sample_sort_max() { return (int64_t)SS_MAXB * 1024; }
