// gss_prims.hip -- device allocator, error flags and the exclusive scan used throughout.
#include "gss_impl.h"

// ------------------------------------------------------------------------------------
// caching allocator
// ------------------------------------------------------------------------------------
void *dev_pool::get(size_t bytes)
{
    if (bytes == 0) bytes = 16;
    auto it = free_blocks.lower_bound(bytes);
    // reuse a cached block unless it is more than 4x too large
    if (it != free_blocks.end() && it->first <= 4 * bytes + (1u << 20)) {
        void *p = it->second;
        size_t cap = it->first;
        free_blocks.erase(it);
        live[p] = cap;
        return p;
    }
    size_t cap = (bytes + 4095) & ~(size_t)4095;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, cap);
    if (e != hipSuccess) {
        // drop the cache and retry once
        (void)hipGetLastError();
        for (auto &kv : free_blocks) {
            (void)hipFree(kv.second);
            bytes_held -= kv.first;
        }
        free_blocks.clear();
        e = hipMalloc(&p, cap);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            throw gss_error{GSS_ERR_OOM, "hipMalloc of " + std::to_string(cap) + " bytes failed"};
        }
    }
    bytes_held += cap;
    live[p] = cap;
    return p;
}

void dev_pool::put(void *p)
{
    auto it = live.find(p);
    if (it == live.end()) return;
    free_blocks.emplace(it->second, p);
    live.erase(it);
}

void dev_pool::release_all()
{
    for (auto &kv : free_blocks) (void)hipFree(kv.second);
    for (auto &kv : live) (void)hipFree(kv.first);
    free_blocks.clear();
    live.clear();
    bytes_held = 0;
}

// ------------------------------------------------------------------------------------
// live kernel timing
// ------------------------------------------------------------------------------------
void gss_ctx_s::prof_begin(const char *name)
{
    if (!prof_filter.empty() && prof_filter != name) {
        prof_pending.push_back(prof_rec{nullptr, nullptr, nullptr});
        return;
    }
    prof_rec r;
    r.name = name;
    for (hipEvent_t *e : {&r.a, &r.b}) {
        if (prof_events.empty()) HIP_OK(hipEventCreate(e));
        else {
            *e = prof_events.back();
            prof_events.pop_back();
        }
    }
    HIP_OK(hipEventRecord(r.a, stream));
    prof_pending.push_back(r);
}

void gss_ctx_s::prof_end()
{
    prof_rec &r = prof_pending.back();
    if (r.name) HIP_OK(hipEventRecord(r.b, stream));
}

void gss_ctx_s::prof_collect()
{
    for (prof_rec &r : prof_pending) {
        if (!r.name) continue;
        float ms = 0.f;
        HIP_OK(hipEventSynchronize(r.b));
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        auto &acc = prof_acc[r.name];
        acc.first += ms;
        acc.second += 1;
        prof_events.push_back(r.a);
        prof_events.push_back(r.b);
    }
    prof_pending.clear();
}

// ------------------------------------------------------------------------------------
// flags
// ------------------------------------------------------------------------------------
uint32_t read_flags(gss_ctx ctx)
{
    uint32_t f = 0;
    HIP_OK(hipMemcpyAsync(&ctx->h_counters[15], ctx->d_flags, sizeof(uint32_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    memcpy(&f, &ctx->h_counters[15], sizeof f);
    return f;
}

gss_status status_from_flags(uint32_t f)
{
    if (f & F_ARG) return GSS_ERR_ARG;
    if (f & F_NOT_SIMPLE) return GSS_ERR_NOT_SIMPLE;
    if (f & F_WEIGHT) return GSS_ERR_WEIGHT;
    if (f & F_ASYM) return GSS_ERR_ASYM;
    if (f & F_NOT_TREE) return GSS_ERR_NOT_TREE;
    if (f & F_TREE_EDGE) return GSS_ERR_TREE_EDGE;
    if (f & F_RANGE) return GSS_ERR_RANGE;
    return GSS_OK;
}

// ------------------------------------------------------------------------------------
// exclusive scan of int32, three phases
// ------------------------------------------------------------------------------------
#define SCAN_BLOCK 256
#define SCAN_ITEMS 16

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_reduce(const int32_t *__restrict__ in,
                                                            int64_t n, int64_t *__restrict__ bsum)
{
    __shared__ int64_t lds[SCAN_BLOCK / GSS_WAVE + 1];
    int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK * SCAN_ITEMS;
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        int64_t k = base + (int64_t)i * SCAN_BLOCK + threadIdx.x;
        if (k < n) s += in[k];
    }
    int64_t tot;
    block_exclusive_scan<int64_t>(s, lds, &tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_bsums(int64_t *__restrict__ bsum, int64_t nb,
                                                     int64_t *__restrict__ total)
{
    __shared__ int64_t lds[1024 / GSS_WAVE + 1];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
        int64_t k = b0 + threadIdx.x;
        int64_t v = (k < nb) ? bsum[k] : 0;
        int64_t tot;
        int64_t ex = block_exclusive_scan<int64_t>(v, lds, &tot);
        if (k < nb) bsum[k] = ex + carry;
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_apply(int32_t *__restrict__ data, int64_t n,
                                                           const int64_t *__restrict__ bsum)
{
    __shared__ int64_t lds[SCAN_BLOCK / GSS_WAVE + 1];
    // each thread owns SCAN_ITEMS consecutive elements of the block's tile
    int64_t base = (int64_t)blockIdx.x * SCAN_BLOCK * SCAN_ITEMS + (int64_t)threadIdx.x * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        int64_t k = base + i;
        v[i] = (k < n) ? data[k] : 0;
        s += v[i];
    }
    int64_t tot;
    int64_t ex = block_exclusive_scan<int64_t>(s, lds, &tot) + bsum[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; i++) {
        int64_t k = base + i;
        if (k < n) data[k] = (int32_t)ex;
        ex += v[i];
    }
}

// one workgroup scans the whole array in chunks (short arrays: one launch instead of three)
#define SMALL_ITEMS 8
__global__ __launch_bounds__(1024) void k_scan_single(int32_t *__restrict__ data, int64_t n,
                                                      int64_t *__restrict__ total)
{
    __shared__ int64_t lds[1024 / GSS_WAVE + 1];
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < n; c0 += 1024 * SMALL_ITEMS) {
        int64_t base = c0 + (int64_t)threadIdx.x * SMALL_ITEMS;
        int32_t v[SMALL_ITEMS];
        int64_t s = 0;
#pragma unroll
        for (int i = 0; i < SMALL_ITEMS; i++) {
            v[i] = (base + i < n) ? data[base + i] : 0;
            s += v[i];
        }
        int64_t tot;
        int64_t ex = block_exclusive_scan<int64_t>(s, lds, &tot) + carry;
#pragma unroll
        for (int i = 0; i < SMALL_ITEMS; i++) {
            if (base + i < n) data[base + i] = (int32_t)ex;
            ex += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) *total = carry;
}

int64_t scan_exclusive_i32(gss_ctx ctx, int32_t *data, int64_t n, bool want_total)
{
    if (n <= 0) return 0;
    if (n <= 32 * 1024) {
        GSS_LAUNCH(k_scan_single, dim3(1), dim3(1024), 0, ctx->stream, data, n, ctx->d_counters + 14);
        HIP_OK(hipGetLastError());
        if (!want_total) return -1;
        HIP_OK(hipMemcpyAsync(&ctx->h_counters[14], ctx->d_counters + 14, sizeof(int64_t),
                              hipMemcpyDeviceToHost, ctx->stream));
        ctx->sync();
        return ctx->h_counters[14];
    }
    int64_t nb = (n + SCAN_BLOCK * SCAN_ITEMS - 1) / (SCAN_BLOCK * SCAN_ITEMS);
    int64_t *bsum = ctx->alloc<int64_t>(nb + 1);
    GSS_LAUNCH(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, ctx->stream, data, n,
                       bsum);
    GSS_LAUNCH(k_scan_bsums, dim3(1), dim3(1024), 0, ctx->stream, bsum, nb,
                       ctx->d_counters + 14);
    GSS_LAUNCH(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_BLOCK), 0, ctx->stream, data, n,
                       bsum);
    HIP_OK(hipGetLastError());
    ctx->free(bsum);
    if (!want_total) return -1;
    HIP_OK(hipMemcpyAsync(&ctx->h_counters[14], ctx->d_counters + 14, sizeof(int64_t),
                          hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    return ctx->h_counters[14];
}
