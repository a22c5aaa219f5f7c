// gss_prims.hip -- device allocator, error flags and the exclusive scan used throughout.
#include "gss_impl.h"
#include "gss_lookback.h"

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
prof_rec *gss_ctx_s::prof_begin(const char *name)
{
    const int64_t bytes = prof_bytes;
    prof_bytes = 0;
    if (!prof_filter.empty() && prof_filter != name) return nullptr;
    prof_rec r;
    r.name = name;
    r.bytes = bytes;
    for (hipEvent_t *e : {&r.a, &r.b}) {
        if (prof_events.empty()) HIP_OK(hipEventCreate(e));
        else {
            *e = prof_events.back();
            prof_events.pop_back();
        }
    }
    prof_pending.push_back(r);
    return &prof_pending.back();
}

void gss_ctx_s::prof_collect()
{
    for (prof_rec &r : prof_pending) {
        if (!r.name) continue;
        float ms = 0.f;
        HIP_OK(hipEventSynchronize(r.b));
        HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
        prof_sum &acc = prof_acc[r.name];
        acc.ms += ms;
        acc.last_ms = ms;
        acc.launches += 1;
        acc.bytes += r.bytes;
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
// exclusive scan of int32, one pass (decoupled look-back between tiles)
// ------------------------------------------------------------------------------------
#define SCAN_BLOCK 256
#define SCAN_ROUNDS 4
#define SCAN_TILE (SCAN_BLOCK * 4 * SCAN_ROUNDS)  // elements per tile

// Thread t of round r owns the four consecutive elements at tile offset 4 (r*256 + t),
// read and written as one 16-byte vector, so every round is fully coalesced.
__global__ __launch_bounds__(SCAN_BLOCK) void k_scan_onepass(int32_t *__restrict__ data, int64_t n,
                                                             int64_t ntiles, uint64_t *__restrict__ status,
                                                             uint32_t epoch, unsigned long long *ticket,
                                                             int64_t *__restrict__ total)
{
    constexpr int NW = SCAN_BLOCK / GSS_WAVE;
    __shared__ int64_t s_wsum[SCAN_ROUNDS][NW];
    __shared__ int64_t s_tile, s_excl;
    const int lane = lane_id(), wid = threadIdx.x / GSS_WAVE;
    if (threadIdx.x == 0) s_tile = lb_ticket(ticket, ntiles);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * SCAN_TILE;
    int4 v[SCAN_ROUNDS];
    int64_t incl[SCAN_ROUNDS];
#pragma unroll
    for (int r = 0; r < SCAN_ROUNDS; r++) {
        const int64_t e = base + ((int64_t)r * SCAN_BLOCK + threadIdx.x) * 4;
        if (e + 4 <= n) {
            v[r] = *(const int4 *)(data + e);
        } else {
            v[r].x = (e < n) ? data[e] : 0;
            v[r].y = (e + 1 < n) ? data[e + 1] : 0;
            v[r].z = (e + 2 < n) ? data[e + 2] : 0;
            v[r].w = 0;
        }
        int64_t x = (int64_t)v[r].x + v[r].y + v[r].z + v[r].w;
#pragma unroll
        for (int d = 1; d < GSS_WAVE; d <<= 1) {
            int64_t y = __shfl_up(x, d, GSS_WAVE);
            if (lane >= d) x += y;
        }
        incl[r] = x;
        if (lane == GSS_WAVE - 1) s_wsum[r][wid] = x;
    }
    __syncthreads();
    // offsets of (round, wave) pieces in tile order, and the tile total
    int64_t off[SCAN_ROUNDS];
    int64_t run = 0;
#pragma unroll
    for (int r = 0; r < SCAN_ROUNDS; r++) {
        for (int w = 0; w < NW; w++) {
            if (w == wid) off[r] = run;
            run += s_wsum[r][w];
        }
    }
    const int64_t tile_total = run;
    if (wid == 0) {
        int64_t excl = 0;
        if (tile == 0) {
            if (lane == 0) lb_store(status, lb_word(LB_INC, epoch, (uint64_t)tile_total));
        } else {
            if (lane == 0) lb_store(status + tile, lb_word(LB_AGG, epoch, (uint64_t)tile_total));
            excl = lb_lookback_wave(status, 1, tile, epoch);
            if (lane == 0) lb_store(status + tile, lb_word(LB_INC, epoch, (uint64_t)(excl + tile_total)));
        }
        if (lane == 0) {
            s_excl = excl;
            if (tile == ntiles - 1) *total = excl + tile_total;
        }
    }
    __syncthreads();
    const int64_t excl = s_excl;
#pragma unroll
    for (int r = 0; r < SCAN_ROUNDS; r++) {
        const int64_t e = base + ((int64_t)r * SCAN_BLOCK + threadIdx.x) * 4;
        const int64_t p0 = excl + off[r] + incl[r] - ((int64_t)v[r].x + v[r].y + v[r].z + v[r].w);
        int4 o;
        o.x = (int32_t)p0;
        o.y = (int32_t)(p0 + v[r].x);
        o.z = (int32_t)(p0 + v[r].x + v[r].y);
        o.w = (int32_t)(p0 + v[r].x + v[r].y + v[r].z);
        if (e + 4 <= n) {
            *(int4 *)(data + e) = o;
        } else {
            if (e < n) data[e] = o.x;
            if (e + 1 < n) data[e + 1] = o.y;
            if (e + 2 < n) data[e + 2] = o.z;
        }
    }
}

// Byte fill by a kernel: 16-byte stores over the aligned middle, single bytes at the
// ends.  A kernel rather than a runtime memset, so the recovery's launches can be
// captured into a graph and replayed with the fills as ordinary kernel nodes.
__global__ void k_fill_bytes(uint8_t *__restrict__ p, uint64_t bytes, uint32_t v4)
{
    const uint64_t head = min(bytes, (uint64_t)((16 - ((uintptr_t)p & 15)) & 15));
    const uint64_t chunks = (bytes - head) / 16;
    const uint64_t tail0 = head + chunks * 16;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint4 q = make_uint4(v4, v4, v4, v4);
    uint4 *body = (uint4 *)(p + head);
    for (uint64_t i = t; i < chunks; i += stride) body[i] = q;
    if (t < head) p[t] = (uint8_t)v4;
    if (t < bytes - tail0) p[tail0 + t] = (uint8_t)v4;
}

void fill_bytes(gss_ctx ctx, void *p, int value, size_t bytes)
{
    if (!p || bytes == 0) return;
    const uint32_t v = (uint32_t)(value & 0xff) * 0x01010101u;
    const unsigned blocks = (unsigned)std::min<uint64_t>(std::max<uint64_t>((bytes / 16 + 255) / 256, 1), 2048);
    GSS_LAUNCH(k_fill_bytes, dim3(blocks), dim3(256), 0, ctx->stream, (uint8_t *)p, (uint64_t)bytes, v);
}

// capturing: compares replayed device bytes with the recorded ones, in chunks passed by
// value, and raises the graph's mismatch word on a difference
struct ReplayBytes {
    uint8_t b[512];
};
__global__ void k_check_replay(const uint8_t *__restrict__ dev, uint32_t n, ReplayBytes expect, uint64_t words,
                               uint32_t id, uint32_t *flag)
{
    const uint32_t i = threadIdx.x;
    const bool bad = i < n && ((words >> (i / 8)) & 1) && dev[i] != expect.b[i];
    if (__any(bad) && lane_id() == 0) atomicMax(flag, id);  // the last differing check (numbered from 1)
}

void gss_ctx_s::check_replay(const void *dev, const void *expect, size_t bytes, uint64_t words)
{
    gss_ctx ctx = this;
    for (size_t off = 0; off < bytes; off += sizeof(ReplayBytes)) {
        ReplayBytes e;
        const size_t n = std::min(bytes - off, sizeof(ReplayBytes));
        memcpy(e.b, (const uint8_t *)expect + off, n);
        // chunk c covers words [c * 64, c * 64 + 64); the mask names the first 64 only
        const uint64_t w = off == 0 ? words : ~0ull;
        GSS_LAUNCH(k_check_replay, dim3(1), dim3(512), 0, stream, (const uint8_t *)dev + off, (uint32_t)n, e, w,
                   ++cap_checks, cap_flag);
    }
}

uint64_t *lb_begin(gss_ctx ctx, int64_t words, uint32_t *epoch)
{
    if (ctx->cap_mode == gss_ctx_s::CAP_RECORD) ctx->arena_account(sizeof(uint64_t) * words + 16);
    if (ctx->arena) {  // allocation-free call: a fresh, cleared status array from the arena
        uint64_t *s = ctx->alloc<uint64_t>(words);
        fill_bytes(ctx, s, 0, sizeof(uint64_t) * words);
        *epoch = 1;
        return s;
    }
    const int l = ctx->lb_lane;
    if (words > ctx->lb_cap[l]) {
        ctx->free(ctx->lb_status[l]);
        const int64_t cap = std::max<int64_t>(words, 1 << 16);
        ctx->lb_status[l] = ctx->alloc<uint64_t>(cap);
        fill_bytes(ctx, ctx->lb_status[l], 0, sizeof(uint64_t) * cap);
        ctx->lb_cap[l] = cap;
        ctx->lb_epoch[l] = 0;
    }
    if (++ctx->lb_epoch[l] >= (1u << LB_EPOCH_BITS)) {
        fill_bytes(ctx, ctx->lb_status[l], 0, sizeof(uint64_t) * ctx->lb_cap[l]);
        ctx->lb_epoch[l] = 1;
    }
    *epoch = ctx->lb_epoch[l];
    return ctx->lb_status[l];
}

void aux_join(gss_ctx ctx)
{
    HIP_OK(hipEventRecord(ctx->ev_join, ctx->aux));
    HIP_OK(hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0));
    for (void *p : ctx->aux_frees) ctx->pool.put(p);
    ctx->aux_frees.clear();
}

// one workgroup scans a short array (at most 1024 * SMALL_ITEMS elements) in one sweep:
// thread t owns the SMALL_ITEMS consecutive elements at t * SMALL_ITEMS, read and written
// as 16-byte vectors when the array is 16-byte aligned; a single latency-bound launch
// instead of the three of the tiled scan
#define SMALL_ITEMS 32
__global__ __launch_bounds__(1024) void k_scan_single(int32_t *__restrict__ data, int64_t n,
                                                      int64_t *__restrict__ total)
{
    __shared__ int64_t lds[1024 / GSS_WAVE + 1];
    const int64_t base = (int64_t)threadIdx.x * SMALL_ITEMS;
    int32_t v[SMALL_ITEMS];
    const bool vec = (((uintptr_t)data & 15) == 0) && base + SMALL_ITEMS <= n;
    if (vec) {
#pragma unroll
        for (int i = 0; i < SMALL_ITEMS; i += 4) {
            const int4 q = *(const int4 *)(data + base + i);
            v[i] = q.x;
            v[i + 1] = q.y;
            v[i + 2] = q.z;
            v[i + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < SMALL_ITEMS; i++) v[i] = (base + i < n) ? data[base + i] : 0;
    }
    int64_t s = 0;
#pragma unroll
    for (int i = 0; i < SMALL_ITEMS; i++) s += v[i];
    int64_t tot;
    int64_t ex = block_exclusive_scan<int64_t>(s, lds, &tot);
    int32_t o[SMALL_ITEMS];
#pragma unroll
    for (int i = 0; i < SMALL_ITEMS; i++) {
        o[i] = (int32_t)ex;
        ex += v[i];
    }
    if (vec) {
#pragma unroll
        for (int i = 0; i < SMALL_ITEMS; i += 4) *(int4 *)(data + base + i) = make_int4(o[i], o[i + 1], o[i + 2], o[i + 3]);
    } else {
#pragma unroll
        for (int i = 0; i < SMALL_ITEMS; i++)
            if (base + i < n) data[base + i] = o[i];
    }
    if (threadIdx.x == 0) *total = tot;
}

void scan_exclusive_i32_dev(gss_ctx ctx, int32_t *data, int64_t n, int64_t *d_total)
{
    if (n <= 0) throw gss_error{GSS_ERR_ARG, "scan: empty array"};
    if (n <= 1024 * SMALL_ITEMS) {
        GSS_LAUNCH_B(8 * n, k_scan_single, dim3(1), dim3(1024), 0, ctx->stream, data, n, d_total);
    } else {
        if (((uintptr_t)data & 15) != 0) throw gss_error{GSS_ERR_ARG, "scan: misaligned array"};
        const int64_t ntiles = (n + SCAN_TILE - 1) / SCAN_TILE;
        uint32_t epoch = 0;
        uint64_t *status = lb_begin(ctx, ntiles, &epoch);
        GSS_LAUNCH_B(8 * n, k_scan_onepass, dim3((unsigned)ntiles), dim3(SCAN_BLOCK), 0, ctx->stream, data, n, ntiles,
                     status, epoch, lb_ticket_ptr(ctx), d_total);
    }
    HIP_OK(hipGetLastError());
}

int64_t scan_exclusive_i32(gss_ctx ctx, int32_t *data, int64_t n, bool want_total)
{
    if (n <= 0) return 0;
    scan_exclusive_i32_dev(ctx, data, n, ctx->d_counters + 14);
    if (!want_total) return -1;
    ctx->readback(&ctx->h_counters[14], ctx->d_counters + 14, sizeof(int64_t));
    return ctx->h_counters[14];
}
