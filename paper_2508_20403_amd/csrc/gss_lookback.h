// gss_lookback.h -- single-pass prefix sums across workgroups by decoupled look-back
// (Merrill and Garland, "Single-pass Parallel Prefix Scan with Decoupled Look-back",
// NVIDIA technical report NVR-2016-002), written for wave64 and used by the scan and
// by the radix-sort scatter.
//
// Each tile owns one status word per counter:
//   bits 63..62  flag: 0 not published, 1 tile aggregate, 2 inclusive prefix
//   bits 61..40  epoch of the launch that wrote it (words of older launches read as
//                unpublished, so the status array is never cleared between launches)
//   bits 39..0   value (counts; every prefix used here is below 2^40)
// Tiles are numbered by a ticket taken when a workgroup starts, so every tile a
// workgroup waits on belongs to a workgroup that is already running; publishing an
// aggregate never waits, hence every wait ends.
#pragma once
#include "gss_dev.h"

#define LB_AGG 1ull
#define LB_INC 2ull
#define LB_EPOCH_BITS 22
#define LB_VALUE_MASK ((1ull << 40) - 1)

__device__ __forceinline__ uint64_t lb_word(uint64_t flag, uint32_t epoch, uint64_t v)
{
    return (flag << 62) | ((uint64_t)epoch << 40) | (v & LB_VALUE_MASK);
}
__device__ __forceinline__ bool lb_ready(uint64_t w, uint32_t epoch)
{
    return (uint32_t)((w >> 40) & ((1u << LB_EPOCH_BITS) - 1)) == epoch;
}
__device__ __forceinline__ void lb_store(uint64_t *p, uint64_t w)
{
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t lb_load(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread per workgroup takes the tile number.  The workgroup holding the last
// ticket puts the counter back to zero: every other workgroup of the launch has taken
// its ticket by then, and the next launch on the stream starts after this one ends.
__device__ __forceinline__ int64_t lb_ticket(unsigned long long *ctr, int64_t ntiles)
{
    unsigned long long t = atomicAdd(ctr, 1ull);
    if (t == (unsigned long long)(ntiles - 1)) atomicExch(ctr, 0ull);
    return (int64_t)t;
}

// Exclusive prefix of tile `tile` >= 1 over tiles [0, tile) for one counter whose
// status words sit `stride` apart; called by a whole wavefront.  Every step inspects
// LB_SPAN = 64 * LB_PER predecessors with independent loads (slot s = q * 64 + lane is
// tile hi - s), so a tile far from the last inclusive prefix still resolves in a few
// round trips: the chain of waits shortens by LB_SPAN tiles per memory latency.
// Returns the same value in every lane.
#define LB_PER 4
#define LB_SPAN (GSS_WAVE * LB_PER)
__device__ __forceinline__ int64_t lb_lookback_wave(const uint64_t *status, int64_t stride, int64_t tile,
                                                    uint32_t epoch)
{
    const int lane = lane_id();
    int64_t excl = 0;
    for (int64_t hi = tile - 1;; hi -= LB_SPAN) {
        uint64_t w[LB_PER];
#pragma unroll
        for (int q = 0; q < LB_PER; q++) {
            const int64_t j = hi - (q * GSS_WAVE + lane);
            w[q] = (j >= 0) ? lb_load(status + j * stride) : 0;
        }
        for (;;) {
            bool ready = true;
#pragma unroll
            for (int q = 0; q < LB_PER; q++) {
                const int64_t j = hi - (q * GSS_WAVE + lane);
                if (j >= 0 && !lb_ready(w[q], epoch)) {
                    ready = false;
                    w[q] = lb_load(status + j * stride);
                }
            }
            if (__ballot(!ready) == 0) break;
            __builtin_amdgcn_s_sleep(4);
        }
        // nearest slot holding an inclusive prefix (tiles before 0 count as inclusive 0)
        int first = LB_SPAN;
#pragma unroll
        for (int q = LB_PER - 1; q >= 0; q--) {
            const int64_t j = hi - (q * GSS_WAVE + lane);
            if (j < 0 || (w[q] >> 62) == LB_INC) first = q * GSS_WAVE + lane;
        }
#pragma unroll
        for (int d = GSS_WAVE / 2; d >= 1; d >>= 1) {
            const int o = __shfl_xor(first, d, GSS_WAVE);
            first = o < first ? o : first;
        }
        int64_t v = 0;
#pragma unroll
        for (int q = 0; q < LB_PER; q++) {
            const int s = q * GSS_WAVE + lane;
            const int64_t j = hi - s;
            if (j >= 0 && s <= first) v += (int64_t)(w[q] & LB_VALUE_MASK);
        }
#pragma unroll
        for (int d = GSS_WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, GSS_WAVE);
        excl += v;
        if (first < LB_SPAN) break;
    }
    return excl;
}

// Exclusive prefix of tile `tile` >= 1 for counter `d`, by one thread, inspecting W
// predecessors per step with independent loads.
template <int W>
__device__ __forceinline__ int64_t lb_lookback_thread(const uint64_t *status, int64_t stride, int64_t d,
                                                      int64_t tile, uint32_t epoch)
{
    int64_t excl = 0;
    for (int64_t hi = tile - 1; hi >= 0; hi -= W) {
        uint64_t w[W];
#pragma unroll
        for (int k = 0; k < W; k++) w[k] = (hi - k >= 0) ? lb_load(status + (hi - k) * stride + d) : 0;
        for (;;) {
            bool all = true;
#pragma unroll
            for (int k = 0; k < W; k++) {
                if (hi - k >= 0 && !lb_ready(w[k], epoch)) {
                    all = false;
                    w[k] = lb_load(status + (hi - k) * stride + d);
                }
            }
            if (all) break;
            __builtin_amdgcn_s_sleep(1);
        }
        bool done = false;
#pragma unroll
        for (int k = 0; k < W; k++) {
            if (!done && hi - k >= 0) {
                excl += (int64_t)(w[k] & LB_VALUE_MASK);
                done = (w[k] >> 62) == LB_INC;
            }
        }
        if (done) break;
    }
    return excl;
}
