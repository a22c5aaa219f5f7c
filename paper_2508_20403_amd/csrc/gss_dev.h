// gss_dev.h -- device helpers of the gfx950 library (not shared with anything else).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GSS_WAVE 64
#define GSS_END (-1)

// ------------------------------------------------------------------------------------
// 128-bit unsigned integers (two's complement wrap-around, exact)
// ------------------------------------------------------------------------------------
struct u128 {
    uint64_t lo, hi;
};

__host__ __device__ __forceinline__ u128 mk128(uint64_t lo, uint64_t hi)
{
    u128 r;
    r.lo = lo;
    r.hi = hi;
    return r;
}
__host__ __device__ __forceinline__ u128 add128(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1ull : 0ull);
    return r;
}
__host__ __device__ __forceinline__ u128 sub128(u128 a, u128 b)
{
    u128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1ull : 0ull);
    return r;
}
__host__ __device__ __forceinline__ u128 neg128(u128 a) { return sub128(mk128(0, 0), a); }
// m << s for s in [0, 127)
__host__ __device__ __forceinline__ u128 shl128(uint64_t m, int s)
{
    if (s == 0) return mk128(m, 0);
    if (s < 64) return mk128(m << s, m >> (64 - s));
    return mk128(0, m << (s - 64));
}

// per-vertex record read by the per-edge kernel with one 32-byte gather
struct VRec {
    u128 D;          // root resistance in fixed point (units of 2^scale)
    int32_t first;   // preorder index (root 0)
    int32_t depth;   // hops from the root
    int32_t parent;  // -1 at the root
    int32_t pad;
};

// Fixed-point term of a positive normal double t: t = mant * 2^(e-52); returns
// mant << (e - emin), i.e. t in units of 2^(emin-52).  Requires e - emin in [0, 74].
__device__ __forceinline__ u128 fixed_term(double t, int emin)
{
    uint64_t b = (uint64_t)__double_as_longlong(t);
    int e = (int)((b >> 52) & 0x7ff) - 1023;
    uint64_t mant = (b & ((1ull << 52) - 1)) | (1ull << 52);
    return shl128(mant, e - emin);
}

// Correctly rounded (round half to even) conversion of x * 2^scale to double for
// 0 < x < 2^127.  Returns false when the result is not a finite normal double.
__device__ __forceinline__ bool u128_to_double_rne(u128 x, int scale, double *out)
{
    int top;  // index of the most significant set bit
    if (x.hi) top = 127 - __clzll((long long)x.hi);
    else if (x.lo) top = 63 - __clzll((long long)x.lo);
    else {
        *out = 0.0;
        return false;
    }
    uint64_t mant;  // 53 significant bits, bit 52 set
    int sh = top - 52;  // value = mant * 2^sh (before rounding)
    if (sh <= 0) {
        mant = x.lo << (-sh);
    } else {
        // keep bits [top .. sh]; the rest decide the rounding
        u128 y;
        if (sh >= 64) y = mk128(x.hi >> (sh - 64), 0);
        else y = mk128((x.lo >> sh) | (sh ? (x.hi << (64 - sh)) : 0), x.hi >> sh);
        mant = y.lo;
        // remainder r = x mod 2^sh ; half = 2^(sh-1)
        bool above_half, exact_half;
        int hb = sh - 1;  // bit index of the half point
        uint64_t hbit, below;
        if (hb >= 64) {
            hbit = (x.hi >> (hb - 64)) & 1ull;
            uint64_t mask_hi = (hb - 64) ? ((1ull << (hb - 64)) - 1) : 0ull;
            below = (x.hi & mask_hi) | x.lo;
        } else {
            hbit = (x.lo >> hb) & 1ull;
            below = hb ? (x.lo & ((1ull << hb) - 1)) : 0ull;
        }
        above_half = hbit && below;
        exact_half = hbit && !below;
        if (above_half || (exact_half && (mant & 1ull))) {
            mant += 1;
            if (mant == (1ull << 53)) {
                mant >>= 1;
                sh += 1;
            }
        }
    }
    long long ex = (long long)sh + 52 + (long long)scale;  // unbiased exponent of the result
    if (ex < -1022 || ex > 1023) {
        *out = 0.0;
        return false;
    }
    uint64_t bits = ((uint64_t)(ex + 1023) << 52) | (mant & ((1ull << 52) - 1));
    *out = __longlong_as_double((long long)bits);
    return true;
}

// ------------------------------------------------------------------------------------
// wave helpers (wave64)
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (GSS_WAVE - 1)); }

// Workgroups are dispatched to the 8 XCDs in turn (workgroup b to XCD b mod 8), and every
// XCD has an L2 of its own.  This bijection of [0, G) gives every XCD a contiguous range
// of tiles, so tiles that read each other's neighbourhood (the rows of nearby vertices)
// share an L2 instead of missing in eight.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t G)
{
    constexpr int64_t X = 8;
    const int64_t per = G / X, rem = G % X, xcd = b % X, idx = b / X;
    return (xcd < rem) ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}
__device__ __forceinline__ uint64_t lanemask_lt()
{
    int l = lane_id();
    return l ? ((~0ull) >> (64 - l)) : 0ull;
}

// exclusive prefix sum of v across the block (blockDim.x <= 1024, multiple of 64).
// lds must hold blockDim.x/64 + 1 entries.  Returns the block total in *total.
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T v, T *lds, T *total)
{
    const int lane = lane_id();
    const int wid = threadIdx.x / GSS_WAVE;
    const int nw = blockDim.x / GSS_WAVE;
    T x = v;
#pragma unroll
    for (int d = 1; d < GSS_WAVE; d <<= 1) {
        T y = __shfl_up(x, d, GSS_WAVE);
        if (lane >= d) x += y;
    }
    if (lane == GSS_WAVE - 1) lds[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < nw; i++) {
            T t = lds[i];
            lds[i] = run;
            run += t;
        }
        lds[nw] = run;
    }
    __syncthreads();
    T res = x - v + lds[wid];
    *total = lds[nw];
    __syncthreads();
    return res;
}

// 32-bit mixing hash (Murmur3 finaliser)
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
// 64-bit mixing hash (splitmix64 finaliser)
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    z ^= z >> 31;
    return z;
}

// error flags collected on the device; the host maps them to a status by precedence
enum : uint32_t {
    F_ARG = 1u << 0,
    F_NOT_SIMPLE = 1u << 1,
    F_WEIGHT = 1u << 2,
    F_ASYM = 1u << 3,
    F_NOT_TREE = 1u << 4,
    F_TREE_EDGE = 1u << 5,
    F_RANGE = 1u << 6,
    F_OVERFLOW = 1u << 7,  // an internal buffer was too small (the host retries)
};
