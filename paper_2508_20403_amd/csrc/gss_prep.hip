// gss_prep.hip -- tree preparation on gfx950.
//
// Builds everything the per-edge step needs from a CSR graph and a parent array:
//   * validation flags (simple, symmetric, positive weights, a rooted spanning tree),
//   * edge numbering: the id of {u,v}, u<v, is the rank of entry (u,v) among the
//     upper-triangle CSR entries,
//   * the Euler tour of the tree, ranked by a recursive sparse-ruling-set list ranking
//     that carries (position, depth, root resistance) sums along the walk,
//   * depth, preorder index and the exact root-to-node resistance
//     D(x) = sum over the root->x path of RN(1/w) in 128-bit fixed point
//     (paper: Def. "Resistance distance", eq. RT, resistive weight 1/w),
//   * a two-level in-block-mask RMQ over the preorder sequence of (depth, parent): for
//     vertices u != v with pre(u) < pre(v), the shallowest vertex in preorder positions
//     (pre(u), pre(v)] is a child of LCA(u, v) (every vertex there at that depth is one),
//     so the minimum's parent is the LCA,
//   * the list of off-tree edges in id order.
#include <algorithm>

#include "gss_impl.h"
#include "gss_lookback.h"

#define PB 256          // default block size
#define ENT_ITEMS 16    // CSR entries per thread in entry-parallel kernels
#ifndef RULE_RATE0
#define RULE_RATE0 8    // level 0 of the list ranking: one ruler per ~RULE_RATE0 arcs (power of two)
#endif
#ifndef RULE_RATE
#define RULE_RATE 8     // upper levels: one ruler per ~RULE_RATE elements (power of two)
#endif
#define BASE_MAX 4096   // lists this short are ranked by one workgroup
#define BASE_THREADS 1024

// ------------------------------------------------------------------------------------
// small device helpers
// ------------------------------------------------------------------------------------
// row u with row_ptr[u] <= k < row_ptr[u+1]  (largest u with row_ptr[u] <= k)
__device__ __forceinline__ int32_t row_of(const int32_t *__restrict__ row_ptr, int32_t n, int64_t k)
{
    int32_t lo = 0, hi = n;  // invariant: row_ptr[lo] <= k, answer in [lo, hi)
    while (hi - lo > 1) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)row_ptr[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// index of key in the sorted range col[lo,hi), or -1
__device__ __forceinline__ int64_t clamp_idx(int64_t x, int64_t lo, int64_t hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

// Position of key in the sorted columns [lo, hi), or -1.  Long rows are first narrowed
// by interpolation between the end columns (a few steps on rows whose columns spread
// evenly, as hub rows of relabelled graphs do; at most four, so skewed rows cost no more
// than four extra loads), then bisected.
__device__ __forceinline__ int64_t find_in_row(const int32_t *__restrict__ col, int64_t lo, int64_t hi,
                                               int32_t key)
{
    const int64_t end = hi;
    if (hi - lo > 32) {
        int32_t a = col[lo], b = col[hi - 1];
        for (int step = 0; step < 4 && hi - lo > 32; step++) {
            if (key < a || key > b) return -1;
            // a <= key <= b: a guess inside [lo, hi)
            const int64_t mid = clamp_idx(
                lo + (int64_t)((double)(key - a) / ((double)(b - a) + 1.0) * (double)(hi - lo)), lo, hi - 1);
            const int32_t c = col[mid];
            if (c == key) return mid;
            if (c < key) {
                lo = mid + 1;
                a = col[lo];  // lo < hi: c < key <= b = col[hi - 1]
            } else {
                hi = mid;
                b = col[hi - 1];  // hi > lo: a <= key < c
            }
        }
    }
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (col[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && col[lo] == key) ? lo : -1;
}

// ------------------------------------------------------------------------------------
// entry tiles: a block owns ETILE consecutive CSR entries; the row of every entry of the
// tile is written to LDS once, so threads then walk the entries coalesced (entry
// base + i*PB + tid).  Reads of row_ptr are clamped so malformed input stays in bounds.
// ------------------------------------------------------------------------------------
#define ETILE (PB * ENT_ITEMS)
#define CK_TREE 0x80000000u  // in a sorted lower-entry key: the column is the row's parent


// tile_row[b] = the row holding entry b*ETILE: one thread per row marks the tiles that
// start inside it (row_ptr reads are clamped, so malformed input yields wrong but
// in-range rows).  With `validate`, the same pass checks row_ptr: row_ptr[0] = 0,
// non-decreasing, row_ptr[n] = nnz, every entry in [0, nnz].
__global__ void k_tile_rows(const int32_t *__restrict__ row_ptr, int32_t n, int64_t nnz, int64_t ntiles,
                            int32_t *__restrict__ tile_row, int validate, uint32_t *flags)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (validate) {
        bool bad = false;
        if (x <= n) {
            if (x == 0 && row_ptr[0] != 0) bad = true;
            if (x < n && row_ptr[x + 1] < row_ptr[x]) bad = true;
            if (x == n && (int64_t)row_ptr[n] != nnz) bad = true;
            if ((int64_t)row_ptr[x] < 0 || (int64_t)row_ptr[x] > nnz) bad = true;
        }
        if (__ballot(bad) && lane_id() == 0) atomicOr(flags, F_ARG);
    }
    if (x >= n || ntiles == 0) return;
    const int64_t lo = clamp_idx(row_ptr[x], 0, nnz), hi = clamp_idx(row_ptr[x + 1], 0, nnz);
    if (hi <= lo) return;
    const int64_t b1 = (hi - 1) / ETILE;
    for (int64_t b = (lo + ETILE - 1) / ETILE; b <= b1 && b < ntiles; b++) tile_row[b] = (int32_t)x;
}

// fills srow[k - base] = row of entry k for the tile starting at base: every row that
// starts inside the tile marks its first entry (LDS max, so the last of several empty
// rows wins), then an inclusive prefix maximum over the tile carries each row to its
// entries.  The work is independent of row lengths (a hub row spanning many tiles costs
// the same as short rows).
// With rs (capacity RS_CAP), rs[r - r0] also receives the tile offset of the start of each
// row r0 < r <= r1 that starts inside the tile, r - r0 < RS_CAP (a row's entries inside the
// tile are then [rs[r - r0], rs[r + 1 - r0]) when both rows start inside it).
#define RS_CAP 1024
__device__ __forceinline__ void load_tile_rows(const int32_t *__restrict__ row_ptr, int32_t n, int64_t nnz,
                                               int64_t base, const int32_t *__restrict__ tile_row, int32_t *srow,
                                               int32_t *rs = nullptr)
{
    constexpr int PER = ETILE / PB;
    __shared__ int32_t s_tmax[PB / GSS_WAVE];
    const int64_t b = base / ETILE;
    const int64_t ntiles = (nnz + ETILE - 1) / ETILE;
    int32_t r0 = tile_row[b];
    int32_t r1 = (b + 1 < ntiles) ? tile_row[b + 1] : n - 1;
    r0 = r0 < 0 ? 0 : (r0 > n - 1 ? n - 1 : r0);
    r1 = r1 < r0 ? r0 : (r1 > n - 1 ? n - 1 : r1);
    for (int i = threadIdx.x; i < ETILE; i += PB) srow[i] = r0;
    __syncthreads();
    for (int32_t r = r0 + 1 + threadIdx.x; r <= r1; r += PB) {
        const int64_t k = row_ptr[r];
        if (k >= base && k < base + ETILE) {
            atomicMax(&srow[k - base], r);
            if (rs && r - r0 < RS_CAP) rs[r - r0] = (int32_t)(k - base);
        }
    }
    __syncthreads();
    // inclusive prefix maximum: thread t owns entries [PER t, PER t + PER)
    int32_t v[PER];
    int32_t run = 0;
#pragma unroll
    for (int i = 0; i < PER; i++) {
        v[i] = srow[threadIdx.x * PER + i];
        run = v[i] > run ? v[i] : run;
        v[i] = run;
    }
    int32_t x = run;  // inclusive max across threads, then shifted to exclusive
#pragma unroll
    for (int d = 1; d < GSS_WAVE; d <<= 1) {
        const int32_t y = __shfl_up(x, d, GSS_WAVE);
        if (lane_id() >= d) x = y > x ? y : x;
    }
    if (lane_id() == GSS_WAVE - 1) s_tmax[threadIdx.x / GSS_WAVE] = x;
    int32_t ex = __shfl_up(x, 1, GSS_WAVE);
    if (lane_id() == 0) ex = r0;
    __syncthreads();
    for (int w = 0; w < (int)(threadIdx.x / GSS_WAVE); w++) ex = s_tmax[w] > ex ? s_tmax[w] : ex;
#pragma unroll
    for (int i = 0; i < PER; i++) srow[threadIdx.x * PER + i] = v[i] > ex ? v[i] : ex;
    __syncthreads();
}


// CSR checks: column range, strictly increasing rows, no self-loops, positive finite
// weights, and per tile the number of upper minus lower entries.  With *mode = 0 it also
// checks symmetry exactly by a mirror search: every lower entry (u, c), c < u, must find
// (c, u) in row c with the same weight; with equally many entries in both triangles,
// mirroring (injective) is then a bijection between them, so every upper entry has its
// mirror too.  With *mode = 1 the transpose comparison (k_sym_compare) checks symmetry
// instead.  Memory-safe on any input: rows are clamped.
// The distant mirror rows (more than RS_CAP rows before the tile) usually form one short
// row range (on a grid, the rows one layer back): when its columns fit the LDS that held
// the tile's row indices, they are loaded there in one coalesced pass and searched like
// the tile's own rows; the near ones (the previous tile's rows) are searched in memory.
__global__ __launch_bounds__(PB) void k_check_entries(const int32_t *__restrict__ row_ptr,
                                                      const int32_t *__restrict__ col,
                                                      const double *__restrict__ w, int32_t n, int64_t nnz,
                                                      const int32_t *__restrict__ tile_row, uint32_t *flags,
                                                      int64_t *__restrict__ bpart, const int64_t *__restrict__ mode)
{
    __shared__ int32_t srow[ETILE];
    __shared__ int32_t scol[ETILE];
    __shared__ int32_t s_rs[RS_CAP];
    const bool search = *mode == 0;
    __shared__ int64_t sh[PB / GSS_WAVE];
    __shared__ int32_t s_prev[2];  // row and column of entry base-1 (-1 if none)
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = tile * ETILE;
    // every global load of the tile is issued before any is used
    int32_t cv[ENT_ITEMS];
    double wv[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        cv[i] = k < nnz ? col[k] : -1;
        wv[i] = k < nnz ? w[k] : 1.0;
    }
    if (threadIdx.x == 0) {
        s_prev[0] = -1;
        s_prev[1] = -1;
        if (base > 0) {
            const int32_t r0 = tile_row[tile];
            const int32_t rc = r0 < 0 ? 0 : (r0 > n - 1 ? n - 1 : r0);
            // entry base-1 lies in row r0 exactly when that row starts before the tile
            if ((int64_t)row_ptr[rc] < base) s_prev[0] = rc;
            s_prev[1] = col[base - 1];
        }
    }
    load_tile_rows(row_ptr, n, nnz, base, tile_row, srow, search ? s_rs : nullptr);  // synchronises
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) scol[i * PB + threadIdx.x] = cv[i];
    __syncthreads();
    // rows r0 < r < r_last lie wholly inside the tile: their starts are in s_rs
    const int32_t nloc = (int32_t)min((int64_t)ETILE, nnz - base);
    const int32_t r0 = srow[0];
    const int32_t r_last = srow[nloc - 1];
    uint32_t f = 0;
    int64_t bal = 0;  // upper minus lower entries
    int32_t uv[ENT_ITEMS];  // row of each entry (srow's LDS is reused for the far rows below)
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        uv[i] = k < nnz ? srow[k - base] : 0;
        if (k >= nnz) continue;
        const int32_t u = uv[i];
        const int32_t c = cv[i];
        if (c < 0 || c >= n) {
            f |= F_ARG;
            continue;
        }
        if (c == u) f |= F_NOT_SIMPLE;
        // columns strictly increase within a row
        const bool prev_same = (k > base) ? (srow[k - 1 - base] == u) : (s_prev[0] == u);
        const int32_t pcol = (k > base) ? scol[k - 1 - base] : s_prev[1];
        if (prev_same && pcol >= c) f |= F_NOT_SIMPLE;
        const double x = wv[i];
        if (!(x > 0.0) || !isfinite(x)) f |= F_WEIGHT;
        bal += (c > u) ? 1 : (c < u ? -1 : 0);
    }
    if (search) {
        // The mirror (c, u) of every lower entry (u, c) is searched in row c.  A row lying
        // wholly inside the tile (r0 < c < r_last, its start within RS_CAP rows of r0) is
        // bisected in LDS; so is a row of the far range [f0, f1] of the other mirror rows
        // when that range was loaded; any other row in global memory, the searches of eight
        // entries in lockstep so that their loads overlap.  lo/hi bisect the row for the
        // first column >= u (tile or far-range offsets for a row in LDS, CSR positions
        // otherwise).  Row bounds are clamped so malformed input stays in bounds.
        auto in_tile = [&](int32_t c) { return c > r0 && c < r_last && c + 1 - r0 < RS_CAP; };
        __shared__ int32_t s_far[2];
        __shared__ int32_t s_frs[RS_CAP];  // far-range row starts, offsets from flo
        // the far range's columns go to srow (the tile's rows are in uv now)
        if (threadIdx.x == 0) {
            s_far[0] = 0x7fffffff;
            s_far[1] = -1;
        }
        int32_t fmn = 0x7fffffff, fmx = -1;
#pragma unroll
        for (int i = 0; i < ENT_ITEMS; i++) {
            const int64_t k = base + (int64_t)i * PB + threadIdx.x;
            const int32_t c = cv[i];
            if (k < nnz && c >= 0 && c < uv[i] && c < r0 - RS_CAP) {  // the distant mirror rows
                fmn = min(fmn, c);
                fmx = max(fmx, c);
            }
        }
        for (int d = 32; d > 0; d >>= 1) {
            fmn = min(fmn, __shfl_xor(fmn, d, GSS_WAVE));
            fmx = max(fmx, __shfl_xor(fmx, d, GSS_WAVE));
        }
        __syncthreads();  // the rows in srow are no longer read; s_far initialised
        if (lane_id() == 0 && fmx >= 0) {
            atomicMin(&s_far[0], fmn);
            atomicMax(&s_far[1], fmx);
        }
        __syncthreads();
        const int32_t f0 = s_far[0], f1 = s_far[1];  // uniform across the workgroup
        int64_t flo = 0;
        int32_t fcnt = 0;
        bool far_lds = false;
        if (f1 >= 0 && f1 - f0 + 2 <= RS_CAP) {  // columns are in [0, n), so f1 + 1 <= n
            // the range's first ETILE entries; a row is searched in LDS when it ends within them
            flo = clamp_idx(row_ptr[f0], 0, nnz);
            const int64_t fhi = clamp_idx(row_ptr[f1 + 1], flo, nnz);
            far_lds = true;
            fcnt = (int32_t)min(fhi - flo, (int64_t)ETILE);
            for (int32_t i = threadIdx.x; i < fcnt; i += PB) srow[i] = col[flo + i];
            for (int32_t r = threadIdx.x; r <= f1 + 1 - f0; r += PB)
                s_frs[r] = (int32_t)(clamp_idx(row_ptr[f0 + r], flo, fhi) - flo);
            __syncthreads();
        }
        constexpr int MB = 8;
#pragma unroll 1
        for (int h = 0; h < ENT_ITEMS; h += MB) {
            int32_t lo[MB], hi[MB], end[MB], key[MB];
            uint32_t inlds = 0, infar = 0;
#pragma unroll
            for (int q = 0; q < MB; q++) {
                const int64_t k = base + (int64_t)(h + q) * PB + threadIdx.x;
                lo[q] = hi[q] = end[q] = 0;
                key[q] = -1;
                if (k >= nnz) continue;
                const int32_t u = uv[h + q];
                const int32_t c = cv[h + q];
                if (c < 0 || c >= u) continue;  // not a lower entry (or out of range, flagged above)
                key[q] = u;
                if (in_tile(c)) {
                    // (clamped to the tile: on a malformed row_ptr, which the row checks flag,
                    // the starts may be stale)
                    inlds |= 1u << q;
                    lo[q] = min(max(s_rs[c - r0], 0), nloc);
                    hi[q] = end[q] = min(max(s_rs[c + 1 - r0], lo[q]), nloc);
                } else if (far_lds && c >= f0 && c <= f1 && s_frs[c + 1 - f0] <= fcnt) {
                    infar |= 1u << q;
                    lo[q] = min(max(s_frs[c - f0], 0), fcnt);
                    hi[q] = end[q] = min(max(s_frs[c + 1 - f0], lo[q]), fcnt);
                } else {
                    lo[q] = (int32_t)clamp_idx(row_ptr[c], 0, nnz);
                    hi[q] = end[q] = (int32_t)clamp_idx(row_ptr[c + 1], lo[q], nnz);
                }
            }
            for (;;) {
                bool busy = false;
#pragma unroll
                for (int q = 0; q < MB; q++) {
                    if (key[q] >= 0 && lo[q] < hi[q]) {
                        const int32_t mid = lo[q] + ((hi[q] - lo[q]) >> 1);
                        int32_t cm;
                        if (((inlds | infar) >> q) & 1u) {
                            const int32_t *lds = ((inlds >> q) & 1u) ? scol : srow;
                            cm = lds[mid];
                        } else {
                            cm = col[mid];
                        }
                        if (cm < key[q]) lo[q] = mid + 1;
                        else hi[q] = mid;
                        busy = true;
                    }
                }
                if (!__any(busy)) break;
            }
#pragma unroll
            for (int q = 0; q < MB; q++) {
                if (key[q] < 0) continue;
                const bool loc = (inlds >> q) & 1u, far = (infar >> q) & 1u;
                const int64_t pos = loc ? base + lo[q] : far ? flo + lo[q] : (int64_t)lo[q];
                int32_t cf = -1;
                if (lo[q] < end[q]) {
                    if (loc || far) {
                        const int32_t *lds = loc ? scol : srow;
                        cf = lds[lo[q]];
                    } else {
                        cf = col[pos];
                    }
                }
                if (cf != key[q] || w[pos] != wv[h + q]) f |= F_ASYM;
            }
        }
    }
    for (int d = 32; d > 0; d >>= 1) {
        f |= __shfl_xor(f, d, GSS_WAVE);
        bal += __shfl_xor(bal, d, GSS_WAVE);
    }
    if (lane_id() == 0) {
        sh[threadIdx.x / GSS_WAVE] = bal;
        if (f) atomicOr(flags, f);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < PB / GSS_WAVE; i++) bal += sh[i];
        bpart[tile] = bal;  // per-tile partial sums (no contended atomics)
    }
}

// sums the per-block balances (upper minus lower entries) of k_check_entries into *total
__global__ __launch_bounds__(1024) void k_balance_total(const int64_t *__restrict__ bpart, int64_t nblk,
                                                        int64_t *total)
{
    __shared__ int64_t s1[1024 / GSS_WAVE];
    int64_t a = 0;
    for (int64_t i = threadIdx.x; i < nblk; i += 1024) a += bpart[i];
    for (int d = 32; d > 0; d >>= 1) a += __shfl_xor(a, d, GSS_WAVE);
    if (lane_id() == 0) s1[threadIdx.x / GSS_WAVE] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 1024 / GSS_WAVE; i++) a += s1[i];
        *total = a;
    }
}

// start values of the preparation's flags and counters (one launch instead of a copy
// and several fills): roots, smallest root, exponent range, tree edges found, off-tree
// and upper-entry totals, triangle balance
__global__ void k_prep_init(uint32_t *flags, int64_t *counters, int32_t n)
{
    if (threadIdx.x == 0) {
        *flags = 0;
        counters[0] = 0;
        counters[1] = n;
        counters[2] = (int64_t)1 << 40;
        counters[3] = -((int64_t)1 << 40);
        counters[4] = 0;
        counters[5] = 0;
        counters[6] = 0;
        counters[7] = 0;
        counters[9] = 0;
        counters[10] = 0;
        counters[13] = 0;
    }
}

// child counts to zero, first children and tree-edge positions to -1
__global__ void k_tree_init(int32_t *__restrict__ ccnt, int32_t *__restrict__ fc, int32_t *__restrict__ tpos,
                            int32_t n)
{
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) {
        ccnt[x] = 0;
        fc[x] = -1;
        tpos[x] = -1;
    }
}

// Tree edges found from the child's side: the entry (x, c) of row x with c = parent[x] is
// the tree edge of x.  Its position and resistance 1/w are recorded (tpos[x], tinv[x]).
// Per tile: the number of tree edges found and the exponent range of their resistances,
// written to part[tile] (no atomics on shared words; k_tree_total combines them).  One
// streaming pass over the columns; a weight is read only where an entry matches.
// Memory-safe on any input: rows are clamped and parent values are only compared.
__global__ __launch_bounds__(PB) void k_tree_entries(const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col,
                                                     const double *__restrict__ w,
                                                     const int32_t *__restrict__ parent, int32_t n, int64_t nnz,
                                                     const int32_t *__restrict__ tile_row,
                                                     int32_t *__restrict__ tpos, double *__restrict__ tinv,
                                                     int4 *__restrict__ part, int2 *__restrict__ remote)
{
    __shared__ int32_t srow[ETILE];
    __shared__ int32_t sred[4][PB / GSS_WAVE];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t base = tile * ETILE;
    int32_t cv[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        cv[i] = k < nnz ? col[k] : -1;
    }
    load_tile_rows(row_ptr, n, nnz, base, tile_row, srow);  // synchronises
    int32_t pu[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) pu[i] = cv[i] >= 0 ? parent[srow[i * PB + threadIdx.x]] : -1;
    // In one tile of eight: the lower entries, and those whose column lies outside the
    // tile's rows (their mirror rows are not in the tile); the sample chooses how
    // symmetry is checked.
    const int32_t nloc = (int32_t)min((int64_t)ETILE, nnz - base);
    const int32_t r0 = srow[0], r_last = srow[nloc - 1];
    int far = 0, low = 0;
    if ((tile & 7) == 0) {
#pragma unroll
        for (int i = 0; i < ENT_ITEMS; i++) {
            const int32_t u = srow[i * PB + threadIdx.x];
            const bool lower = cv[i] >= 0 && cv[i] < u;
            low += lower ? 1 : 0;
            far += (lower && (cv[i] < r0 || cv[i] > r_last)) ? 1 : 0;
        }
    }
    uint32_t f = 0;
    int found = 0;
    int emin = 1 << 30, emax = -(1 << 30);
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        if (cv[i] < 0 || cv[i] != pu[i]) continue;
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        const int32_t x = srow[i * PB + threadIdx.x];
        found++;
        const double t = 1.0 / w[k];
        tpos[x] = (int32_t)k;
        tinv[x] = t;
        const int ef = (int)(((uint64_t)__double_as_longlong(t) >> 52) & 0x7ff);
        if (ef == 0 || ef == 0x7ff) {
            f |= F_RANGE;
        } else {
            emin = min(emin, ef - 1023);
            emax = max(emax, ef - 1023);
        }
    }
    for (int d = 32; d > 0; d >>= 1) {
        f |= __shfl_xor(f, d, GSS_WAVE);
        found += __shfl_xor(found, d, GSS_WAVE);
        far += __shfl_xor(far, d, GSS_WAVE);
        low += __shfl_xor(low, d, GSS_WAVE);
        emin = min(emin, __shfl_xor(emin, d, GSS_WAVE));
        emax = max(emax, __shfl_xor(emax, d, GSS_WAVE));
    }
    const int wid = threadIdx.x / GSS_WAVE;
    __shared__ int32_t s_far[2][PB / GSS_WAVE];
    if (lane_id() == 0) {
        sred[0][wid] = (int32_t)f;
        sred[1][wid] = found;
        sred[2][wid] = emin;
        sred[3][wid] = emax;
        s_far[0][wid] = far;
        s_far[1][wid] = low;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < PB / GSS_WAVE; i++) {
            f |= (uint32_t)sred[0][i];
            found += sred[1][i];
            emin = min(emin, sred[2][i]);
            emax = max(emax, sred[3][i]);
            far += s_far[0][i];
            low += s_far[1][i];
        }
        part[tile] = make_int4((int32_t)f, found, emin, emax);
        remote[tile] = make_int2(far, low);
    }
}

// combines the per-tile results of k_tree_entries: flags, the number of tree edges found
// (counters[4]), the exponent range (counters[2], counters[3]), the sampled lower entries
// (counters[6]) and those among them whose column lies outside their tile's rows
// (counters[5]), and the symmetry method they choose (counters[7]: 1 = transposition)
__global__ __launch_bounds__(1024) void k_tree_total(const int4 *__restrict__ part, const int2 *__restrict__ remote,
                                                     int64_t ntiles, uint32_t *flags, int64_t *counters)
{
    __shared__ int32_t sred[4][1024 / GSS_WAVE];
    __shared__ int64_t s_far[2][1024 / GSS_WAVE];
    uint32_t f = 0;
    int64_t found = 0, far = 0, low = 0;
    int emin = 1 << 30, emax = -(1 << 30);
    for (int64_t i = threadIdx.x; i < ntiles; i += 1024) {
        const int4 p = part[i];
        f |= (uint32_t)p.x;
        found += p.y;
        far += remote[i].x;
        low += remote[i].y;
        emin = min(emin, p.z);
        emax = max(emax, p.w);
    }
    for (int d = 32; d > 0; d >>= 1) {
        f |= __shfl_xor(f, d, GSS_WAVE);
        found += __shfl_xor(found, d, GSS_WAVE);
        far += __shfl_xor(far, d, GSS_WAVE);
        low += __shfl_xor(low, d, GSS_WAVE);
        emin = min(emin, __shfl_xor(emin, d, GSS_WAVE));
        emax = max(emax, __shfl_xor(emax, d, GSS_WAVE));
    }
    const int wid = threadIdx.x / GSS_WAVE;
    if (lane_id() == 0) {
        sred[0][wid] = (int32_t)f;
        sred[1][wid] = (int32_t)found;  // per wave below 2^31: at most n tree edges
        sred[2][wid] = emin;
        sred[3][wid] = emax;
        s_far[0][wid] = far;
        s_far[1][wid] = low;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 1024 / GSS_WAVE; i++) {
            f |= (uint32_t)sred[0][i];
            found += sred[1][i];
            far += s_far[0][i];
            low += s_far[1][i];
            emin = min(emin, sred[2][i]);
            emax = max(emax, sred[3][i]);
        }
        if (f) atomicOr(flags, f);
        counters[4] = found;
        counters[5] = far;
        counters[6] = low;
        counters[7] = 2 * far > low ? 1 : 0;  // symmetry by transposition (else mirror search)
        if (emin <= emax) {
            counters[2] = emin;
            counters[3] = emax;
        }
    }
}

// The vertex passes.  LINK = false: parent checks and roots, which the first host wait
// reads (counter atomics only where there is something to count: the root's block, or an
// error).  LINK = true: child counts and the children of every vertex as a list linked by
// atomic exchange (fc[p] = the child that linked itself last, nsib[x] = the child linked
// before x; the order of siblings is immaterial to every later result), enqueued after
// the read-back so that it runs while the host waits.  One vertex per thread, so every
// thread's exchange is in flight at once.
template <bool LINK>
__global__ __launch_bounds__(PB) void k_tree_vertices(const int32_t *__restrict__ parent, int32_t n,
                                                      int32_t *__restrict__ ccnt, int32_t *__restrict__ fc,
                                                      int32_t *__restrict__ nsib, uint32_t *flags, int64_t *counters)
{
    const int64_t xx = xcd_tile(blockIdx.x, gridDim.x) * PB + threadIdx.x;
    if (xx >= n) return;
    const int32_t x = (int32_t)xx;
    const int32_t p = parent[x];
    if (!LINK) {
        if (p == -1) {
            atomicAdd((unsigned long long *)&counters[0], 1ull);
            atomicMin((long long *)&counters[1], (long long)x);
        } else if (p < 0 || p >= n || p == x) {
            atomicOr(flags, F_NOT_TREE);
        }
        return;
    }
    int32_t s = -1;
    if (p >= 0 && p < n && p != x) {
        atomicAdd(&ccnt[p], 1);
        s = atomicExch(&fc[p], x);
    }
    nsib[x] = s;
}

// Per-vertex tour record of level 0 of the list ranking: the successors of both arcs
// of x (arc 2x = down(parent x -> x), arc 2x+1 = up(x -> parent x)), the parent, the
// tree degree and the fixed-point resistance term of the tree edge (x, parent x), so
// one 32-byte load serves a step of the walk whichever arc it is on.
struct __attribute__((aligned(32))) TRec {
    int32_t nd, nu, par, deg;
    u128 t;
};

// What the tree passes' counters say about the tour: the root (counters[1], the smallest
// root; n when there is none), the exponent range of the resistances (counters[2], [3]),
// the tree edges found (counters[4], against need).  The fixed-point terms are used when
// no resistance is out of range (F_RANGE), every tree edge was found and the range is at
// most 74 (else zero terms; the host reports the error); their exact 127-bit sum is
// checked when the range exceeds 44 (every term is below 2^(53 + range) and there are
// fewer than 2^30 of them, so below that their sum, a bound on every root resistance,
// stays below 2^127).  The same rule as the host's, read on the device, so the tour can
// be built before the host has read the counters.
struct TermsInfo {
    int32_t root;
    int emin;
    bool ok, sums;
};
__device__ __forceinline__ TermsInfo terms_info(const int64_t *counters, const uint32_t *flags, int64_t need,
                                                int32_t n)
{
    TermsInfo r;
    r.root = (int32_t)counters[1];
    int64_t emin = counters[2], emax = counters[3];
    if (n == 1) emin = emax = 0;
    const bool missing = counters[4] != need;
    const bool range_bad = (__hip_atomic_load(flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & F_RANGE) != 0 ||
                           (!missing && emax - emin > 74);
    r.ok = !range_bad && !missing;
    if (!r.ok) emin = emax = 0;
    r.emin = (int)emin;
    r.sums = r.ok && emax - emin > 44;
    return r;
}

// Tour records, the successor array of the arcs (read by the ruler selection) and, when
// the exact sum of the terms is needed, the per-block sums for the 127-bit range check.
// Successors: the down arc into x continues with the down arc into its first child, or
// returns (up arc of x); the up arc of x continues with the down arc into its next
// sibling, or the up arc of its parent, or ends the tour when the parent is the root (or
// is no vertex: a parent array that is no tree, which the host rejects, still gives
// successors inside the arcs).  The root's arcs are not on the tour (-2).  Every read
// is a coalesced per-vertex load (the children lists are linked through the vertices
// themselves).
__global__ __launch_bounds__(PB) void k_tour_rec(const int32_t *__restrict__ tpos, const double *__restrict__ tinv,
                                                 const int32_t *__restrict__ parent,
                                                 const int32_t *__restrict__ ccnt, const int32_t *__restrict__ fc,
                                                 const int32_t *__restrict__ nsib, int32_t n,
                                                 const int64_t *__restrict__ counters, const uint32_t *flags,
                                                 int64_t need, TRec *__restrict__ trec, int32_t *__restrict__ succ,
                                                 u128 *__restrict__ bsum, uint64_t *__restrict__ bcarry)
{
    __shared__ uint64_t slo[PB], shi[PB], sc[PB];
    const TermsInfo ti = terms_info(counters, flags, need, n);
    const int32_t root = ti.root;
    int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    u128 t = mk128(0, 0);
    if (x < n) {
        if (ti.ok && x != root && tpos[x] >= 0) t = fixed_term(tinv[x], ti.emin);
        const int32_t c = fc[x];
        TRec e;
        e.par = parent[x];
        e.deg = ccnt[x];
        e.t = t;
        if (x == root) {
            e.nd = -2;
            e.nu = -2;
        } else {
            e.nd = (c >= 0) ? 2 * c : 2 * x + 1;
            const int32_t s = nsib[x];
            if (s >= 0) e.nu = 2 * s;
            else if (e.par == root || e.par < 0 || e.par >= n || e.par == x) e.nu = GSS_END;
            else e.nu = 2 * e.par + 1;
        }
        trec[x] = e;
        *(int2 *)(succ + 2 * (int64_t)x) = make_int2(e.nd, e.nu);
    }
    if (!ti.sums) return;
    slo[threadIdx.x] = t.lo;
    shi[threadIdx.x] = t.hi;
    sc[threadIdx.x] = 0;
    __syncthreads();
    for (int s = PB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            u128 a = mk128(slo[threadIdx.x], shi[threadIdx.x]);
            u128 b = mk128(slo[threadIdx.x + s], shi[threadIdx.x + s]);
            u128 r = add128(a, b);
            uint64_t c = sc[threadIdx.x] + sc[threadIdx.x + s];
            if (r.hi < a.hi || (r.hi == a.hi && r.lo < a.lo)) c++;
            slo[threadIdx.x] = r.lo;
            shi[threadIdx.x] = r.hi;
            sc[threadIdx.x] = c;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = mk128(slo[0], shi[0]);
        bcarry[blockIdx.x] = sc[0];
    }
}

__global__ __launch_bounds__(1024) void k_terms_total(const u128 *__restrict__ bsum,
                                                      const uint64_t *__restrict__ bcarry, int64_t nb,
                                                      uint32_t *flags, const int64_t *__restrict__ counters,
                                                      int64_t need, int32_t n)
{
    if (!terms_info(counters, flags, need, n).sums) return;  // the sum is bounded anyway
    __shared__ uint64_t slo[1024], shi[1024], sc[1024];
    u128 s = mk128(0, 0);
    uint64_t c = 0;
    for (int64_t i = threadIdx.x; i < nb; i += 1024) {
        u128 r = add128(s, bsum[i]);
        if (r.hi < s.hi || (r.hi == s.hi && r.lo < s.lo)) c++;
        c += bcarry[i];
        s = r;
    }
    slo[threadIdx.x] = s.lo;
    shi[threadIdx.x] = s.hi;
    sc[threadIdx.x] = c;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            u128 a = mk128(slo[threadIdx.x], shi[threadIdx.x]);
            u128 b = mk128(slo[threadIdx.x + h], shi[threadIdx.x + h]);
            u128 r = add128(a, b);
            uint64_t cc = sc[threadIdx.x] + sc[threadIdx.x + h];
            if (r.hi < a.hi || (r.hi == a.hi && r.lo < a.lo)) cc++;
            slo[threadIdx.x] = r.lo;
            shi[threadIdx.x] = r.hi;
            sc[threadIdx.x] = cc;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && (sc[0] != 0 || (shi[0] >> 63))) atomicOr(flags, F_RANGE);
}

// ------------------------------------------------------------------------------------
// list ranking
// ------------------------------------------------------------------------------------
struct LVal {
    int32_t cnt, dep;
    u128 D;
};
__device__ __forceinline__ LVal lv_add(LVal a, LVal b)
{
    LVal r;
    r.cnt = a.cnt + b.cnt;
    r.dep = a.dep + b.dep;
    r.D = add128(a.D, b.D);
    return r;
}
__device__ __forceinline__ LVal lv_sub(LVal a, LVal b)
{
    LVal r;
    r.cnt = a.cnt - b.cnt;
    r.dep = a.dep - b.dep;
    r.D = sub128(a.D, b.D);
    return r;
}
__device__ __forceinline__ LVal lv_zero()
{
    LVal r;
    r.cnt = 0;
    r.dep = 0;
    r.D = mk128(0, 0);
    return r;
}

// element of an upper level of the list ranking (a ruler of the level below): its
// successor and its sublist sum in one 32-byte record, so a step of a walk is one load
struct __attribute__((aligned(32))) LRec {
    int32_t nxt, cnt, dep, pad;
    u128 D;
};
__device__ __forceinline__ LRec lrec(int32_t nxt, const LVal &v)
{
    LRec r;
    r.nxt = nxt;
    r.cnt = v.cnt;
    r.dep = v.dep;
    r.pad = 0;
    r.D = v.D;
    return r;
}
__device__ __forceinline__ void lv_acc(LVal &acc, const LRec &e)
{
    acc.cnt += e.cnt;
    acc.dep += e.dep;
    acc.D = add128(acc.D, e.D);
}

__device__ __forceinline__ bool is_ruler(int32_t i, int32_t head, int32_t level)
{
    return i == head || (mix32((uint32_t)i * 0x9E3779B9u + (uint32_t)level * 0x7F4A7C15u) &
                         ((level == 0 ? RULE_RATE0 : RULE_RATE) - 1)) == 0;
}

// level-0 step: adds arc i (of vertex i>>1, whose tour record is e) to acc and
// returns the arc's successor
__device__ __forceinline__ int32_t arc_step(int32_t i, const TRec &e, LVal &acc)
{
    acc.cnt += 1;
    if (i & 1) {
        acc.dep -= 1;
        acc.D = sub128(acc.D, e.t);
        return e.nu;
    }
    acc.dep += 1;
    acc.D = add128(acc.D, e.t);
    return e.nd;
}

// The list ranking runs without host round trips: every level's length and head live
// in device memory, and each level's buffers are sized by a capacity (1.3x the expected
// ruler count plus a margin).  A level that outgrows its capacity raises F_OVERFLOW and
// the host repeats the ranking with larger capacities.
//
// Level l: elements i < N_l with successor nxt[i] (GSS_END ends the list, -2 = not in
// the list) and value val(i).  Rulers (the head and a hashed 1/RULE_RATE sample) walk
// their sublists once; the sublist sums and the next rulers form the level l+1 list.
// Level 0 (the 2n arcs, read from the per-vertex tour records) keeps nothing per arc:
// once level 1 is ranked, every ruler walks its sublist again from its prefix and writes
// the vertex records and the LCA sequence directly.  Upper levels record for every
// element its ruler (owner) and the exclusive sum of the sublist before it (loc), and
// their way down is the coalesced pass rpre[owner] + loc.

// Ruler selection and numbering in one pass (a stream compaction with decoupled
// look-back): rid[i] = number of rulers before i (written for rulers only), relem[rid] =
// i, the level length R_{l+1} and head; owner[i] = -1 for every element when an owner
// array is given (upper levels).  Thread t of
// round r owns the four consecutive elements at tile offset 4 (r*256 + t).
#define RC_BLOCK 256
#define RC_ROUNDS 4
#define RC_TILE (RC_BLOCK * 4 * RC_ROUNDS)
__global__ __launch_bounds__(RC_BLOCK) void k_ruler_compact(int64_t cap, int64_t ntiles, const int64_t *__restrict__ Np,
                                                           const int32_t *__restrict__ nxt,
                                                           const int32_t *__restrict__ headp, int32_t level,
                                                           int32_t *__restrict__ rid, int32_t *__restrict__ owner,
                                                           int32_t *__restrict__ relem, int64_t cap_next,
                                                           int32_t *__restrict__ head_next, int64_t *__restrict__ R_out,
                                                           uint64_t *__restrict__ status, uint32_t epoch,
                                                           unsigned long long *ticket, uint32_t *flags)
{
    constexpr int NW = RC_BLOCK / GSS_WAVE;
    __shared__ int32_t s_wsum[RC_ROUNDS][NW];
    __shared__ int64_t s_tile, s_excl;
    const int lane = lane_id(), wid = threadIdx.x / GSS_WAVE;
    if (threadIdx.x == 0) s_tile = lb_ticket(ticket, ntiles);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t Nr = *Np;
    const int64_t N = Nr < cap ? Nr : cap;  // a longer list has already raised F_OVERFLOW
    const int32_t head = *headp;
    const int64_t base = tile * RC_TILE;
    uint32_t fl[RC_ROUNDS];
    int32_t incl[RC_ROUNDS];
#pragma unroll
    for (int r = 0; r < RC_ROUNDS; r++) {
        const int64_t e = base + ((int64_t)r * RC_BLOCK + threadIdx.x) * 4;
        int nx[4];
        if (e + 4 <= N) {
            const int4 v = *(const int4 *)(nxt + e);
            nx[0] = v.x;
            nx[1] = v.y;
            nx[2] = v.z;
            nx[3] = v.w;
            if (owner) *(int4 *)(owner + e) = make_int4(-1, -1, -1, -1);
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                nx[q] = (e + q < N) ? nxt[e + q] : -2;
                if (owner && e + q < N) owner[e + q] = -1;
            }
        }
        uint32_t f = 0;
#pragma unroll
        for (int q = 0; q < 4; q++)
            if (nx[q] != -2 && is_ruler((int32_t)(e + q), head, level)) f |= 1u << q;
        fl[r] = f;
        int32_t x = __popc(f);
#pragma unroll
        for (int d = 1; d < GSS_WAVE; d <<= 1) {
            const int32_t y = __shfl_up(x, d, GSS_WAVE);
            if (lane >= d) x += y;
        }
        incl[r] = x;
        if (lane == GSS_WAVE - 1) s_wsum[r][wid] = x;
    }
    __syncthreads();
    int64_t off[RC_ROUNDS];
    int64_t run = 0;
#pragma unroll
    for (int r = 0; r < RC_ROUNDS; r++) {
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
            if (tile == ntiles - 1) *R_out = excl + tile_total;
        }
    }
    __syncthreads();
    const int64_t excl = s_excl;
#pragma unroll
    for (int r = 0; r < RC_ROUNDS; r++) {
        const int64_t e = base + ((int64_t)r * RC_BLOCK + threadIdx.x) * 4;
        int64_t p = excl + off[r] + incl[r] - __popc(fl[r]);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if ((fl[r] >> q) & 1u) {
                const int64_t i = e + q;
                rid[i] = (int32_t)p;
                if (p < cap_next) relem[p] = (int32_t)i;
                else atomicOr(flags, F_OVERFLOW);
                if (i == head) *head_next = (int32_t)p;
                p++;
            }
        }
    }
}

// level-0 walk: one thread per ruler r < R_1; per arc one tour-record load, nothing
// written; per ruler the sublist sum and the next ruler
__global__ __launch_bounds__(PB) void k_walk0(int64_t cap_next, const int64_t *__restrict__ Rp,
                                              const int32_t *__restrict__ relem, const int32_t *__restrict__ rid,
                                              const TRec *__restrict__ trec, const int32_t *__restrict__ headp,
                                              int64_t N, int32_t *__restrict__ rnxt, LRec *__restrict__ rrec,
                                              uint32_t *flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= cap_next || r >= *Rp) return;
    const int32_t head = *headp;
    int32_t i = relem[r];
    LVal acc = lv_zero();
    int32_t j;
    for (int64_t steps = 0;; steps++) {
        const TRec e = trec[i >> 1];
        j = arc_step(i, e, acc);
        if (j < 0 || is_ruler(j, head, 0)) break;
        if (steps > N) {  // a cycle without rulers beyond this one: not a tree
            atomicOr(flags, F_NOT_TREE);
            j = GSS_END;
            break;
        }
        i = j;
    }
    int32_t nr = (j < 0) ? GSS_END : rid[j];
    if (nr >= cap_next) nr = GSS_END;  // overflow, already flagged by k_ruler_compact
    rnxt[r] = nr;
    rrec[r] = lrec(nr, acc);
}

// level-0 way down: ruler r walks its sublist again from its exclusive prefix rpre[r].
// The down arc into x is the (arcs before it + 1)-th step of the tour, and x's preorder
// index is (that position + depth(x)) / 2; it writes x's vertex record (depth, preorder
// index, exact root resistance, parent, tree degree) and the LCA sequence entry
// epk[pre(x)] = depth(x) << 32 | parent(x).  A valid tour reaches every vertex; the
// base level checks that it holds all 2(n-1) arcs.
__global__ __launch_bounds__(PB) void k_walk0_down(int64_t cap_next, const int64_t *__restrict__ Rp,
                                                   const int32_t *__restrict__ relem, const TRec *__restrict__ trec,
                                                   const LVal *__restrict__ rpre, const int32_t *__restrict__ headp,
                                                   int64_t N, int32_t n, VRec *__restrict__ vrec,
                                                   uint64_t *__restrict__ epk, uint32_t *flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= cap_next || r >= *Rp) return;
    const int32_t head = *headp;
    int32_t i = relem[r];
    LVal acc = rpre[r];
    for (int64_t steps = 0;; steps++) {
        const TRec e = trec[i >> 1];
        const int32_t pos = acc.cnt + 1;
        const int32_t j = arc_step(i, e, acc);
        if (!(i & 1)) {
            const int32_t x = i >> 1;
            const int32_t pre = (pos + acc.dep) >> 1;
            if (pos < 1 || pre < 1 || pre >= n) {
                atomicOr(flags, F_NOT_TREE);
                break;
            }
            VRec v;
            v.D = acc.D;
            v.first = pre;
            v.depth = acc.dep;
            v.parent = e.par;
            v.pad = e.deg;
            vrec[x] = v;
            epk[pre] = ((uint64_t)(uint32_t)acc.dep << 32) | (uint32_t)e.par;
        }
        if (j < 0 || is_ruler(j, head, 0) || steps > N) break;
        i = j;
    }
}

// upper-level walk (level l >= 1): one thread per ruler r < R_{l+1}; per element one
// record load, its owner and local prefix written; per ruler the next level's record
__global__ __launch_bounds__(PB) void k_walk1(int64_t cap_next, const int64_t *__restrict__ Rp,
                                              const int32_t *__restrict__ relem, const int32_t *__restrict__ rid,
                                              const LRec *__restrict__ rec, const int32_t *__restrict__ headp,
                                              int32_t level, int64_t N, int32_t *__restrict__ owner,
                                              LVal *__restrict__ loc, int32_t *__restrict__ rnxt,
                                              LRec *__restrict__ rrec, uint32_t *flags)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= cap_next || r >= *Rp) return;
    const int32_t head = *headp;
    int32_t i = relem[r];
    LVal acc = lv_zero();
    int32_t j;
    for (int64_t steps = 0;; steps++) {
        const LRec e = rec[i];
        owner[i] = (int32_t)r;
        loc[i] = acc;
        lv_acc(acc, e);
        j = e.nxt;
        if (j < 0 || is_ruler(j, head, level)) break;
        if (steps > N) {  // a cycle without rulers beyond this one: not a tree
            atomicOr(flags, F_NOT_TREE);
            j = GSS_END;
            break;
        }
        i = j;
    }
    int32_t nr = (j < 0) ? GSS_END : rid[j];
    if (nr >= cap_next) nr = GSS_END;  // overflow, already flagged by k_ruler_compact
    rnxt[r] = nr;
    rrec[r] = lrec(nr, acc);
}

// base case: Wyllie pointer jumping in LDS, exclusive prefix from the head; every thread
// owns BASE_MAX / BASE_THREADS elements
__global__ __launch_bounds__(BASE_THREADS) void k_rank_base(const int64_t *__restrict__ Np, int64_t cap,
                                                            const int32_t *__restrict__ nxt,
                                                            const LRec *__restrict__ rec,
                                                            const int32_t *__restrict__ headp, int64_t expect,
                                                            LVal *__restrict__ pre, uint32_t *flags)
{
    constexpr int PER = BASE_MAX / BASE_THREADS;
    __shared__ int32_t snx[BASE_MAX];
    __shared__ LVal ssuf[BASE_MAX];
    const int64_t N64 = *Np;
    if (N64 > BASE_MAX || N64 > cap) {  // uniform across the workgroup
        if (threadIdx.x == 0) atomicOr(flags, F_OVERFLOW);
        return;
    }
    const int32_t N = (int32_t)N64;
    const int32_t head = *headp;
    for (int32_t i = threadIdx.x; i < N; i += BASE_THREADS) {
        snx[i] = nxt[i];
        const LRec e = rec[i];
        ssuf[i].cnt = e.cnt;
        ssuf[i].dep = e.dep;
        ssuf[i].D = e.D;
    }
    __syncthreads();
    int rounds = 1;
    while ((1 << rounds) < N + 1) rounds++;
    rounds += 1;
    for (int r = 0; r < rounds; r++) {
        int32_t nxv[PER];
        LVal add[PER];
        bool upd[PER];
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int32_t i = threadIdx.x + k * BASE_THREADS;
            nxv[k] = -1;
            add[k] = lv_zero();
            upd[k] = false;
            if (i < N) {
                int32_t nx = snx[i];
                if (nx >= 0) {
                    add[k] = ssuf[nx];
                    upd[k] = true;
                    nx = snx[nx];
                }
                nxv[k] = nx;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PER; k++) {
            const int32_t i = threadIdx.x + k * BASE_THREADS;
            if (upd[k]) {
                ssuf[i] = lv_add(ssuf[i], add[k]);
                snx[i] = nxv[k];
            }
        }
        __syncthreads();
    }
    for (int32_t i = threadIdx.x; i < N; i += BASE_THREADS)
        if (snx[i] >= 0) atomicOr(flags, F_NOT_TREE);
    // the tour from the head must hold every arc: fewer means some vertices never reach
    // the root through their parents (a cycle)
    if (threadIdx.x == 0 && (head < 0 || head >= N || ssuf[head].cnt != expect)) atomicOr(flags, F_NOT_TREE);
    __syncthreads();
    if (head >= 0 && head < N)
        for (int32_t i = threadIdx.x; i < N; i += BASE_THREADS) pre[i] = lv_sub(ssuf[head], ssuf[i]);
}

// downward pass, levels >= 1: pre[i] = rpre[owner[i]] + loc[i]
__global__ void k_rank_apply(int64_t cap, const int64_t *__restrict__ Np, const int32_t *__restrict__ owner,
                             const LVal *__restrict__ loc, const LVal *__restrict__ rpre, LVal *__restrict__ pre)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cap || i >= *Np) return;
    const int32_t o = owner[i];
    pre[i] = (o >= 0) ? lv_add(rpre[o], loc[i]) : lv_zero();
}

__global__ void k_level_init(int64_t N0, const int64_t *__restrict__ head0, int nlev, int64_t *__restrict__ len,
                             int32_t *__restrict__ heads)
{
    for (int l = threadIdx.x; l <= nlev; l += blockDim.x) {
        len[l] = (l == 0) ? N0 : 0;
        heads[l] = (l == 0) ? (int32_t)*head0 : -1;
    }
}

// mult: the attempt's capacity multiplier (1, 2, 4 or 8); div: a divisor of the first
// attempt's capacities (1 normally; larger values drive the capacity retry in tests)
static inline int64_t next_cap(int64_t cap, int mult, int div, int level)
{
    const int64_t rate = level == 0 ? RULE_RATE0 : RULE_RATE;
    return cap * mult * 21 / (rate * 16 * div) + 256;  // 1.3125x the expected ruler count
}

// Ranks the Euler tour (succ over N = 2n arcs, tour records trec, head arc in *d_head)
// and emits vrec / epk.  Returns without a host round trip; F_OVERFLOW in the flags asks
// for a retry with a larger capacity multiplier.
static void euler_rank(gss_ctx ctx, gss_tree t, const int32_t *succ, const TRec *trec, const int64_t *d_head,
                       int mult, std::vector<void *> &bufs)
{
    hipStream_t st = ctx->stream;
    const int32_t n = t->n;
    const int64_t N0 = 2 * (int64_t)n;
    struct Lv {
        int64_t cap;
        const int32_t *nxt;    // successors (ruler selection, base level)
        const LRec *rec;       // records (levels >= 1)
        const int32_t *headp;
        const int64_t *Np;
        LVal *pre;             // exclusive prefixes (levels >= 1)
        int32_t *relem;        // this level's rulers
        int32_t *owner;        // ruler of each element (levels >= 1)
        LVal *loc;             // sum of the element's sublist before it (levels >= 1)
    };
    // device scalars: level lengths and heads
    const int max_levels = 40;
    int64_t *d_len = ctx->alloc<int64_t>(max_levels + 1);
    int32_t *d_heads = ctx->alloc<int32_t>(max_levels + 1);
    bufs.push_back(d_len);
    bufs.push_back(d_heads);
    GSS_LAUNCH(k_level_init, dim3(1), dim3(64), 0, st, N0, d_head, max_levels, d_len, d_heads);
    std::vector<Lv> lv;
    lv.push_back(Lv{N0, succ, nullptr, d_heads, d_len, nullptr, nullptr, nullptr, nullptr});
    // upward: build levels until the capacity fits one workgroup
    for (int l = 0; l == 0 || lv.back().cap > BASE_MAX; l++) {
        if (l + 1 >= max_levels) throw gss_error{GSS_ERR_HIP, "list ranking: too many levels"};
        Lv &a = lv.back();
        const int64_t cap = a.cap;
        const int64_t cap2 = std::min<int64_t>(next_cap(cap, mult, ctx->rank_cap_div, l), cap);
        int32_t *rid = ctx->alloc<int32_t>(cap + 1);
        a.relem = ctx->alloc<int32_t>(cap2 + 1);
        int32_t *rnxt = ctx->alloc<int32_t>(cap2 + 1);
        LRec *rrec = ctx->alloc<LRec>(cap2 + 1);
        for (void *p : {(void *)rid, (void *)a.relem, (void *)rnxt, (void *)rrec}) bufs.push_back(p);
        if (l > 0) {
            a.owner = ctx->alloc<int32_t>(cap + 1);
            a.loc = ctx->alloc<LVal>(cap + 1);
            bufs.push_back(a.owner);
            bufs.push_back(a.loc);
        }
        const int64_t ntiles = (cap + RC_TILE - 1) / RC_TILE;
        uint32_t epoch = 0;
        uint64_t *status = lb_begin(ctx, ntiles, &epoch);
        // successor read (and owner cleared) per element; rid and relem written per ruler
        GSS_LAUNCH_B((l == 0 ? 4 : 8) * cap + 8 * cap2, k_ruler_compact, dim3((unsigned)ntiles), dim3(RC_BLOCK), 0,
                     st, cap, ntiles, a.Np, a.nxt, a.headp, l, rid, a.owner, a.relem, cap2, d_heads + l + 1,
                     d_len + l + 1, status, epoch, lb_ticket_ptr(ctx), ctx->d_flags);
        // one record per element (level 0: a vertex's tour record serves both of its
        // arcs; upper levels also write the element's owner and local prefix); per ruler
        // its successor and record
        if (l == 0)
            GSS_LAUNCH_B(16 * N0 + 44 * cap2, k_walk0, dim3(grid_for(cap2, PB)), dim3(PB), 0, st, cap2, d_len + 1,
                         a.relem, rid, trec, a.headp, N0, rnxt, rrec, ctx->d_flags);
        else
            GSS_LAUNCH_B(60 * cap + 44 * cap2, k_walk1, dim3(grid_for(cap2, PB)), dim3(PB), 0, st, cap2,
                         d_len + l + 1, a.relem, rid, a.rec, a.headp, l, cap, a.owner, a.loc, rnxt, rrec,
                         ctx->d_flags);
        lv.push_back(Lv{cap2, rnxt, rrec, d_heads + l + 1, d_len + l + 1, nullptr, nullptr, nullptr, nullptr});
    }
    // base level
    Lv &b = lv.back();
    b.pre = ctx->alloc<LVal>(b.cap + 1);
    bufs.push_back(b.pre);
    GSS_LAUNCH(k_rank_base, dim3(1), dim3(BASE_THREADS), 0, st, b.Np, b.cap, b.nxt, b.rec, b.headp, N0 - 2, b.pre,
               ctx->d_flags);
    // downward
    for (int l = (int)lv.size() - 2; l >= 1; l--) {
        Lv &a = lv[l];
        a.pre = ctx->alloc<LVal>(a.cap + 1);
        bufs.push_back(a.pre);
        GSS_LAUNCH_B(4 * a.cap + 24 * a.cap + 24 * lv[l + 1].cap + 24 * a.cap, k_rank_apply,
                     dim3(grid_for(a.cap, PB)), dim3(PB), 0, st, a.cap, a.Np, a.owner, a.loc, lv[l + 1].pre, a.pre);
    }
    if (lv.size() == 1) throw gss_error{GSS_ERR_HIP, "list ranking: tour shorter than one workgroup"};
    // level 0: per arc its tour record read; per vertex a 32-byte record and its LCA
    // sequence entry; per ruler its prefix
    const int64_t cap1 = lv[1].cap;
    GSS_LAUNCH_B(16 * N0 + 4 * N0 + 16 * N0 + 28 * cap1, k_walk0_down, dim3(grid_for(cap1, PB)), dim3(PB), 0, st,
                 cap1, d_len + 1, lv[0].relem, trec, lv[1].pre, d_heads, N0, n, t->vrec, t->epk, ctx->d_flags);
    HIP_OK(hipGetLastError());
}

// ------------------------------------------------------------------------------------
// RMQ over the preorder LCA sequence: blocks of 64 positions, superblocks of 64 blocks
// ------------------------------------------------------------------------------------
// One wave handles a run of up to 64 packed values, lane i holding value i (+inf past
// the end).  Lane i computes: mask = positions q <= i whose value is strictly smaller
// than every value in (q, i] (so the lowest set bit at or above a start s is the
// position of the minimum of [s, i]); the prefix minimum of [0, i]; the suffix minimum
// of [i, run end].
//
// The mask is the chain i, psv(i), psv(psv(i)), ... of previous strictly smaller values
// (mask(i) = {i} + mask(psv(i))).  psv comes from binary lifting over window minima
// that end at each lane, and the chain union from six pointer-doubling steps, all with
// lane permutes: about 170 instructions per run instead of a 64-step scan per lane.
__device__ __forceinline__ uint64_t bperm64(uint64_t v, int src)
{
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)v);
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(uint32_t)(v >> 32));
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ void wave_run(uint64_t v, uint64_t &mask, uint64_t &pre, uint64_t &suf)
{
    const int lane = lane_id();
    // win[k] = minimum of the (up to) 2^k values ending at this lane
    uint64_t win[6];
    win[0] = v;
#pragma unroll
    for (int k = 1; k < 6; k++) {
        const int h = 1 << (k - 1);
        const uint64_t y = __shfl_up(win[k - 1], h, GSS_WAVE);
        win[k] = (lane >= h && y < win[k - 1]) ? y : win[k - 1];
    }
    // previous strictly smaller value: skip maximal windows whose minimum is >= v
    int pos = lane - 1;
#pragma unroll
    for (int k = 5; k >= 0; k--) {
        const uint64_t t = bperm64(win[k], pos > 0 ? pos : 0);
        if (pos >= 0 && t >= v) pos -= 1 << k;
    }
    int j = pos >= 0 ? pos : -1;
    uint64_t m = 1ull << lane;
#pragma unroll
    for (int s = 0; s < 6; s++) {
        const int src = j > 0 ? j : 0;
        const uint64_t mj = bperm64(m, src);
        const int jj = __builtin_amdgcn_ds_bpermute(src << 2, j);
        if (j >= 0) {
            m |= mj;
            j = jj;
        }
    }
    mask = m;
    pre = v;
    suf = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        uint64_t a = __shfl_up(pre, d, GSS_WAVE);
        if (lane >= d) pre = a < pre ? a : pre;
        uint64_t b = __shfl_down(suf, d, GSS_WAVE);
        if (lane + d < 64) suf = b < suf ? b : suf;
    }
}

#define RMQ_WPB 4
// positions -> blocks of 64: masks, prefix and suffix minima, block minima
__global__ __launch_bounds__(RMQ_WPB * 64) void k_rmq_blocks(const uint64_t *__restrict__ epk, int32_t L,
                                                             uint64_t *__restrict__ pmask,
                                                             uint64_t *__restrict__ ppre,
                                                             uint64_t *__restrict__ psuf,
                                                             uint64_t *__restrict__ bmin, int32_t nb)
{
    const int lane = lane_id();
    int32_t b = blockIdx.x * RMQ_WPB + threadIdx.x / 64;
    if (b >= nb) return;  // whole wave
    int32_t p = b * 64 + lane;
    int32_t cnt = min(64, L - b * 64);
    uint64_t v = (lane < cnt) ? epk[p] : ~0ull;
    uint64_t mask, pre, suf;
    wave_run(v, mask, pre, suf);
    if (lane < cnt) {
        pmask[p] = mask;
        ppre[p] = pre;
        psuf[p] = suf;
    }
    if (lane == cnt - 1) bmin[b] = pre;
}

// blocks -> superblocks of 64 blocks: the same over block minima
__global__ __launch_bounds__(RMQ_WPB * 64) void k_rmq_super(const uint64_t *__restrict__ bmin, int32_t nb,
                                                            uint64_t *__restrict__ bmask,
                                                            uint64_t *__restrict__ bpre,
                                                            uint64_t *__restrict__ bsuf,
                                                            uint64_t *__restrict__ sb0, int32_t nsb)
{
    const int lane = lane_id();
    int32_t s = blockIdx.x * RMQ_WPB + threadIdx.x / 64;
    if (s >= nsb) return;
    int32_t b = s * 64 + lane;
    int32_t cnt = min(64, nb - s * 64);
    uint64_t v = (lane < cnt) ? bmin[b] : ~0ull;
    uint64_t mask, pre, suf;
    wave_run(v, mask, pre, suf);
    if (lane < cnt) {
        bmask[b] = mask;
        bpre[b] = pre;
        bsuf[b] = suf;
    }
    if (lane == cnt - 1) sb0[s] = pre;
}

__global__ __launch_bounds__(1024) void k_rmq_sparse(uint64_t *__restrict__ st, int32_t nsb,
                                                     int32_t levels)
{
    for (int32_t k = 1; k < levels; k++) {
        const uint64_t *prev = st + (int64_t)(k - 1) * nsb;
        uint64_t *cur = st + (int64_t)k * nsb;
        int32_t half = 1 << (k - 1);
        for (int32_t i = threadIdx.x; i + 2 * half <= nsb; i += blockDim.x) {
            uint64_t a = prev[i], b = prev[i + half];
            cur[i] = a < b ? a : b;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// edge numbering, off-tree edges (id order) and tree edge ids
// ------------------------------------------------------------------------------------
// The id of edge {u, v}, u < v, is the rank of the upper entry (u, v) among all upper
// entries in CSR order; an upper entry is a tree edge when parent[u] = v or parent[v] =
// u.  One pass with decoupled look-back: every tile counts its upper and its off-tree
// upper entries, takes the counts of the tiles before it from their published status
// (two counters, wave 0 and wave 1 look back in parallel), ranks both kinds inside the
// tile in entry order (round, wave, lane), writes every off-tree edge's id, endpoints
// and weight at its place, and gives each tree edge's id to the child endpoint
// (tree_eid).  The last tile writes both totals.  With lkey and *mode = 1 (symmetry by
// transposition) it only numbers the edges: every lower entry (u, c), c < u, is written
// at its rank among the lower entries (its position minus the upper entries before it)
// as the key c << 32 | u (bit 31: c is u's parent) and its weight, ubase[tile] receives
// the
// tile's first edge id: the transpose check sorts the lower entries by column and
// compares them with the upper ones.  Memory-safe on any input: rows are clamped, output
// places are bounded by Mcap (F_TREE_EDGE beyond it) and by Lcap (F_ASYM beyond it:
// more lower entries than half of all), and parent values are only compared.
__global__ __launch_bounds__(PB) void k_off_write(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ w,
    const int32_t *__restrict__ parent, int32_t n, int64_t nnz, int64_t ntiles, const int32_t *__restrict__ tile_row,
    int64_t Mcap, int32_t *__restrict__ off_id, int32_t *__restrict__ off_u, int32_t *__restrict__ off_v,
    double *__restrict__ off_w, const int32_t *__restrict__ vbase, int32_t G, int32_t *__restrict__ off_g,
    int32_t *__restrict__ tree_eid, uint64_t *__restrict__ status, uint32_t epoch, unsigned long long *ticket,
    int64_t *__restrict__ m_total, int64_t *__restrict__ off_total, uint32_t *flags, int64_t Lcap,
    uint64_t *__restrict__ lkey, double *__restrict__ lw, int32_t *__restrict__ ubase,
    const int64_t *__restrict__ mode)
{
    constexpr int NW = PB / GSS_WAVE;
    static_assert(ENT_ITEMS * NW <= GSS_WAVE, "one wave scans the piece counts");
    __shared__ int32_t srow[ETILE];
    __shared__ int32_t s_cnt[2][ENT_ITEMS][NW];
    __shared__ int64_t s_off[2][ENT_ITEMS][NW];
    __shared__ int64_t s_tile, s_ex[2];
    const int lane = lane_id(), wid = threadIdx.x / GSS_WAVE;
    if (threadIdx.x == 0) s_tile = lb_ticket(ticket, ntiles);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * ETILE;
    int32_t cv[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        cv[i] = k < nnz ? col[k] : -1;
    }
    load_tile_rows(row_ptr, n, nnz, base, tile_row, srow);  // synchronises
    // Under transposition the off-tree edges are placed after the sort (k_sym_compare),
    // which also tells which upper entries are their column vertex's tree edge: no
    // gather of the column's parent here.
    const bool defer = lkey && *mode == 1;
    int32_t pu[ENT_ITEMS], pc[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int32_t u = srow[i * PB + threadIdx.x];
        const bool up = cv[i] > u && cv[i] < n;  // k >= nnz has cv = -1
        const bool low = cv[i] >= 0 && cv[i] < u;
        pu[i] = (up || (defer && low)) ? parent[u] : -1;
        pc[i] = (up && !defer) ? parent[cv[i]] : -1;
    }
    uint64_t um[ENT_ITEMS], om[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int32_t u = srow[i * PB + threadIdx.x];
        const bool up = cv[i] > u && cv[i] < n;
        um[i] = __ballot(up);
        om[i] = __ballot(!defer && up && pu[i] != cv[i] && pc[i] != u);
        if (lane == 0) {
            s_cnt[0][i][wid] = __popcll(um[i]);
            s_cnt[1][i][wid] = __popcll(om[i]);
        }
    }
    __syncthreads();
    // wave 0 handles the upper entries, wave 1 the off-tree ones: exclusive offsets of the
    // (round, wave) pieces inside the tile, then the tile's place among the tiles before it
    if (wid < 2) {
        const int i = lane / NW, w2 = lane % NW;
        const bool has = lane < ENT_ITEMS * NW;
        int64_t x = has ? (int64_t)s_cnt[wid][i][w2] : 0;
        const int64_t own = x;
#pragma unroll
        for (int d = 1; d < GSS_WAVE; d <<= 1) {
            const int64_t y = __shfl_up(x, d, GSS_WAVE);
            if (lane >= d) x += y;
        }
        if (has) s_off[wid][i][w2] = x - own;
        const int64_t tot = __shfl(x, GSS_WAVE - 1, GSS_WAVE);
        int64_t excl = 0;
        if (tile == 0) {
            if (lane == 0) lb_store(status + wid, lb_word(LB_INC, epoch, (uint64_t)tot));
        } else {
            if (lane == 0) lb_store(status + 2 * tile + wid, lb_word(LB_AGG, epoch, (uint64_t)tot));
            excl = lb_lookback_wave(status + wid, 2, tile, epoch);
            if (lane == 0) lb_store(status + 2 * tile + wid, lb_word(LB_INC, epoch, (uint64_t)(excl + tot)));
        }
        if (lane == 0) {
            s_ex[wid] = excl;
            if (tile == ntiles - 1 && (wid == 0 || !defer)) *(wid == 0 ? m_total : off_total) = excl + tot;
        }
    }
    // batches: the graphs of the tile's first and last rows bound every entry's graph
    // (usually one graph per tile, so no per-entry search)
    __shared__ int32_t s_glo, s_ghi;
    if (off_g && wid == 2 && lane < 2) {
        const int64_t last = min((int64_t)ETILE, nnz - base) - 1;
        const int32_t u = srow[lane == 0 ? 0 : last];
        int32_t lo = 0, hi = G;  // vbase[lo] <= u < vbase[hi]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (vbase[mid] <= u) lo = mid;
            else hi = mid;
        }
        if (lane == 0) s_glo = lo;
        else s_ghi = lo;
    }
    __syncthreads();
    const uint64_t lt = lanemask_lt();
    const int64_t ex_u = s_ex[0], ex_o = s_ex[1];
    if (defer) {
        if (threadIdx.x == 0) ubase[tile] = (int32_t)ex_u;
        // lower entries at their rank: position minus the upper entries before it; bit 31
        // of the key marks the row's own tree edge (column = parent of the row)
#pragma unroll
        for (int i = 0; i < ENT_ITEMS; i++) {
            const int64_t k = base + (int64_t)i * PB + threadIdx.x;
            const int32_t u = srow[i * PB + threadIdx.x];
            if (k >= nnz || cv[i] < 0 || cv[i] >= u) continue;
            const int64_t r = k - (ex_u + s_off[0][i][wid] + __popcll(um[i] & lt));
            if (r < 0 || r >= Lcap) {
                atomicOr(flags, F_ASYM);
                continue;
            }
            lkey[r] = ((uint64_t)(uint32_t)cv[i] << 32) | (pu[i] == cv[i] ? CK_TREE : 0u) | (uint32_t)u;
            lw[r] = w[k];
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        if (!((um[i] >> lane) & 1ull)) continue;
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        const int32_t u = srow[i * PB + threadIdx.x];
        const int32_t id = (int32_t)(ex_u + s_off[0][i][wid] + __popcll(um[i] & lt));
        if (!((om[i] >> lane) & 1ull)) {  // a tree edge: its id goes to the child
            if (pc[i] == u) tree_eid[cv[i]] = id;
            if (pu[i] == cv[i]) tree_eid[u] = id;
            continue;
        }
        const int64_t o = ex_o + s_off[1][i][wid] + __popcll(om[i] & lt);
        if (o >= Mcap) {
            atomicOr(flags, F_TREE_EDGE);  // more off-tree entries than m - n + 1
            continue;
        }
        off_id[o] = id;
        off_u[o] = u;
        off_v[o] = cv[i];
        off_w[o] = w[k];
        if (off_g) {
            int32_t lo = s_glo, hi = s_ghi + 1;  // vbase[lo] <= u < vbase[hi]
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (vbase[mid] <= u) lo = mid;
                else hi = mid;
            }
            off_g[o] = lo;
        }
    }
}

// Transpose comparison (exact symmetry), and the off-tree edges under transposition.
// The lower entries (u, c), c < u, in CSR order are ordered by (u, c); sorted stably by
// column they are ordered by (c, u), the order in which their mirrors (c, u) appear among
// the upper entries, which is edge-id order.  So the graph is symmetric exactly when
// there are as many lower as upper entries (the balance of k_check_entries) and the j-th
// sorted lower entry is (x, c) with weight w for the upper entry (c, x) of weight w with
// id j, for every j (keys c << 32 | x).  The sorted entry also says whether c is x's
// parent (bit 31), so an upper entry (u, v) is a tree edge when parent[u] = v or that bit
// is set: the off-tree edges are written here, in id order (decoupled look-back over
// the tiles for their places), with the tree edge ids.  Memory-safe on any input: rows
// are clamped, ids are bounded by Lcap (F_ASYM beyond it) and places by Mcap.
__global__ __launch_bounds__(PB) void k_sym_compare(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col, const double *__restrict__ w,
    const int32_t *__restrict__ parent, int32_t n, int64_t nnz, int64_t ntiles, const int32_t *__restrict__ tile_row,
    const int32_t *__restrict__ ubase, int64_t Lcap, const uint64_t *__restrict__ lkey,
    const double *__restrict__ lw, int64_t Mcap, int32_t *__restrict__ off_id, int32_t *__restrict__ off_u,
    int32_t *__restrict__ off_v, double *__restrict__ off_w, const int32_t *__restrict__ vbase, int32_t G,
    int32_t *__restrict__ off_g, int32_t *__restrict__ tree_eid, uint64_t *__restrict__ status, uint32_t epoch,
    unsigned long long *ticket, int64_t *__restrict__ off_total, uint32_t *flags)
{
    constexpr int NW = PB / GSS_WAVE;
    static_assert(ENT_ITEMS * NW <= GSS_WAVE, "one wave scans the piece counts");
    __shared__ int32_t srow[ETILE];
    __shared__ int32_t s_cnt[2][ENT_ITEMS][NW];
    __shared__ int32_t s_off[2][ENT_ITEMS][NW];
    __shared__ int64_t s_tile, s_ex;
    __shared__ int32_t s_glo, s_ghi;
    const int lane = lane_id(), wid = threadIdx.x / GSS_WAVE;
    if (threadIdx.x == 0) s_tile = lb_ticket(ticket, ntiles);
    __syncthreads();
    const int64_t tile = s_tile;
    const int64_t base = tile * ETILE;
    int32_t cv[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        cv[i] = k < nnz ? col[k] : -1;
    }
    load_tile_rows(row_ptr, n, nnz, base, tile_row, srow);  // synchronises
    const int64_t ub = ubase[tile];
    uint64_t um[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int32_t u = srow[i * PB + threadIdx.x];
        um[i] = __ballot(cv[i] > u && cv[i] < n);
        if (lane == 0) s_cnt[0][i][wid] = __popcll(um[i]);
    }
    __syncthreads();
    if (wid == 0) {  // the upper entries' ranks inside the tile
        const int i = lane / NW, w2 = lane % NW;
        const bool has = lane < ENT_ITEMS * NW;
        int32_t x = has ? s_cnt[0][i][w2] : 0;
        const int32_t own = x;
#pragma unroll
        for (int d = 1; d < GSS_WAVE; d <<= 1) {
            const int32_t y = __shfl_up(x, d, GSS_WAVE);
            if (lane >= d) x += y;
        }
        if (has) s_off[0][i][w2] = x - own;
    }
    __syncthreads();
    // compare, and classify: off-tree unless parent[u] = v or the mirror's tree bit
    const uint64_t lt = lanemask_lt();
    uint32_t f = 0;
    uint64_t om[ENT_ITEMS];
    int32_t jid[ENT_ITEMS], tchild[ENT_ITEMS];
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        const int32_t u = srow[i * PB + threadIdx.x];
        const bool up = (um[i] >> lane) & 1ull;
        bool off = false;
        jid[i] = -1;
        tchild[i] = -1;
        if (up) {
            const int64_t k = base + (int64_t)i * PB + threadIdx.x;
            const int64_t j = ub + s_off[0][i][wid] + __popcll(um[i] & lt);
            if (j < 0 || j >= Lcap) {
                f |= F_ASYM;
            } else {
                const uint64_t lkv = lkey[j];
                if ((lkv & ~(uint64_t)CK_TREE) != (((uint64_t)(uint32_t)u << 32) | (uint32_t)cv[i]) || lw[j] != w[k])
                    f |= F_ASYM;
                jid[i] = (int32_t)j;
                if (parent[u] == cv[i]) tchild[i] = u;
                else if (lkv & CK_TREE) tchild[i] = cv[i];
                else off = true;
            }
        }
        om[i] = __ballot(off);
        if (lane == 0) s_cnt[1][i][wid] = __popcll(om[i]);
    }
    __syncthreads();
    if (wid == 1) {  // off-tree places: ranks inside the tile, the tile's place by look-back
        const int i = lane / NW, w2 = lane % NW;
        const bool has = lane < ENT_ITEMS * NW;
        int32_t x = has ? s_cnt[1][i][w2] : 0;
        const int32_t own = x;
#pragma unroll
        for (int d = 1; d < GSS_WAVE; d <<= 1) {
            const int32_t y = __shfl_up(x, d, GSS_WAVE);
            if (lane >= d) x += y;
        }
        if (has) s_off[1][i][w2] = x - own;
        const int64_t tot = __shfl(x, GSS_WAVE - 1, GSS_WAVE);
        int64_t excl = 0;
        if (tile == 0) {
            if (lane == 0) lb_store(status, lb_word(LB_INC, epoch, (uint64_t)tot));
        } else {
            if (lane == 0) lb_store(status + tile, lb_word(LB_AGG, epoch, (uint64_t)tot));
            excl = lb_lookback_wave(status, 1, tile, epoch);
            if (lane == 0) lb_store(status + tile, lb_word(LB_INC, epoch, (uint64_t)(excl + tot)));
        }
        if (lane == 0) {
            s_ex = excl;
            if (tile == ntiles - 1) *off_total = excl + tot;
        }
    }
    if (off_g && wid == 2 && lane < 2) {
        const int64_t last = min((int64_t)ETILE, nnz - base) - 1;
        const int32_t u = srow[lane == 0 ? 0 : last];
        int32_t lo = 0, hi = G;  // vbase[lo] <= u < vbase[hi]
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if (vbase[mid] <= u) lo = mid;
            else hi = mid;
        }
        if (lane == 0) s_glo = lo;
        else s_ghi = lo;
    }
    __syncthreads();
    const int64_t ex_o = s_ex;
#pragma unroll
    for (int i = 0; i < ENT_ITEMS; i++) {
        if (jid[i] < 0) continue;
        if (tchild[i] >= 0) {
            tree_eid[tchild[i]] = jid[i];
            continue;
        }
        const int64_t k = base + (int64_t)i * PB + threadIdx.x;
        const int32_t u = srow[i * PB + threadIdx.x];
        const int64_t o = ex_o + s_off[1][i][wid] + __popcll(om[i] & lt);
        if (o >= Mcap) {
            atomicOr(flags, F_TREE_EDGE);  // more off-tree entries than m - n + 1
            continue;
        }
        off_id[o] = jid[i];
        off_u[o] = u;
        off_v[o] = cv[i];
        off_w[o] = w[k];
        if (off_g) {
            int32_t lo = s_glo, hi = s_ghi + 1;  // vbase[lo] <= u < vbase[hi]
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (vbase[mid] <= u) lo = mid;
                else hi = mid;
            }
            off_g[o] = lo;
        }
    }
    for (int d = 32; d > 0; d >>= 1) f |= __shfl_xor(f, d, GSS_WAVE);
    if (lane == 0 && f) atomicOr(flags, f);
}

// the root's vertex record (preorder index 0, depth 0, D = 0, its tree degree), its LCA
// sequence entry (never inside a query range) and the head arc of the tour (the down
// arc into its first child; n > 1); the tour writes every other record
__global__ void k_vrec_root(VRec *vrec, int32_t n, const int64_t *__restrict__ counters, uint64_t *__restrict__ epk,
                            const int32_t *__restrict__ ccnt, const int32_t *__restrict__ fc, int64_t *head)
{
    const int64_t root = counters[1];  // the smallest root; n when there is none
    if (root < 0 || root >= n) {
        *head = -2;  // no tour: the ranking flags the parent array as no tree
        return;
    }
    VRec r;
    r.D = mk128(0, 0);
    r.first = 0;
    r.depth = 0;
    r.parent = -1;
    r.pad = ccnt[root];
    vrec[root] = r;
    epk[0] = (uint64_t)(uint32_t)root;
    if (n > 1) *head = 2 * (int64_t)fc[root];
}


// ------------------------------------------------------------------------------------
// host orchestration
// ------------------------------------------------------------------------------------
static void fail(gss_status s, const char *msg) { throw gss_error{s, msg}; }

void free_tree_arrays(gss_tree t)
{
    gss_ctx c = t->ctx;
    void *ptrs[] = {t->tree_eid, t->vrec,       t->epk,    t->pmask,
                    t->ppre,   t->psuf,   t->bmin,   t->bmask,    t->bpre,       t->bsuf,   t->sbst,
                    t->off_id, t->off_u,  t->off_v,  t->off_w,    t->off_g,      t->d_vbase, t->own_row_ptr,
                    t->own_col, t->own_parent, t->own_w, t->d_obase};
    for (void *p : ptrs) c->free(p);
}

// head of the Euler list: the down arc of the root's first child

void prep_tree(gss_ctx ctx, gss_tree t, uint32_t flags)
{
    hipStream_t st = ctx->stream;
    const int32_t n = t->n;
    const int64_t nnz = t->nnz;
    const bool validate = !(flags & GSS_PREP_TRUSTED);
    GSS_LAUNCH(k_prep_init, dim3(1), dim3(64), 0, st, ctx->d_flags, ctx->d_counters, n);

    // the row at the start of every tile of ETILE entries (and the row_ptr checks)
    const int64_t etiles = nnz > 0 ? (nnz + ETILE - 1) / ETILE : 0;
    int32_t *tile_row = ctx->alloc<int32_t>(etiles + 1);
    if (nnz > 0) fill_bytes(ctx, tile_row, 0, sizeof(int32_t) * (etiles + 1));
    GSS_LAUNCH_B(8 * (int64_t)n, k_tile_rows, dim3(grid_for((int64_t)n + 1, PB)), dim3(PB), 0, st, t->row_ptr, n, nnz,
                 etiles, tile_row, validate ? 1 : 0, ctx->d_flags);
    struct TileRowsFree {
        gss_ctx c;
        int32_t *p;
        ~TileRowsFree() { c->free(p); }
    } tile_row_guard{ctx, tile_row};

    // A symmetric simple graph has m = nnz / 2 edges (with validation the checks below
    // confirm it; trusted input promises it).  The edge count found by the numbering is
    // compared with m at the final synchronisation.
    const int64_t m = nnz / 2;
    t->m = m;
    t->M = m - (n - 1) + (t->virt_root >= 0 ? t->G : 0);
    if (t->M < 0) t->M = 0;  // fewer entries than a tree needs: the counts below fail
    t->off_id = ctx->alloc<int32_t>(t->M + 1);
    t->off_u = ctx->alloc<int32_t>(t->M + 1);
    t->off_v = ctx->alloc<int32_t>(t->M + 1);
    t->off_w = ctx->alloc<double>(t->M + 1);
    t->tree_eid = ctx->alloc<int32_t>(n);
    if (nnz > 0 && (t->G > 1 || t->virt_root >= 0)) t->off_g = ctx->alloc<int32_t>(t->M + 1);

    // tree checks on the context stream: the tree edges from the child's rows, then the
    // parent array (roots, cycles of length one, child lists)
    int32_t *ccnt = ctx->alloc<int32_t>(n);
    int32_t *fc = ctx->alloc<int32_t>(n);
    int32_t *tpos = ctx->alloc<int32_t>(n);
    int32_t *nsib = ctx->alloc<int32_t>(n);
    double *tinv = ctx->alloc<double>(n);
    GSS_LAUNCH(k_tree_init, dim3(grid_for(n, PB)), dim3(PB), 0, st, ccnt, fc, tpos, n);
    if (nnz > 0) {
        int4 *part = ctx->alloc<int4>(etiles);
        int2 *remote = ctx->alloc<int2>(etiles);
        GSS_LAUNCH_B(4 * nnz + 4 * (int64_t)n + 20 * (int64_t)n, k_tree_entries, dim3((unsigned)etiles), dim3(PB),
                     0, st, t->row_ptr, t->col, t->w, t->parent, n, nnz, tile_row, tpos, tinv, part, remote);
        GSS_LAUNCH(k_tree_total, dim3(1), dim3(1024), 0, st, part, remote, etiles, ctx->d_flags, ctx->d_counters);
        ctx->free(part);
        ctx->free(remote);
    }
    GSS_LAUNCH_B(4 * (int64_t)n, k_tree_vertices<false>, dim3(grid_for(n, PB)), dim3(PB), 0, st, t->parent, n, ccnt,
                 fc, nsib, ctx->d_flags, ctx->d_counters);

    struct Transpose {
        uint64_t *lk, *lk2;
        double *lw, *lw2;
        int32_t *ub;
        int64_t Lcap;
    } tr{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    // The auxiliary stream numbers the edges (off-tree edges, tree edge ids) and validates
    // the CSR (entry checks and symmetry) beside the rest of the tree preparation, which
    // waits for it only at its end; everything on the context stream is memory-safe on a
    // malformed CSR.  It starts after the tree passes above (which the first host wait
    // needs), so they have the device to themselves.  Symmetry is checked by mirror
    // search when most lower entries find their mirror row inside their own tile
    // (searched in LDS; grid-like graphs), by transposition (a sort of the lower entries
    // by column, then a streaming comparison) when most mirror rows lie elsewhere (random
    // columns, where every search is a chain of random loads); the tree pass's sample
    // chose, in counters[7], which the kernels read and the host reads at its first wait
    // (the sort and the comparison are enqueued only for transposition).
    {
        AuxScope aux(ctx);
        hipStream_t sa = ctx->stream;
        fill_bytes(ctx, t->tree_eid, 0xFF, sizeof(int32_t) * n);
        if (nnz > 0) {
            uint32_t epoch = 0;
            uint64_t *status = lb_begin(ctx, 2 * etiles, &epoch);
            // transposition: the lower entries (key, weight) at their ranks, and each tile's
            // first edge id
            const int64_t Lcap = m;
            uint64_t *lk = nullptr, *lk2 = nullptr;
            int32_t *ub = nullptr;
            double *lw = nullptr, *lw2 = nullptr;
            const int64_t *mode = ctx->d_counters + 7;
            if (validate) {
                lk = ctx->alloc<uint64_t>(Lcap + 1);
                lk2 = ctx->alloc<uint64_t>(Lcap + 1);
                lw = ctx->alloc<double>(Lcap + 1);
                lw2 = ctx->alloc<double>(Lcap + 1);
                ub = ctx->alloc<int32_t>(etiles + 1);
            }
            // columns and both parents read per entry; per off-tree edge its id, endpoints
            // and weight written, per tree edge its id
            GSS_LAUNCH_B(8 * nnz + 28 * t->M + 4 * (int64_t)n, k_off_write,
                         dim3((unsigned)etiles), dim3(PB), 0, sa, t->row_ptr, t->col, t->w, t->parent, n, nnz, etiles,
                         tile_row, t->M, t->off_id, t->off_u, t->off_v, t->off_w, t->d_vbase, t->G, t->off_g,
                         t->tree_eid, status, epoch, lb_ticket_ptr(ctx), ctx->d_counters + 13, ctx->d_counters + 9,
                         ctx->d_flags, Lcap, lk, lw, ub, mode);
            if (validate) {
                int64_t *bpart = ctx->alloc<int64_t>(etiles + 1);
                GSS_LAUNCH_B(12 * nnz + 4 * (int64_t)(n + 1), k_check_entries, dim3((unsigned)etiles), dim3(PB), 0,
                             sa, t->row_ptr, t->col, t->w, n, nnz, tile_row, ctx->d_flags, bpart, mode);
                GSS_LAUNCH(k_balance_total, dim3(1), dim3(1024), 0, sa, bpart, etiles, ctx->d_counters + 10);
                ctx->free(bpart);
            }
            tr = Transpose{lk, lk2, lw, lw2, ub, Lcap};
        }
    }

    HIP_OK(hipMemcpyAsync(ctx->h_counters, ctx->d_counters, 8 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&ctx->h_counters[15], ctx->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    HIP_OK(hipEventRecord(ctx->ev_read, st));
    // memory-safe on any parent array: only valid parents are linked
    GSS_LAUNCH_B(12 * (int64_t)n, k_tree_vertices<true>, dim3(grid_for(n, PB)), dim3(PB), 0, st, t->parent, n, ccnt,
                 fc, nsib, ctx->d_flags, ctx->d_counters);
    // Tour records (successors, parent, degree, fixed-point term), the tour ranking and
    // the RMQ structure are enqueued before the host reads the counters: they take the
    // root and the terms' scale from device memory and are memory-safe on any parent
    // array (only valid parents are linked, successors stay inside the arcs, every walk
    // is bounded), so the host's wait overlaps them; the verdict on the tree comes after.
    const int64_t need = (int64_t)(n - 1) - (t->virt_root >= 0 ? t->G : 0);  // tree edges that are graph edges
    TRec *trec = ctx->alloc<TRec>(n);
    int32_t *succ = ctx->alloc<int32_t>(2 * (int64_t)n);
    int64_t tb = grid_for(n, PB);
    u128 *tbs = ctx->alloc<u128>(tb);
    uint64_t *tbc = ctx->alloc<uint64_t>(tb);
    // per vertex: tree-edge position, resistance, parent, child count, first child and
    // next sibling read; record and both successors written
    GSS_LAUNCH_B(68 * (int64_t)n, k_tour_rec, dim3((unsigned)tb), dim3(PB), 0, st, tpos, tinv, t->parent, ccnt, fc,
                 nsib, n, ctx->d_counters, ctx->d_flags, need, trec, succ, tbs, tbc);
    GSS_LAUNCH(k_terms_total, dim3(1), dim3(1024), 0, st, tbs, tbc, tb, ctx->d_flags, ctx->d_counters, need, n);

    // Euler tour
    t->L = n;  // the LCA sequence is indexed by preorder
    t->vrec = ctx->alloc<VRec>(n);
    t->epk = ctx->alloc<uint64_t>(t->L);
    GSS_LAUNCH(k_vrec_root, dim3(1), dim3(1), 0, st, t->vrec, n, ctx->d_counters, t->epk, ccnt, fc,
               ctx->d_counters + 12);
    // the tour is ranked without waiting for the host: its flags (overflow, cycle) are read
    // together with the off-tree enumeration's below; every kernel in between is
    // memory-safe on a failed ranking
    std::vector<void *> rank_bufs;
    int mult = 1;
    t->rank_attempts = n > 1 ? 1 : 0;
    if (n > 1) euler_rank(ctx, t, succ, trec, ctx->d_counters + 12, mult, rank_bufs);

    // RMQ structure
    int32_t L = t->L;
    t->nb = (L + 63) / 64;
    t->nsb = (t->nb + 63) / 64;
    int lv = 1;
    while ((1 << lv) <= t->nsb) lv++;
    t->sblevels = lv;
    t->pmask = ctx->alloc<uint64_t>(L);
    t->ppre = ctx->alloc<uint64_t>(L);
    t->psuf = ctx->alloc<uint64_t>(L);
    t->bmin = ctx->alloc<uint64_t>(t->nb);
    t->bmask = ctx->alloc<uint64_t>(t->nb);
    t->bpre = ctx->alloc<uint64_t>(t->nb);
    t->bsuf = ctx->alloc<uint64_t>(t->nb);
    t->sbst = ctx->alloc<uint64_t>((int64_t)t->sblevels * t->nsb);
    auto build_rmq = [&]() {
        GSS_LAUNCH_B(32 * (int64_t)L + 8 * (int64_t)t->nb, k_rmq_blocks, dim3(grid_for(t->nb, RMQ_WPB)),
                     dim3(RMQ_WPB * 64), 0, st, t->epk, L, t->pmask, t->ppre, t->psuf, t->bmin, t->nb);
        GSS_LAUNCH(k_rmq_super, dim3(grid_for(t->nsb, RMQ_WPB)), dim3(RMQ_WPB * 64), 0, st, t->bmin, t->nb,
                   t->bmask, t->bpre, t->bsuf, t->sbst, t->nsb);
        GSS_LAUNCH(k_rmq_sparse, dim3(1), dim3(1024), 0, st, t->sbst, t->nsb, t->sblevels);
    };
    build_rmq();
    ctx->free(ccnt);
    ctx->free(fc);
    ctx->free(tpos);
    ctx->free(nsib);
    ctx->free(tinv);
    ctx->free(tbs);
    ctx->free(tbc);

    // the tree passes' counters (the GPU ranks on meanwhile)
    ctx->sync_read();
    uint32_t f;
    memcpy(&f, &ctx->h_counters[15], sizeof f);
    const int64_t roots = ctx->h_counters[0];
    if (tr.lk) {
        if (ctx->h_counters[7] == 1) {
            // transposition: the lower entries sorted stably by column (the column digits
            // of the keys), compared with the upper entries in id order
            AuxScope aux(ctx);
            int kb = 1;
            while (kb < 4 && ((uint64_t)(n - 1) >> (8 * kb)) != 0) kb++;
            lsd_sort_kw(ctx, tr.lk, tr.lw, tr.lk2, tr.lw2, tr.Lcap, 32, kb);
            uint32_t epoch = 0;
            uint64_t *status = lb_begin(ctx, etiles, &epoch);
            // per entry its column, per upper entry its weight, its row's parent and its
            // sorted mirror; per off-tree edge its id, endpoints and weight written
            GSS_LAUNCH_B(4 * nnz + 12 * m + 16 * tr.Lcap + 28 * t->M, k_sym_compare, dim3((unsigned)etiles), dim3(PB),
                         0, ctx->stream, t->row_ptr, t->col, t->w, t->parent, n, nnz, etiles, tile_row, tr.ub, tr.Lcap,
                         tr.lk, tr.lw, t->M, t->off_id, t->off_u, t->off_v, t->off_w, t->d_vbase, t->G, t->off_g,
                         t->tree_eid, status, epoch, lb_ticket_ptr(ctx), ctx->d_counters + 9, ctx->d_flags);
            for (void *p : {(void *)tr.lk, (void *)tr.lk2, (void *)tr.lw, (void *)tr.lw2, (void *)tr.ub})
                ctx->free(p);
        } else {
            // mirror search: the lists were not written; they return to the pool once the
            // auxiliary stream is joined
            AuxScope aux(ctx);
            for (void *p : {(void *)tr.lk, (void *)tr.lk2, (void *)tr.lw, (void *)tr.lw2, (void *)tr.ub})
                ctx->free(p);
        }
    }
    // Errors keep their precedence (CSR checks, symmetry, then the tree): on any error
    // the auxiliary stream's checks are awaited and read before the verdict.
    auto fail_checked = [&](uint32_t tree_f) {
        aux_join(ctx);
        HIP_OK(hipMemcpyAsync(ctx->h_counters + 9, ctx->d_counters + 9, 5 * sizeof(int64_t), hipMemcpyDeviceToHost,
                              st));
        const uint32_t all = read_flags(ctx) | tree_f;  // syncs
        for (void *p : rank_bufs) ctx->free(p);
        ctx->free(succ);
        ctx->free(trec);
        const uint32_t fg = all & (F_ARG | F_NOT_SIMPLE | F_WEIGHT);
        if (fg) fail(status_from_flags(fg), "invalid graph");
        if (validate && ((all & F_ASYM) || ctx->h_counters[10] != 0 || nnz % 2))
            fail(GSS_ERR_ASYM, "the graph is not symmetric");
        if (all & F_NOT_TREE) fail(GSS_ERR_NOT_TREE, "parent array is not a rooted tree");
        fail(status_from_flags(all), "invalid input");
    };
    if ((f & (F_ARG | F_NOT_SIMPLE | F_WEIGHT | F_ASYM)) || (f & F_NOT_TREE) || roots != 1)
        fail_checked(roots != 1 ? F_NOT_TREE : 0);
    // the host's copy of the device's rule (terms_info)
    t->root = (int32_t)ctx->h_counters[1];
    int64_t emin = ctx->h_counters[2], emax = ctx->h_counters[3];
    bool tree_edge_missing = ctx->h_counters[4] != need;
    bool range_bad = (f & F_RANGE) != 0;
    if (n == 1) emin = emax = 0;
    if (!range_bad && !tree_edge_missing && emax - emin > 74) range_bad = true;
    if (range_bad || tree_edge_missing) emin = emax = 0;  // keep the fixed-point terms bounded
    t->emin = (int32_t)emin;
    t->scale = (int32_t)emin - 52;

    aux_join(ctx);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(&ctx->h_counters[9], ctx->d_counters + 9, 5 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    f = read_flags(ctx);  // syncs
    uint32_t earlier = 0;  // flags raised outside the ranking (kept over a retry)
    for (;;) {
        for (void *p : rank_bufs) ctx->free(p);
        rank_bufs.clear();
        if (!(f & F_OVERFLOW)) break;
        if (mult >= 8) {
            if (f & F_NOT_TREE) break;
            ctx->free(succ);
            ctx->free(trec);
            fail(GSS_ERR_HIP, "list ranking: level capacity exceeded");
        }
        // a level outgrew its capacity (vanishingly rare): rank again with more room; an
        // attempt that ran out of room proves nothing about the tree
        earlier = f & ~(F_OVERFLOW | F_NOT_TREE);
        fill_bytes(ctx, ctx->d_flags, 0, sizeof(uint32_t));
        mult *= 2;
        t->rank_attempts++;
        euler_rank(ctx, t, succ, trec, ctx->d_counters + 12, mult, rank_bufs);
        build_rmq();
        f = read_flags(ctx) | earlier;
    }
    ctx->free(succ);
    ctx->free(trec);
    // the auxiliary stream's CSR checks first (their precedence), then the tree's
    const uint32_t fg = f & (F_ARG | F_NOT_SIMPLE | F_WEIGHT);
    if (fg) fail(status_from_flags(fg), "invalid graph");
    if (validate && ((f & F_ASYM) || ctx->h_counters[10] != 0 || nnz % 2))
        fail(GSS_ERR_ASYM, "the graph is not symmetric");
    if (f & F_NOT_TREE) fail(GSS_ERR_NOT_TREE, "parent array has a cycle");
    if (tree_edge_missing) fail(GSS_ERR_TREE_EDGE, "a tree edge is not an edge of the graph");
    if (range_bad || (f & F_RANGE)) fail(GSS_ERR_RANGE, "tree resistances exceed the 127-bit fixed point");
    if (ctx->h_counters[13] != t->m) fail(GSS_ERR_ASYM, "upper and lower triangles differ in size");
    if (nnz > 0 && (ctx->h_counters[9] != t->M || (f & F_TREE_EDGE)))
        fail(GSS_ERR_TREE_EDGE, "off-tree edge count does not match m-n+1");
    if (t->virt_root < 0) {  // a single graph: one range covering everything
        t->vbase = {0, (int64_t)n};
        t->ebase = {0, t->m};
        t->Mg = {t->M};
        t->obase = {0, t->M};
    }
}

// ------------------------------------------------------------------------------------
// batches: the disjoint union of G graphs, each graph's root linked to a virtual root
// ------------------------------------------------------------------------------------
struct UnionDesc {
    const int32_t *row_ptr, *col, *parent;
    const double *w;
    int32_t n;
    int32_t pad;
    int64_t nnz, vbase, ebase;  // first union vertex and first union CSR entry
};

// union CSR rows, columns and parents; per-graph checks that the union could hide
__global__ void k_union_fill(const UnionDesc *__restrict__ d, int32_t G, int64_t Ntot, int64_t nnz_tot,
                             int32_t vroot, int32_t *__restrict__ rp, int32_t *__restrict__ col,
                             double *__restrict__ w, int32_t *__restrict__ parent, int32_t *__restrict__ roots,
                             uint32_t *flags)
{
    int32_t g = blockIdx.y;
    const UnionDesc D = d[g];
    uint32_t f = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < D.n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t r = D.row_ptr[i];
        if (i == 0 && r != 0) f |= F_ARG;
        if (i == D.n - 1 && (int64_t)D.row_ptr[D.n] != D.nnz) f |= F_ARG;
        rp[D.vbase + i] = (int32_t)(D.ebase + r);
        int32_t p = D.parent[i];
        if (p == -1) {
            atomicAdd(&roots[g], 1);
            parent[D.vbase + i] = vroot;
        } else if (p < 0 || p >= D.n) {
            f |= F_NOT_TREE;
            parent[D.vbase + i] = -2;  // out of range in the union too
        } else {
            parent[D.vbase + i] = (int32_t)(D.vbase + p);
        }
    }
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < D.nnz; k += (int64_t)gridDim.x * blockDim.x) {
        int32_t c = D.col[k];
        if (c < 0 || c >= D.n) f |= F_ARG;
        col[D.ebase + k] = (int32_t)(D.vbase + c);
        w[D.ebase + k] = D.w[k];
    }
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        rp[Ntot] = (int32_t)nnz_tot;      // the virtual root's row is empty
        rp[Ntot + 1] = (int32_t)nnz_tot;
        parent[vroot] = -1;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_roots_check(const int32_t *__restrict__ roots, int32_t G, uint32_t *flags)
{
    int32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < G && roots[g] != 1) atomicOr(flags, F_NOT_TREE);
}

void prep_batch(gss_ctx ctx, gss_tree t, int32_t G, const gss_csr *gs, const int32_t *const *parents, uint32_t flags)
{
    hipStream_t st = ctx->stream;
    std::vector<UnionDesc> hd(G);
    int64_t N = 0, E = 0;
    t->vbase.assign(G + 1, 0);
    for (int32_t g = 0; g < G; g++) {
        hd[g].row_ptr = gs[g].row_ptr;
        hd[g].col = gs[g].col;
        hd[g].w = gs[g].w;
        hd[g].parent = parents[g];
        hd[g].n = gs[g].n;
        hd[g].pad = 0;
        hd[g].nnz = gs[g].nnz;
        hd[g].vbase = N;
        hd[g].ebase = E;
        t->vbase[g] = N;
        N += gs[g].n;
        E += gs[g].nnz;
    }
    t->vbase[G] = N;
    if (N + 1 >= (1 << 30) || E >= ((int64_t)1 << 31)) fail(GSS_ERR_ARG, "batch too large");
    const int32_t n = (int32_t)(N + 1);
    t->n = n;
    t->nnz = E;
    t->G = G;
    t->virt_root = (int32_t)N;
    t->own_row_ptr = ctx->alloc<int32_t>(n + 1);
    t->own_col = ctx->alloc<int32_t>(E + 1);
    t->own_w = ctx->alloc<double>(E + 1);
    t->own_parent = ctx->alloc<int32_t>(n);
    t->row_ptr = t->own_row_ptr;
    t->col = t->own_col;
    t->w = t->own_w;
    t->parent = t->own_parent;
    std::vector<int32_t> vb32(G + 1);
    for (int32_t g = 0; g <= G; g++) vb32[g] = (int32_t)t->vbase[g];
    t->d_vbase = ctx->alloc<int32_t>(G + 1);
    UnionDesc *dd = ctx->alloc<UnionDesc>(G);
    int32_t *roots = ctx->alloc<int32_t>(G);
    HIP_OK(hipMemcpyAsync(t->d_vbase, vb32.data(), sizeof(int32_t) * (G + 1), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(dd, hd.data(), sizeof(UnionDesc) * G, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemsetAsync(roots, 0, sizeof(int32_t) * G, st));
    HIP_OK(hipMemsetAsync(ctx->d_flags, 0, sizeof(uint32_t), st));
    // enough workgroups per graph that the largest graph's copy runs at bandwidth
    int64_t most = 1;
    for (int32_t g = 0; g < G; g++) most = std::max<int64_t>(most, std::max<int64_t>(gs[g].nnz, gs[g].n));
    const unsigned gx = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(64, most / (PB * 16)));
    GSS_LAUNCH_B(24 * (int64_t)E + 16 * (int64_t)N, k_union_fill, dim3(gx, G), dim3(PB), 0, st, dd, G, N, E,
                 t->virt_root, t->own_row_ptr, t->own_col, t->own_w, t->own_parent, roots, ctx->d_flags);
    GSS_LAUNCH(k_roots_check, dim3(grid_for(G, PB)), dim3(PB), 0, st, roots, G, ctx->d_flags);
    uint32_t f = read_flags(ctx);
    ctx->free(dd);
    ctx->free(roots);
    if (f) fail(status_from_flags(f), "invalid graph in the batch");
    prep_tree(ctx, t, flags);
    // per-graph edge and off-tree ranges
    // a symmetric simple graph holds nnz / 2 upper entries (the union passed its checks,
    // and it is symmetric exactly when every graph is)
    t->ebase.assign(G + 1, 0);
    for (int32_t g = 0; g < G; g++) t->ebase[g + 1] = t->ebase[g] + gs[g].nnz / 2;
    t->Mg.assign(G, 0);
    t->obase.assign(G + 1, 0);
    for (int32_t g = 0; g < G; g++) {
        t->Mg[g] = (t->ebase[g + 1] - t->ebase[g]) - (gs[g].n - 1);
        t->obase[g + 1] = t->obase[g] + t->Mg[g];
    }
    t->d_obase = ctx->alloc<int64_t>(G + 1);
    HIP_OK(hipMemcpyAsync(t->d_obase, t->obase.data(), sizeof(int64_t) * (G + 1), hipMemcpyHostToDevice, st));
    ctx->sync();  // the host vector is the copy's source
}
