// gss_impl.h -- host-side internals of the gfx950 library.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/gss.h"
#include "gss_dev.h"

// Thrown inside the library only; every exported function catches it.
struct gss_error {
    gss_status status;
    std::string msg;
};

#define HIP_OK(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw gss_error{GSS_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// Caching device allocator: blocks are kept per context and reused by size.  All work
// of a context runs on its one stream, so a block returned to the cache may be handed
// out again immediately (stream order keeps earlier users ahead of later ones).
struct dev_pool {
    std::multimap<size_t, void *> free_blocks;  // capacity -> pointer
    std::map<void *, size_t> live;              // pointer -> capacity
    size_t bytes_held = 0;

    void *get(size_t bytes);
    void put(void *p);
    void release_all();
};

struct prof_rec {
    const char *name;
    hipEvent_t a, b;
    int64_t bytes;  // algorithmic bytes of the launch (0: no model)
};
struct prof_sum {
    double ms = 0;
    int64_t launches = 0;
    int64_t bytes = 0;
    double last_ms = 0;  // the latest launch
};

struct GraphEntry;  // a recorded (and possibly captured) recovery, gss_api.hip

struct gss_ctx_s {
    // live kernel timing with HIP events on the context stream (off by default)
    bool prof = false;
    std::string prof_filter;                       // empty: every kernel
    std::vector<prof_rec> prof_pending;
    std::vector<hipEvent_t> prof_events;           // free events
    std::map<std::string, prof_sum> prof_acc;      // name -> totals
    int64_t prof_bytes = 0;                        // algorithmic bytes of the next launch
    // a timed launch's event pair (the launch records its own start and end), or null
    prof_rec *prof_begin(const char *name);
    void prof_collect();                           // after a sync: accumulate elapsed times

    // subtask engine settings (autotuned) and the learned cost model
    int32_t local_max = 64;       // subtasks up to this size use the persistent kernel
    int32_t local_blocks = 2048;  // workgroups of the persistent kernel (4 wavefronts each)
    int32_t local_chunk = 0;      // queue entries per pop (0: from the queue length)
    int64_t batch_own_nnz = (int64_t)1 << 25;  // batch graphs this large are prepared on their own
    int32_t rank_cap_div = 1;     // list ranking: first-attempt level capacities divided by this
    int32_t sort_cap = 0;         // sample sort: largest bucket sorted in LDS (0: the kernel's limit)
    bool sort_radix = false;      // short sorts by the radix sort instead of the sample sort
    bool record = false;          // record per-subtask features and cycles
    bool model_ready = false;     // cost-model weights loaded
    std::vector<float> trace_feat;      // [rows * 12]
    std::vector<double> trace_cycles;   // [rows]
    std::vector<int32_t> trace_size;    // [rows]
    std::vector<int32_t> trace_lca;     // [rows] LCA vertex of the subtask
    std::vector<int64_t> trace_plen;    // [rows] length of the prefix it was resolved in
    float *mlp_w = nullptr;             // device weights (FP32 master copy)
    void *mlp_wbf16 = nullptr;          // device BF16 copy for inference

    int device = 0;
    hipStream_t stream = nullptr;
    std::string last_error;
    dev_pool pool;
    uint32_t *d_flags = nullptr;      // device error flags
    int64_t *d_counters = nullptr;    // small device scratch (32 words; words 15 and 31: the
                                      // look-back tickets of the main and the auxiliary stream)
    int64_t *h_counters = nullptr;    // pinned host mirror
    // pinned staging area for small host-to-device copies (asynchronous, unlike copies
    // from pageable memory): a bump area that restarts at every synchronisation of the
    // stream, by which time every copy staged before it has run
    char *h_stage = nullptr;
    size_t stage_off = 0;
    static constexpr size_t STAGE_BYTES = (size_t)1 << 20;
    hipEvent_t ev_done = nullptr;
    // status words of single-pass (look-back) scans and sorts, reused by epoch; one set
    // per stream (lane 0: the context stream, lane 1: the auxiliary stream)
    uint64_t *lb_status[2] = {nullptr, nullptr};
    int64_t lb_cap[2] = {0, 0};
    uint32_t lb_epoch[2] = {0, 0};
    int lb_lane = 0;
    // auxiliary stream (default priority, non-blocking) for independent work inside a
    // call: forked from and joined back into the context stream with events
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipEvent_t ev_read = nullptr;  // marks read-backs the host waits for while later work runs
    std::vector<void *> aux_frees;   // blocks released by auxiliary work, freed at the join

    // allocation-free calls: scratch is bumped out of a fixed device arena (the
    // library's static scratch array) instead of the pool; frees are no-ops and the
    // caller rolls the offset back between rounds (arena_mark / arena_reset)
    char *arena = nullptr;
    size_t arena_size = 0, arena_off = 0, arena_peak = 0;

    // Memoized graph capture of recoveries (gss_ctx_set_capture).  A recording call runs
    // eagerly and logs, in order, every value it reads back to the host (the tape) and
    // the arena bytes its allocations would take.  A capturing call runs the same host
    // code with the stream in capture mode: read-backs take their values from the tape
    // (a kernel compares the device value with it and raises cap_flag on a difference),
    // allocations come from a graph-owned arena, host data is staged in graph-owned
    // pinned memory, and synchronisations are skipped.
    enum { CAP_OFF = 0, CAP_RECORD = 1, CAP_CAPTURE = 2 };
    bool capture_on = false;
    int cap_mode = CAP_OFF;
    std::vector<uint8_t> tape;
    size_t tape_pos = 0;
    std::vector<std::pair<void *, size_t>> pending;  // asynchronous read-backs, delivered at the next sync
    size_t rec_h2d = 0;                              // recording: host-to-device bytes (64-byte units)
    char *cap_host = nullptr;                        // capturing: the graph's pinned staging block
    size_t cap_host_size = 0, cap_host_off = 0;
    uint32_t *cap_flag = nullptr;                    // capturing: the graph's mismatch word
    hipStream_t cap_stream = nullptr;
    std::vector<GraphEntry *> graphs;                // recorded and captured recoveries
    int64_t n_syncs = 0, n_records = 0, n_captures = 0, n_replays = 0;
    uint32_t cap_checks = 0;                         // capturing: read-back checks enqueued so far

    template <typename T>
    T *alloc(size_t count)
    {
        const size_t bytes = count * sizeof(T) + 16;
        if (arena) return (T *)arena_bump(bytes);
        if (cap_mode == CAP_RECORD) arena_account(bytes);
        return (T *)pool.get(bytes);
    }
    // recording: the arena offset the same allocation would move to
    void arena_account(size_t bytes)
    {
        const size_t off = (arena_off + 255) & ~(size_t)255;
        arena_off = off + bytes;
        if (arena_off > arena_peak) arena_peak = arena_off;
    }
    void *arena_bump(size_t bytes)
    {
        const size_t off = (arena_off + 255) & ~(size_t)255;
        if (off + bytes > arena_size)
            throw gss_error{GSS_ERR_OOM, "the allocation-free entry point's scratch (" +
                                             std::to_string(arena_size >> 20) + " MiB) is too small for this "
                                             "input (it needs more than " + std::to_string((off + bytes) >> 20) +
                                             " MiB); use gss_recover"};
        arena_off = off + bytes;
        if (arena_off > arena_peak) arena_peak = arena_off;
        return arena + off;
    }
    size_t arena_mark() const { return arena_off; }
    void arena_reset(size_t mark)
    {
        if (arena || cap_mode == CAP_RECORD) arena_off = mark;
    }
    void free(void *p)
    {
        if (!p) return;
        if (arena && (char *)p >= arena && (char *)p < arena + arena_size) return;
        if (lb_lane == 1) aux_frees.push_back(p);  // still in use by the auxiliary stream
        else pool.put(p);
    }
    // waits for the stream (skipped while capturing); asynchronous read-backs are
    // delivered (recording: appended to the tape; capturing: taken from it)
    void sync()
    {
        if (cap_mode != CAP_CAPTURE) {
            HIP_OK(hipStreamSynchronize(stream));
            if (aux && stream != aux) HIP_OK(hipStreamSynchronize(aux));
            stage_off = 0;
            n_syncs++;
        }
        for (auto &pb : pending) tape_io(pb.first, pb.second);
        pending.clear();
    }
    // waits for the context stream up to ev_read (recorded by the caller after its
    // read-backs; work enqueued after it keeps running, and so does the auxiliary
    // stream), so the caller reads back only what the context stream produced before the
    // event (staging memory is kept)
    void sync_read()
    {
        if (cap_mode != CAP_CAPTURE) {
            HIP_OK(hipEventSynchronize(ev_read));
            n_syncs++;
        }
    }
    // a read-back whose wait comes later: the copy is followed by ev_read, the caller
    // enqueues independent work and then calls wait_early() before reading dst (recording
    // and capturing take the ordinary read-back)
    bool early_pending = false;
    void readback_early(void *dst, const void *src, size_t bytes, uint64_t words = ~0ull)
    {
        if (cap_mode != CAP_OFF) {
            readback(dst, src, bytes, words);
            return;
        }
        HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
        HIP_OK(hipEventRecord(ev_read, stream));
        early_pending = true;
    }
    void wait_early()
    {
        if (!early_pending) return;
        early_pending = false;
        HIP_OK(hipEventSynchronize(ev_read));
        n_syncs++;
    }
    // a tape entry: its length (4 bytes), then the bytes read back
    void tape_io(void *dst, size_t bytes)
    {
        const uint32_t len = (uint32_t)bytes;
        if (cap_mode == CAP_RECORD) {
            tape.insert(tape.end(), (const uint8_t *)&len, (const uint8_t *)&len + sizeof len);
            tape.insert(tape.end(), (const uint8_t *)dst, (const uint8_t *)dst + bytes);
        } else if (cap_mode == CAP_CAPTURE) {
            uint32_t rec = 0;
            if (tape_pos + sizeof rec <= tape.size()) memcpy(&rec, tape.data() + tape_pos, sizeof rec);
            if (tape_pos + sizeof rec + bytes > tape.size() || rec != len)
                throw gss_error{GSS_ERR_HIP, "capture left the recorded path"};
            memcpy(dst, tape.data() + tape_pos + sizeof rec, bytes);
            tape_pos += sizeof rec + bytes;
        }
    }
    // copies bytes device bytes to the host and waits for them.  words: the 8-byte words
    // of the range the caller uses (bit i: word i; the first 64 words), the only ones a
    // replay compares with the recording (the others may hold leftovers of other calls)
    void readback(void *dst, const void *src, size_t bytes, uint64_t words = ~0ull)
    {
        if (cap_mode == CAP_CAPTURE) {
            sync();  // delivers earlier asynchronous read-backs first, in the recorded order
            tape_io(dst, bytes);
            check_replay(src, dst, bytes, words);
            return;
        }
        HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
        sync();
        tape_io(dst, bytes);
    }
    // the same, delivered by the next sync()
    void readback_async(void *dst, const void *src, size_t bytes)
    {
        if (cap_mode != CAP_CAPTURE) HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, stream));
        pending.push_back({dst, bytes});
    }
    void check_replay(const void *dev, const void *expect, size_t bytes, uint64_t words);  // capturing
    // enqueues a copy of bytes host bytes to dst on the stream; src may be reused at once
    void h2d(void *dst, const void *src, size_t bytes)
    {
        if (bytes == 0) return;
        if (cap_mode == CAP_RECORD) rec_h2d += (bytes + 63) & ~(size_t)63;
        if (cap_mode == CAP_CAPTURE) {  // the graph reads its own pinned copy at every replay
            if (cap_host_off + bytes > cap_host_size) throw gss_error{GSS_ERR_HIP, "capture staging overflow"};
            char *h = cap_host + cap_host_off;
            cap_host_off += (bytes + 63) & ~(size_t)63;
            memcpy(h, src, bytes);
            HIP_OK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, stream));
            return;
        }
        if (!h_stage || bytes > STAGE_BYTES) {
            HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream));
            return;
        }
        if (stage_off + bytes > STAGE_BYTES) sync();
        char *h = h_stage + stage_off;
        memcpy(h, src, bytes);
        stage_off += (bytes + 63) & ~(size_t)63;
        HIP_OK(hipMemcpyAsync(dst, h, bytes, hipMemcpyHostToDevice, stream));
    }
};

struct gss_tree_s {
    gss_ctx ctx = nullptr;
    int32_t n = 0;
    int64_t nnz = 0, m = 0, M = 0;
    const int32_t *row_ptr = nullptr, *col = nullptr, *parent = nullptr;
    const double *w = nullptr;
    int32_t root = 0;
    int32_t emin = 0;    // smallest binary exponent of any tree resistance 1/w
    int32_t scale = 0;   // root resistances are integers in units of 2^scale
    int32_t rank_attempts = 0;  // list-ranking attempts (more than one after a capacity retry)
    // edges
    int32_t *tree_eid = nullptr; // [n] edge id of (x, parent x), -1 at root
    // tree / Euler tour
    VRec *vrec = nullptr;        // [n] root resistance, preorder index, depth, parent
    int32_t L = 0;               // LCA sequence length n
    uint64_t *epk = nullptr;     // [L] (depth << 32) | parent of the vertex at each preorder index
    uint64_t *pmask = nullptr;   // [L] in-block suffix-minimum masks
    uint64_t *ppre = nullptr;    // [L] minimum from the block start to each position
    uint64_t *psuf = nullptr;    // [L] minimum from each position to the block end
    int32_t nb = 0, nsb = 0, sblevels = 0;
    uint64_t *bmin = nullptr;    // [nb] block minima
    uint64_t *bmask = nullptr;   // [nb] in-superblock masks over block minima
    uint64_t *bpre = nullptr;    // [nb] prefix minima of block minima within a superblock
    uint64_t *bsuf = nullptr;    // [nb] suffix minima of block minima within a superblock
    uint64_t *sbst = nullptr;    // [sblevels * nsb] sparse table over superblock minima
    // off-tree edges in id order
    int32_t *off_id = nullptr, *off_u = nullptr, *off_v = nullptr;
    double *off_w = nullptr;
    // batches: the union of G graphs whose trees hang under a virtual root (a vertex
    // with no graph edges; its tree edges carry zero resistance)
    int32_t G = 1;
    int32_t virt_root = -1;
    int32_t *off_g = nullptr;            // [M] graph of each off-tree edge (batches only)
    int32_t *d_vbase = nullptr;          // [G+1] first union vertex of each graph
    std::vector<int64_t> vbase;          // host copy
    std::vector<int64_t> ebase;          // [G+1] first union edge id of each graph
    std::vector<int64_t> Mg;             // [G] off-tree edges of each graph
    std::vector<int64_t> obase;          // [G+1] first off-tree index of each graph
    int64_t *d_obase = nullptr;          // device copy (batches only)
    // union arrays owned by a batch tree
    int32_t *own_row_ptr = nullptr, *own_col = nullptr, *own_parent = nullptr;
    double *own_w = nullptr;
    // a batch split into parts (a union of the smaller graphs and every large graph on
    // its own): graph g of the batch is graph part_idx[g] of parts[part_of[g]]
    std::vector<gss_tree_s *> parts;
    std::vector<int32_t> part_of, part_idx;
};

// ---- host entry points of the translation units --------------------------------------
void prep_tree(gss_ctx ctx, gss_tree t, uint32_t flags);
void prep_batch(gss_ctx ctx, gss_tree t, int32_t G, const gss_csr *gs, const int32_t *const *parents,
                uint32_t flags);
void free_tree_arrays(gss_tree t);
gss_status recover_impl(gss_ctx ctx, gss_tree t, const gss_params *prms, uint8_t *const *masks,
                        int32_t *const *orders, double *stretch, gss_info *infos);
// recover_impl over a batch tree, part by part when it is split
gss_status recover_batch_impl(gss_ctx ctx, gss_tree t, const gss_params *prms, uint8_t *const *masks,
                              int32_t *const *orders, gss_info *infos);
void edge_lca_impl(gss_ctx ctx, gss_tree t, int32_t beta, int32_t *lca, int32_t *bstar);
gss_status autotune_impl(gss_ctx ctx, gss_tree t, const gss_params *p, uint8_t *const *masks,
                         int32_t *const *orders, const char *cache_path, int32_t *out_lm, int32_t *out_lb,
                         int32_t *out_ch, double *out_ms);
bool tuning_valid(int32_t local_max, int32_t local_blocks, int32_t chunk);
// allocation-free recovery (gss_noalloc.hip): the device scratch array's address, looked
// up once per device at context creation, and the recovery that draws on it
void noalloc_scratch_init(int device);
gss_status recover_noalloc_impl(gss_ctx ctx, gss_tree t, const gss_params *p, uint8_t *mask, int32_t *order,
                                double *stretch, gss_info *info);
// K of graph g: the override when >= 0, else floor(fl(alpha * n_g))
int64_t target_count(gss_tree t, int32_t g, const gss_params *p);

// ---- sorting (gss_sort.hip) -----------------------------------------------------------
// sorts n <= sample_sort_max() pairs by (key, value); result in (k, v), (k2, v2) scratch
void sample_sort_pairs(gss_ctx ctx, uint64_t *&k, int32_t *&v, uint64_t *&k2, int32_t *&v2, int64_t n);
// one pass of the greedy under the loose condition over a resolved prefix (gss_loose.hip)
int64_t loose_greedy(gss_ctx ctx, int32_t n, int32_t vroot, int64_t P, int32_t c, const int32_t *ancU,
                     const int32_t *ancV, uint8_t *state);
int64_t sample_sort_max();
// stable LSD radix sort of (key, double value) pairs by the key bits [shift, shift + 8
// passes), for large arrays (count, scan, scatter per 8-bit digit); the pointers are
// swapped so that k, w hold the result (k2, w2 the scratch).  With run (device), nothing
// is sorted unless *run is nonzero.
void lsd_sort_kw(gss_ctx ctx, uint64_t *&k, double *&w, uint64_t *&k2, double *&w2, int64_t n, int shift,
                 int passes, const int64_t *run = nullptr);

// ---- shared launch helpers (gss_prims.hip) -------------------------------------------
// exclusive scan of int32 counts in place over [0,n); returns the total (host sync)
int64_t scan_exclusive_i32(gss_ctx ctx, int32_t *data, int64_t n, bool want_total);
// the same, leaving the total in device memory (no host round trip)
void scan_exclusive_i32_dev(gss_ctx ctx, int32_t *data, int64_t n, int64_t *d_total);
// status array of at least `words` words for one look-back launch, its epoch, and the
// ticket counter (always zero between launches)
uint64_t *lb_begin(gss_ctx ctx, int64_t words, uint32_t *epoch);
// feGRASS's spanning tree (gss_treegen.hip)
void spanning_tree_impl(gss_ctx ctx, const gss_csr *g, int32_t *parent, int32_t *root, double *weff, uint32_t flags);
// byte fill of device memory on the context stream by a kernel (capturable)
void fill_bytes(gss_ctx ctx, void *p, int value, size_t bytes);
inline unsigned long long *lb_ticket_ptr(gss_ctx ctx)
{
    return (unsigned long long *)(ctx->d_counters + (ctx->lb_lane ? 31 : 15));
}

// Work enqueued while an AuxScope is alive goes to the auxiliary stream, which first
// waits for everything enqueued on the context stream so far.  The host code in the
// scope must not synchronise; blocks it frees stay reserved until aux_join.  Every
// block the scope allocates must be allocated inside it (before the context stream's
// later work is enqueued), so the two streams never share a pool block.
struct AuxScope {
    gss_ctx ctx;
    hipStream_t saved;
    explicit AuxScope(gss_ctx c) : ctx(c), saved(c->stream)
    {
        HIP_OK(hipEventRecord(ctx->ev_fork, ctx->stream));
        HIP_OK(hipStreamWaitEvent(ctx->aux, ctx->ev_fork, 0));
        ctx->stream = ctx->aux;
        ctx->lb_lane = 1;
    }
    ~AuxScope()
    {
        ctx->stream = saved;
        ctx->lb_lane = 0;
    }
};
// the context stream waits for the auxiliary stream's work; its deferred frees return
// to the pool (later users are ordered after the join)
void aux_join(gss_ctx ctx);
uint32_t read_flags(gss_ctx ctx);
gss_status status_from_flags(uint32_t f);

// every kernel launch goes through this, so it can be timed when asked: a timed launch
// carries its start and stop events in the dispatch itself (no separate event packets
// between kernels, so timing barely changes the stream's pace)
#define GSS_LAUNCH(kern, grid, block, shmem, stream, ...)                                         \
    do {                                                                                          \
        prof_rec *pr_ = ctx->prof ? ctx->prof_begin(#kern) : nullptr;                              \
        if (pr_)                                                                                  \
            hipExtLaunchKernelGGL(kern, grid, block, shmem, stream, pr_->a, pr_->b, 0, __VA_ARGS__); \
        else                                                                                      \
            hipLaunchKernelGGL(kern, grid, block, shmem, stream, __VA_ARGS__);                    \
    } while (0)
// the same, stating the launch's algorithmic bytes: the least HBM traffic the step it
// performs needs (each input read once, each output written once), for roofline figures
#define GSS_LAUNCH_B(bytes, kern, grid, block, shmem, stream, ...)          \
    do {                                                                    \
        if (ctx->prof) ctx->prof_bytes = (int64_t)(bytes);                  \
        GSS_LAUNCH(kern, grid, block, shmem, stream, __VA_ARGS__);          \
    } while (0)

inline unsigned grid_for(int64_t items, int block, int per_thread = 1)
{
    int64_t g = (items + (int64_t)block * per_thread - 1) / ((int64_t)block * per_thread);
    if (g < 1) g = 1;
    return (unsigned)g;
}
