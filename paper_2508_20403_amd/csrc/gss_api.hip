// gss_api.hip -- the exported C ABI (declared in include/gss.h).
#include <algorithm>
#include <cmath>
#include <iterator>

#include "gss_impl.h"
#include "gss_subtask.h"

namespace {
thread_local std::string g_err;

// after a failed call: wait for auxiliary-stream work and release its deferred blocks
void aux_settle(gss_ctx ctx)
{
    if (!ctx) return;
    ctx->lb_lane = 0;
    if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
    for (void *p : ctx->aux_frees) ctx->pool.put(p);
    ctx->aux_frees.clear();
}

template <typename F>
gss_status guarded(gss_ctx ctx, F &&f)
{
    try {
        gss_status s = f();
        if (ctx && ctx->prof) ctx->prof_collect();
        return s;
    } catch (const gss_error &e) {
        aux_settle(ctx);
        if (ctx) ctx->last_error = e.msg;
        g_err = e.msg;
        if (ctx && e.status == GSS_ERR_HIP) (void)hipGetLastError();
        return e.status;
    } catch (const std::bad_alloc &) {
        aux_settle(ctx);
        if (ctx) ctx->last_error = "host allocation failed";
        return GSS_ERR_OOM;
    } catch (...) {
        aux_settle(ctx);
        if (ctx) ctx->last_error = "unexpected exception";
        return GSS_ERR_HIP;
    }
}
}  // namespace

int64_t target_count(gss_tree t, int32_t g, const gss_params *p)
{
    if (p->k_override >= 0) return p->k_override;
    int64_t ng;
    if (!t->parts.empty()) {
        gss_tree q = t->parts[t->part_of[g]];
        const int32_t i = t->part_idx[g];
        ng = q->vbase.empty() ? q->n : q->vbase[i + 1] - q->vbase[i];
    } else {
        ng = t->vbase.empty() ? t->n : t->vbase[g + 1] - t->vbase[g];
    }
    return (int64_t)std::floor(p->alpha * (double)ng);
}

// ------------------------------------------------------------------------------------
// memoized graph capture of recoveries
// ------------------------------------------------------------------------------------
// A recovery is a pure function of the tree (whose arrays may not change until it is
// freed), the parameters, the output pointers and the context's settings.  The first call
// with a given key runs eagerly and records what it reads back; the second runs the same
// host code while the stream is captured, every read-back replaced by its recorded value
// (and a device-side comparison with it), and launches the graph; later calls replay it.
struct GraphEntry {
    gss_tree t = nullptr;
    std::vector<uint8_t> key, tape;
    size_t arena_bytes = 0, h2d_bytes = 0;
    std::vector<gss_info> infos;
    gss_status status = GSS_OK;
    bool no_capture = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *arena = nullptr;
    uint32_t *flag = nullptr;
    char *pinned = nullptr;  // host data the graph's copies read at every replay
    void release()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (arena) (void)hipFree(arena);
        if (flag) (void)hipFree(flag);
        if (pinned) (void)hipHostFree(pinned);
        exec = nullptr;
        graph = nullptr;
        arena = nullptr;
        flag = nullptr;
        pinned = nullptr;
    }
    ~GraphEntry() { release(); }
};

namespace {
constexpr size_t MAX_GRAPHS = 8;  // remembered recoveries per context (oldest dropped first)

std::vector<uint8_t> graph_key(gss_ctx ctx, gss_tree t, int32_t G, const gss_params *p, uint8_t *const *masks,
                               int32_t *const *orders, const double *stretch)
{
    std::vector<uint8_t> k;
    auto put = [&](const void *x, size_t n) { k.insert(k.end(), (const uint8_t *)x, (const uint8_t *)x + n); };
    put(&t, sizeof t);
    put(&G, sizeof G);
    put(p, sizeof(gss_params) * (size_t)G);
    for (int32_t g = 0; g < G; g++) {
        const void *m = masks[g], *o = orders ? orders[g] : nullptr;
        put(&m, sizeof m);
        put(&o, sizeof o);
    }
    put(&stretch, sizeof stretch);
    const int64_t s[7] = {ctx->local_max, ctx->local_blocks, ctx->local_chunk, ctx->sort_cap,
                          ctx->sort_radix ? 1 : 0, ctx->model_ready ? 1 : 0, ctx->device};
    put(s, sizeof s);
    put(&ctx->mlp_w, sizeof ctx->mlp_w);
    put(&ctx->mlp_wbf16, sizeof ctx->mlp_wbf16);
    return k;
}

void drop_entry(gss_ctx ctx, GraphEntry *e)
{
    auto it = std::find(ctx->graphs.begin(), ctx->graphs.end(), e);
    if (it != ctx->graphs.end()) ctx->graphs.erase(it);
    delete e;
}

// one launch of a captured recovery and its single synchronisation; false when a
// replayed read-back value differed from the recorded one
bool replay(gss_ctx ctx, GraphEntry *e)
{
    HIP_OK(hipGraphLaunch(e->exec, ctx->stream));
    HIP_OK(hipMemcpyAsync(&ctx->h_counters[16], e->flag, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    uint32_t f = 0;
    memcpy(&f, &ctx->h_counters[16], sizeof f);
    if (f) ctx->last_error = "graph replay: read-back check " + std::to_string(f) + " differed from the recording";
    return f == 0;
}

// the capturing call: the same host code, read-backs from the tape, into a graph
template <typename F>
bool capture(gss_ctx ctx, GraphEntry *e, int32_t ninfo, F &&fn)
{
    if (!ctx->cap_stream) HIP_OK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    const size_t arena_bytes = e->arena_bytes + 4096;
    if (hipMalloc(&e->arena, arena_bytes) != hipSuccess || hipMalloc((void **)&e->flag, 256) != hipSuccess ||
        hipHostMalloc((void **)&e->pinned, e->h2d_bytes + 64, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        e->release();
        return false;
    }
    hipStream_t user = ctx->stream;
    ctx->arena = (char *)e->arena;
    ctx->arena_size = arena_bytes;
    ctx->arena_off = ctx->arena_peak = 0;
    ctx->cap_mode = gss_ctx_s::CAP_CAPTURE;
    ctx->tape = e->tape;
    ctx->tape_pos = 0;
    ctx->pending.clear();
    ctx->cap_host = e->pinned;
    ctx->cap_host_size = e->h2d_bytes + 64;
    ctx->cap_host_off = 0;
    ctx->cap_flag = e->flag;
    ctx->stream = ctx->cap_stream;
    ctx->cap_checks = 0;
    std::string why;
    const hipError_t eb = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed);
    bool ok = eb == hipSuccess;
    if (!ok) why = std::string("begin: ") + hipGetErrorString(eb);
    if (ok) {
        try {
            fill_bytes(ctx, e->flag, 0, sizeof(uint32_t));
            std::vector<gss_info> tmp((size_t)std::max<int32_t>(ninfo, 1));
            const gss_status s = fn(tmp.data());
            ok = s == e->status && ctx->tape_pos == ctx->tape.size() && ctx->pending.empty();
            if (!ok)
                why = "the capturing call left the recorded path (status " + std::to_string(s) + ", tape " +
                      std::to_string(ctx->tape_pos) + "/" + std::to_string(ctx->tape.size()) + ")";
        } catch (const gss_error &x) {
            ok = false;
            why = "exception: " + x.msg;
        } catch (...) {
            ok = false;
            why = "exception";
        }
        hipGraph_t g = nullptr;
        const hipError_t ee = hipStreamEndCapture(ctx->cap_stream, &g);
        if (ee != hipSuccess) {
            if (ok) why = std::string("end: ") + hipGetErrorString(ee);
            ok = false;
        }
        e->graph = g;
    }
    (void)hipGetLastError();
    ctx->stream = user;
    ctx->cap_mode = gss_ctx_s::CAP_OFF;
    ctx->arena = nullptr;
    ctx->arena_size = ctx->arena_off = ctx->arena_peak = 0;
    ctx->tape.clear();
    ctx->tape_pos = 0;
    ctx->pending.clear();
    ctx->cap_host = nullptr;
    ctx->cap_host_size = ctx->cap_host_off = 0;
    ctx->cap_flag = nullptr;
    if (ok && e->graph) {
        const hipError_t ei = hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            ok = false;
            why = std::string("instantiate: ") + hipGetErrorString(ei);
        }
    }
    if (!ok) {
        (void)hipGetLastError();
        e->release();
        ctx->last_error = "graph capture abandoned, the call ran eagerly: " + why;
    }
    return ok;
}

// runs fn(infos) (a recovery writing ninfo infos) eagerly, or records, captures or
// replays it as the key's history says
template <typename F>
gss_status memoized(gss_ctx ctx, gss_tree t, std::vector<uint8_t> key, int32_t ninfo, gss_info *infos, F &&fn)
{
    if (!ctx->capture_on || ctx->record || ctx->prof || ctx->arena || ctx->cap_mode != gss_ctx_s::CAP_OFF)
        return fn(infos);
    GraphEntry *e = nullptr;
    for (GraphEntry *x : ctx->graphs)
        if (x->t == t && x->key == key) e = x;
    auto deliver = [&](GraphEntry *x) {
        if (infos) std::copy(x->infos.begin(), x->infos.begin() + ninfo, infos);
        return x->status;
    };
    if (e && e->exec) {
        if (replay(ctx, e)) {
            ctx->n_replays++;
            return deliver(e);
        }
        drop_entry(ctx, e);  // never expected: the recovery is deterministic
        e = nullptr;
    }
    if (e && !e->no_capture) {
        if (capture(ctx, e, ninfo, fn) && replay(ctx, e)) {
            ctx->n_captures++;
            return deliver(e);
        }
        e->release();
        e->no_capture = true;
    }
    if (e) return fn(infos);
    // recording
    std::vector<gss_info> tmp((size_t)std::max<int32_t>(ninfo, 1));
    ctx->cap_mode = gss_ctx_s::CAP_RECORD;
    ctx->tape.clear();
    ctx->tape_pos = 0;
    ctx->pending.clear();
    ctx->arena_off = ctx->arena_peak = 0;
    ctx->rec_h2d = 0;
    gss_status s;
    try {
        s = fn(tmp.data());
    } catch (...) {
        ctx->cap_mode = gss_ctx_s::CAP_OFF;
        ctx->tape.clear();
        ctx->pending.clear();
        ctx->arena_off = ctx->arena_peak = 0;
        throw;
    }
    ctx->cap_mode = gss_ctx_s::CAP_OFF;
    GraphEntry *n = new GraphEntry();
    n->t = t;
    n->key = std::move(key);
    n->tape.swap(ctx->tape);
    n->arena_bytes = ctx->arena_peak;
    n->h2d_bytes = ctx->rec_h2d;
    ctx->arena_off = ctx->arena_peak = 0;
    n->infos.assign(tmp.begin(), tmp.begin() + ninfo);
    n->status = s;
    if (ctx->graphs.size() >= MAX_GRAPHS) drop_entry(ctx, ctx->graphs.front());
    ctx->graphs.push_back(n);
    ctx->n_records++;
    return deliver(n);
}

void drop_tree_graphs(gss_ctx ctx, gss_tree t)
{
    std::vector<GraphEntry *> gone;
    for (GraphEntry *x : ctx->graphs)
        if (x->t == t) gone.push_back(x);
    for (GraphEntry *x : gone) drop_entry(ctx, x);
}
}  // namespace

// frees a tree, its parts and the arrays it owns
static void delete_tree(gss_tree t)
{
    for (gss_tree p : t->parts) delete_tree(p);
    free_tree_arrays(t);
    delete t;
}

// one graph on its own, borrowing the caller's arrays (as gss_tree_prep)
static gss_tree prep_single_part(gss_ctx ctx, const gss_csr &g, const int32_t *parent, uint32_t flags)
{
    if (g.nnz >= ((int64_t)1 << 31) || g.n >= (1 << 30)) throw gss_error{GSS_ERR_ARG, "graph too large"};
    gss_tree t = new gss_tree_s();
    t->ctx = ctx;
    t->n = g.n;
    t->nnz = g.nnz;
    t->row_ptr = g.row_ptr;
    t->col = g.col;
    t->w = g.w;
    t->parent = parent;
    try {
        prep_tree(ctx, t, flags);
    } catch (...) {
        (void)hipStreamSynchronize(ctx->stream);
        delete_tree(t);
        throw;
    }
    return t;
}

// recover_impl over a batch tree: the union and every graph prepared on its own in turn
gss_status recover_batch_impl(gss_ctx ctx, gss_tree t, const gss_params *prms, uint8_t *const *masks,
                              int32_t *const *orders, gss_info *infos)
{
    if (t->parts.empty()) return recover_impl(ctx, t, prms, masks, orders, nullptr, infos);
    gss_status worst = GSS_OK;
    for (size_t q = 0; q < t->parts.size(); q++) {
        std::vector<gss_params> pp;
        std::vector<uint8_t *> mp;
        std::vector<int32_t *> op;
        std::vector<int32_t> gid;
        for (int32_t g = 0; g < t->G; g++)
            if (t->part_of[g] == (int32_t)q) gid.push_back(g);
        std::sort(gid.begin(), gid.end(), [&](int32_t a, int32_t b) { return t->part_idx[a] < t->part_idx[b]; });
        for (int32_t g : gid) {
            pp.push_back(prms[g]);
            mp.push_back(masks[g]);
            op.push_back(orders ? orders[g] : nullptr);
        }
        std::vector<gss_info> ip(gid.size());
        const gss_status s = recover_impl(ctx, t->parts[q], pp.data(), mp.data(), orders ? op.data() : nullptr,
                                          nullptr, infos ? ip.data() : nullptr);
        if (s < 0) return s;
        if (s > worst) worst = s;
        if (infos)
            for (size_t i = 0; i < gid.size(); i++) infos[gid[i]] = ip[i];
    }
    return worst;
}

extern "C" {

gss_status gss_ctx_create(int device, void *hip_stream, gss_ctx *out)
{
    if (!out) return GSS_ERR_ARG;
    *out = nullptr;
    gss_ctx ctx = new (std::nothrow) gss_ctx_s();
    if (!ctx) return GSS_ERR_OOM;
    gss_status s = guarded(ctx, [&]() -> gss_status {
        int count = 0;
        HIP_OK(hipGetDeviceCount(&count));
        if (device < 0 || device >= count) throw gss_error{GSS_ERR_ARG, "no such device"};
        HIP_OK(hipSetDevice(device));
        ctx->device = device;
        ctx->stream = (hipStream_t)hip_stream;
        HIP_OK(hipMalloc(&ctx->d_flags, 256));
        HIP_OK(hipMalloc(&ctx->d_counters, 32 * sizeof(int64_t)));
        HIP_OK(hipHostMalloc(&ctx->h_counters, 32 * sizeof(int64_t), hipHostMallocDefault));
        HIP_OK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
        HIP_OK(hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&ctx->ev_read, hipEventDisableTiming));
        HIP_OK(hipHostMalloc(&ctx->h_stage, gss_ctx_s::STAGE_BYTES, hipHostMallocDefault));
        HIP_OK(hipMemset(ctx->d_flags, 0, 256));
        HIP_OK(hipMemset(ctx->d_counters, 0, 32 * sizeof(int64_t)));
        noalloc_scratch_init(device);  // once per device, with the device current
        return GSS_OK;
    });
    if (s != GSS_OK) {
        g_err = ctx->last_error;
        if (ctx->d_flags) (void)hipFree(ctx->d_flags);
        if (ctx->d_counters) (void)hipFree(ctx->d_counters);
        if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
        if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
        if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
        if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_read) (void)hipEventDestroy(ctx->ev_read);
        if (ctx->ev_read) (void)hipEventDestroy(ctx->ev_read);
        if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
        delete ctx;
        return s;
    }
    *out = ctx;
    return GSS_OK;
}

gss_status gss_ctx_set_stream(gss_ctx ctx, void *hip_stream)
{
    if (!ctx) return GSS_ERR_ARG;
    // the context's work must stay in one stream order: drain the old stream first
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        ctx->sync();
        ctx->stream = (hipStream_t)hip_stream;
        return GSS_OK;
    });
}

gss_status gss_ctx_destroy(gss_ctx ctx)
{
    if (!ctx) return GSS_ERR_ARG;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
    while (!ctx->graphs.empty()) drop_entry(ctx, ctx->graphs.back());
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    ctx->pool.release_all();
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    if (ctx->ev_read) (void)hipEventDestroy(ctx->ev_read);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    if (ctx->d_counters) (void)hipFree(ctx->d_counters);
    if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    delete ctx;
    return GSS_OK;
}

gss_status gss_tree_prep(gss_ctx ctx, const gss_csr *g, const int32_t *parent, uint32_t flags, gss_tree *out)
{
    if (!ctx || !g || !out) return GSS_ERR_ARG;
    *out = nullptr;
    if (g->n < 1 || g->nnz < 0 || g->nnz >= ((int64_t)1 << 31) || g->n >= (1 << 30) || !g->row_ptr ||
        !parent || (g->nnz > 0 && (!g->col || !g->w))) {
        ctx->last_error = "bad graph arguments";
        return GSS_ERR_ARG;
    }
    gss_tree t = new (std::nothrow) gss_tree_s();
    if (!t) return GSS_ERR_OOM;
    t->ctx = ctx;
    t->n = g->n;
    t->nnz = g->nnz;
    t->row_ptr = g->row_ptr;
    t->col = g->col;
    t->w = g->w;
    t->parent = parent;
    gss_status s = guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        prep_tree(ctx, t, flags);
        return GSS_OK;
    });
    if (s != GSS_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        free_tree_arrays(t);
        delete t;
        return s;
    }
    *out = t;
    return GSS_OK;
}

gss_status gss_batch_prep(gss_ctx ctx, int32_t nb, const gss_csr *graphs, const int32_t *const *parents,
                          uint32_t flags, gss_tree *out)
{
    if (!ctx || nb < 1 || !graphs || !parents || !out) return GSS_ERR_ARG;
    *out = nullptr;
    for (int32_t g = 0; g < nb; g++) {
        const gss_csr &c = graphs[g];
        if (c.n < 1 || c.nnz < 0 || !c.row_ptr || !parents[g] || (c.nnz > 0 && (!c.col || !c.w))) {
            ctx->last_error = "bad graph arguments in the batch";
            return GSS_ERR_ARG;
        }
    }
    // graphs that fill the GPU by themselves are prepared and recovered on their own (no
    // copy into the union); the rest share one union
    std::vector<int32_t> own, rest;
    for (int32_t g = 0; g < nb; g++) (graphs[g].nnz >= ctx->batch_own_nnz ? own : rest).push_back(g);
    if (rest.size() == 1) {
        own.push_back(rest[0]);
        rest.clear();
    }
    gss_tree t = new (std::nothrow) gss_tree_s();
    if (!t) return GSS_ERR_OOM;
    t->ctx = ctx;
    gss_status s = guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        if (own.empty()) {
            prep_batch(ctx, t, nb, graphs, parents, flags);
            return GSS_OK;
        }
        t->G = nb;
        t->part_of.assign(nb, 0);
        t->part_idx.assign(nb, 0);
        t->n = 0;
        if (!rest.empty()) {
            std::vector<gss_csr> gs;
            std::vector<const int32_t *> ps;
            for (size_t i = 0; i < rest.size(); i++) {
                gs.push_back(graphs[rest[i]]);
                ps.push_back(parents[rest[i]]);
                t->part_of[rest[i]] = 0;
                t->part_idx[rest[i]] = (int32_t)i;
            }
            gss_tree u = new gss_tree_s();
            u->ctx = ctx;
            t->parts.push_back(u);  // freed with t on failure
            prep_batch(ctx, u, (int32_t)rest.size(), gs.data(), ps.data(), flags);
        }
        for (int32_t g : own) {
            t->part_of[g] = (int32_t)t->parts.size();
            t->part_idx[g] = 0;
            t->parts.push_back(prep_single_part(ctx, graphs[g], parents[g], flags));
        }
        for (gss_tree p : t->parts) {
            t->n += p->n;
            t->m += p->m;
            t->M += p->M;
        }
        return GSS_OK;
    });
    if (s != GSS_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        delete_tree(t);
        return s;
    }
    *out = t;
    return GSS_OK;
}

int32_t gss_tree_num_graphs(gss_tree t) { return t ? t->G : -1; }

int64_t gss_tree_graph_edges(gss_tree t, int32_t g)
{
    if (!t || g < 0 || g >= t->G) return -1;
    if (!t->parts.empty()) {
        gss_tree p = t->parts[t->part_of[g]];
        return p->ebase.empty() ? p->m : gss_tree_graph_edges(p, t->part_idx[g]);
    }
    if (t->ebase.empty()) return t->m;
    return t->ebase[g + 1] - t->ebase[g];
}


gss_status gss_recover_batch(gss_ctx ctx, gss_tree t, const gss_params *params, uint8_t *const *masks,
                             int32_t *const *orders, gss_info *infos)
{
    if (!ctx || !t || !params || !masks || t->ctx != ctx) return GSS_ERR_ARG;
    for (int32_t g = 0; g < t->G; g++) {
        const gss_params &p = params[g];
        if (!masks[g] || !(p.alpha >= 0.0 && p.alpha <= 1.0) || p.beta < 0 || p.beta > GSS_MAX_BETA ||
            p.reserved != 0 || (p.sched != GSS_SCHED_EDGECOUNT && p.sched != GSS_SCHED_LEARNED)) {
            ctx->last_error = "bad recovery parameters in the batch";
            return GSS_ERR_ARG;
        }
    }
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        ctx->record = (params[0].flags & GSS_F_RECORD) != 0;
        gss_status s = memoized(ctx, t, graph_key(ctx, t, t->G, params, masks, orders, nullptr), t->G, infos,
                                [&](gss_info *inf) { return recover_batch_impl(ctx, t, params, masks, orders, inf); });
        ctx->record = false;
        return s;
    });
}

gss_status gss_autotune(gss_ctx ctx, gss_tree t, const gss_params *params, uint8_t *const *masks,
                        int32_t *const *orders, const char *cache_path, int32_t *local_max, int32_t *local_blocks,
                        int32_t *chunk, double *best_ms)
{
    if (!ctx || !t || !params || !masks || t->ctx != ctx) return GSS_ERR_ARG;
    for (int32_t g = 0; g < t->G; g++) {
        const gss_params &p = params[g];
        if (!masks[g] || !(p.alpha >= 0.0 && p.alpha <= 1.0) || p.beta < 0 || p.beta > GSS_MAX_BETA ||
            p.reserved != 0 || (p.sched != GSS_SCHED_EDGECOUNT && p.sched != GSS_SCHED_LEARNED)) {
            ctx->last_error = "bad recovery parameters";
            return GSS_ERR_ARG;
        }
    }
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        return autotune_impl(ctx, t, params, masks, orders, cache_path, local_max, local_blocks, chunk, best_ms);
    });
}

int64_t gss_target_count(gss_tree t, int32_t g, const gss_params *p)
{
    if (!t || !p || g < 0 || g >= t->G || !(p->alpha >= 0.0 && p->alpha <= 1.0)) return -1;
    return target_count(t, g, p);
}

gss_status gss_tree_free(gss_tree t)
{
    if (!t) return GSS_ERR_ARG;
    (void)hipStreamSynchronize(t->ctx->stream);
    drop_tree_graphs(t->ctx, t);
    delete_tree(t);
    return GSS_OK;
}

int64_t gss_tree_num_edges(gss_tree t) { return t ? t->m : -1; }

gss_status gss_recover(gss_ctx ctx, gss_tree t, const gss_params *p, uint8_t *mask, int32_t *order,
                       double *stretch, gss_info *info)
{
    if (!ctx || !t || !p || !mask || t->ctx != ctx) return GSS_ERR_ARG;
    if (!(p->alpha >= 0.0 && p->alpha <= 1.0) || p->beta < 0 || p->beta > GSS_MAX_BETA || p->reserved != 0 ||
        (p->sched != GSS_SCHED_EDGECOUNT && p->sched != GSS_SCHED_LEARNED)) {
        ctx->last_error = "bad recovery parameters";
        return GSS_ERR_ARG;
    }
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        ctx->record = (p->flags & GSS_F_RECORD) != 0;
        if (t->virt_root >= 0 || !t->parts.empty())
            throw gss_error{GSS_ERR_ARG, "a batch tree needs gss_recover_batch"};
        uint8_t *masks[1] = {mask};
        int32_t *orders[1] = {order};
        gss_status s = memoized(ctx, t, graph_key(ctx, t, 1, p, masks, order ? orders : nullptr, stretch), 1, info,
                                [&](gss_info *inf) {
                                    return recover_impl(ctx, t, p, masks, order ? orders : nullptr, stretch, inf);
                                });
        ctx->record = false;
        return s;
    });
}

gss_status gss_recover_noalloc(gss_ctx ctx, gss_tree t, const gss_params *p, uint8_t *mask, int32_t *order,
                               double *stretch, gss_info *info)
{
    if (!ctx || !t || !p || !mask || t->ctx != ctx) return GSS_ERR_ARG;
    if (!(p->alpha >= 0.0 && p->alpha <= 1.0) || p->beta < 0 || p->beta > GSS_MAX_BETA || p->reserved != 0 ||
        (p->sched != GSS_SCHED_EDGECOUNT && p->sched != GSS_SCHED_LEARNED)) {
        ctx->last_error = "bad recovery parameters";
        return GSS_ERR_ARG;
    }
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        if (t->virt_root >= 0 || !t->parts.empty())
            throw gss_error{GSS_ERR_ARG, "a batch tree needs gss_recover_batch"};
        ctx->record = (p->flags & GSS_F_RECORD) != 0;
        gss_status s = GSS_OK;
        try {
            s = recover_noalloc_impl(ctx, t, p, mask, order, stretch, info);
        } catch (...) {
            ctx->record = false;
            throw;
        }
        ctx->record = false;
        return s;
    });
}

gss_status gss_tree_export(gss_tree t, int32_t *depth, uint64_t *Dlo, uint64_t *Dhi, int32_t *scale)
{
    if (!t) return GSS_ERR_ARG;
    if (!t->parts.empty()) {
        t->ctx->last_error = "a batch with graphs prepared on their own has no single tree";
        return GSS_ERR_ARG;
    }
    gss_ctx ctx = t->ctx;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        if (depth)
            HIP_OK(hipMemcpy2DAsync(depth, sizeof(int32_t), &t->vrec[0].depth, sizeof(VRec), sizeof(int32_t), t->n,
                                    hipMemcpyDeviceToDevice, ctx->stream));
        if (Dlo) HIP_OK(hipMemcpy2DAsync(Dlo, sizeof(uint64_t), &t->vrec[0].D.lo, sizeof(VRec), sizeof(uint64_t),
                                         t->n, hipMemcpyDeviceToDevice, ctx->stream));
        if (Dhi) HIP_OK(hipMemcpy2DAsync(Dhi, sizeof(uint64_t), &t->vrec[0].D.hi, sizeof(VRec), sizeof(uint64_t),
                                         t->n, hipMemcpyDeviceToDevice, ctx->stream));
        if (scale) *scale = t->scale;
        ctx->sync();
        return GSS_OK;
    });
}

gss_status gss_edge_lca(gss_ctx ctx, gss_tree t, int32_t beta, int32_t *lca, int32_t *bstar)
{
    if (!ctx || !t || t->ctx != ctx || beta < 0 || beta > GSS_MAX_BETA) return GSS_ERR_ARG;
    if (!t->parts.empty()) {
        ctx->last_error = "a batch with graphs prepared on their own has no single tree";
        return GSS_ERR_ARG;
    }
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        edge_lca_impl(ctx, t, beta, lca, bstar);
        return GSS_OK;
    });
}

gss_status gss_ctx_profile(gss_ctx ctx, int32_t enable, const char *kernel_name)
{
    if (!ctx) return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        ctx->sync();
        ctx->prof_collect();
        ctx->prof = enable != 0;
        ctx->prof_filter = kernel_name ? kernel_name : "";
        ctx->prof_acc.clear();
        return GSS_OK;
    });
}

int32_t gss_ctx_profile_read(gss_ctx ctx, int32_t idx, char *buf, int32_t buflen, double *total_ms,
                             int64_t *launches, int64_t *alg_bytes, double *last_ms)
{
    if (!ctx) return -1;
    int32_t count = (int32_t)ctx->prof_acc.size();
    if (idx < 0 || idx >= count) return count;
    auto it = ctx->prof_acc.begin();
    std::advance(it, idx);
    if (buf && buflen > 0) {
        size_t k = std::min<size_t>((size_t)buflen - 1, it->first.size());
        memcpy(buf, it->first.data(), k);
        buf[k] = 0;
    }
    if (total_ms) *total_ms = it->second.ms;
    if (launches) *launches = it->second.launches;
    if (alg_bytes) *alg_bytes = it->second.bytes;
    if (last_ms) *last_ms = it->second.last_ms;
    return count;
}

gss_status gss_ctx_set_tuning(gss_ctx ctx, int32_t local_max, int32_t local_blocks, int32_t chunk)
{
    if (!ctx || !tuning_valid(local_max, local_blocks, chunk)) return GSS_ERR_ARG;
    ctx->local_max = local_max;
    ctx->local_blocks = local_blocks;
    ctx->local_chunk = chunk;
    return GSS_OK;
}

gss_status gss_ctx_set_sort(gss_ctx ctx, int32_t radix, int32_t bucket_cap)
{
    if (!ctx || (radix != 0 && radix != 1) || bucket_cap < 0 || bucket_cap == 1 || bucket_cap > 8192)
        return GSS_ERR_ARG;
    ctx->sort_radix = radix != 0;
    ctx->sort_cap = bucket_cap;
    return GSS_OK;
}

gss_status gss_spanning_tree(gss_ctx ctx, const gss_csr *g, uint32_t flags, int32_t *parent, int32_t *root,
                             double *weff)
{
    if (!ctx || !g || !parent || !root || (flags & ~GSS_TREE_WEIGHT) != 0) return GSS_ERR_ARG;
    if (g->n < 1 || g->nnz < 0 || g->nnz >= ((int64_t)1 << 31) || g->n >= (1 << 30) || !g->row_ptr ||
        (g->nnz > 0 && (!g->col || !g->w)))
        return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        spanning_tree_impl(ctx, g, parent, root, weff, flags);
        return GSS_OK;
    });
}

gss_status gss_ctx_set_capture(gss_ctx ctx, int32_t enable)
{
    if (!ctx || (enable != 0 && enable != 1)) return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        if (!enable) {
            HIP_OK(hipStreamSynchronize(ctx->stream));
            while (!ctx->graphs.empty()) drop_entry(ctx, ctx->graphs.back());
        }
        ctx->capture_on = enable != 0;
        return GSS_OK;
    });
}

gss_status gss_ctx_capture_stats(gss_ctx ctx, int64_t *records, int64_t *captures, int64_t *replays,
                                 int64_t *syncs)
{
    if (!ctx) return GSS_ERR_ARG;
    if (records) *records = ctx->n_records;
    if (captures) *captures = ctx->n_captures;
    if (replays) *replays = ctx->n_replays;
    if (syncs) *syncs = ctx->n_syncs;
    return GSS_OK;
}

gss_status gss_ctx_set_rank_capacity(gss_ctx ctx, int32_t divisor)
{
    if (!ctx || divisor < 1 || divisor > 4) return GSS_ERR_ARG;
    ctx->rank_cap_div = divisor;
    return GSS_OK;
}

int32_t gss_tree_rank_attempts(gss_tree t)
{
    if (!t) return -1;
    int32_t a = t->rank_attempts;
    for (gss_tree p : t->parts) a = std::max(a, p->rank_attempts);
    return a;
}

gss_status gss_ctx_set_batch_split(gss_ctx ctx, int64_t own_nnz)
{
    if (!ctx || own_nnz < 0) return GSS_ERR_ARG;
    ctx->batch_own_nnz = own_nnz;
    return GSS_OK;
}

int64_t gss_trace_read(gss_ctx ctx, float *feat, double *cycles, int32_t *size, int32_t *lca, int64_t *prefix_len,
                       int64_t cap)
{
    if (!ctx || cap < 0) return -1;
    int64_t rows = (int64_t)ctx->trace_cycles.size();
    int64_t k = rows < cap ? rows : cap;
    if (feat) memcpy(feat, ctx->trace_feat.data(), sizeof(float) * GSS_NFEAT * k);
    if (cycles) memcpy(cycles, ctx->trace_cycles.data(), sizeof(double) * k);
    if (size) memcpy(size, ctx->trace_size.data(), sizeof(int32_t) * k);
    if (lca) memcpy(lca, ctx->trace_lca.data(), sizeof(int32_t) * k);
    if (prefix_len) memcpy(prefix_len, ctx->trace_plen.data(), sizeof(int64_t) * k);
    return rows;
}

gss_status gss_trace_clear(gss_ctx ctx)
{
    if (!ctx) return GSS_ERR_ARG;
    ctx->trace_feat.clear();
    ctx->trace_cycles.clear();
    ctx->trace_size.clear();
    ctx->trace_lca.clear();
    ctx->trace_plen.clear();
    return GSS_OK;
}

gss_status gss_costmodel_train(gss_ctx ctx, const float *feat, const double *cycles, int64_t n, int32_t epochs,
                               float lr, uint64_t seed, uint32_t flags, float *loss)
{
    if (!ctx || !feat || !cycles || n < 2 || epochs < 1 || !(lr > 0.f) || (flags & ~GSS_TRAIN_WARM)) return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        costmodel_train(ctx, feat, cycles, n, epochs, lr, seed, flags, loss);
        return GSS_OK;
    });
}

gss_status gss_costmodel_load(gss_ctx ctx, const float *weights)
{
    if (!ctx || !weights) return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        costmodel_load(ctx, weights);
        return GSS_OK;
    });
}

gss_status gss_costmodel_save(gss_ctx ctx, float *weights)
{
    if (!ctx || !weights) return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        costmodel_save(ctx, weights);
        return GSS_OK;
    });
}

gss_status gss_costmodel_predict(gss_ctx ctx, const float *feat, int64_t n, float *out)
{
    if (!ctx || (n > 0 && (!feat || !out)) || n < 0) return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        costmodel_predict_log2(ctx, feat, n, out);
        ctx->sync();
        return GSS_OK;
    });
}

gss_status gss_costmodel_grad(gss_ctx ctx, const float *x, const float *y, int32_t nb, float *grad, float *loss)
{
    if (!ctx || !x || !y || !grad || !loss) return GSS_ERR_ARG;
    return guarded(ctx, [&]() -> gss_status {
        HIP_OK(hipSetDevice(ctx->device));
        costmodel_grad(ctx, x, y, nb, grad, loss);
        return GSS_OK;
    });
}

const char *gss_status_str(gss_status s)
{
    switch (s) {
    case GSS_OK: return "GSS_OK";
    case GSS_SHORT: return "GSS_SHORT";
    case GSS_ERR_ARG: return "GSS_ERR_ARG";
    case GSS_ERR_NOT_SIMPLE: return "GSS_ERR_NOT_SIMPLE";
    case GSS_ERR_ASYM: return "GSS_ERR_ASYM";
    case GSS_ERR_WEIGHT: return "GSS_ERR_WEIGHT";
    case GSS_ERR_NOT_TREE: return "GSS_ERR_NOT_TREE";
    case GSS_ERR_TREE_EDGE: return "GSS_ERR_TREE_EDGE";
    case GSS_ERR_RANGE: return "GSS_ERR_RANGE";
    case GSS_ERR_HIP: return "GSS_ERR_HIP";
    case GSS_ERR_OOM: return "GSS_ERR_OOM";
    default: return "GSS_UNKNOWN";
    }
}

const char *gss_last_error(gss_ctx ctx)
{
    if (!ctx) return g_err.c_str();
    return ctx->last_error.c_str();
}

}  // extern "C"
