// gss_tune.hip -- autotuner of the subtask work queue (largest subtask on the persistent
// kernel, workgroups of that kernel, queue entries per pop).  Times each candidate on the
// context stream with HIP events over a full recovery and keeps the fastest; results are
// cached in a text file keyed by device name and workload signature.  The output never
// depends on the setting (tests check it), so tuning only changes speed.
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>

#include "gss_impl.h"
#include "gss_subtask.h"

static std::string tune_key(gss_ctx ctx, gss_tree t, const gss_params *p)
{
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, ctx->device));
    std::ostringstream k;
    k << prop.gcnArchName << "|cu" << prop.multiProcessorCount << "|G" << t->G << "|n" << t->n << "|m" << t->m
      << "|M" << t->M << "|b" << p[0].beta << "|s" << p[0].sched;
    for (int32_t g = 0; g < t->G && g < 4; g++) k << "|a" << p[g].alpha << "k" << p[g].k_override;
    std::string s = k.str();
    for (char &c : s)
        if (c == ' ') c = '_';
    return s;
}

// the ranges gss_ctx_set_tuning accepts
bool tuning_valid(int32_t lm, int32_t lb, int32_t ch)
{
    return lm >= 0 && lm <= GSS_LOCAL_CAP && lb >= 1 && lb <= 65536 && ch >= 0 && ch <= 64;
}

// The last well-formed entry for key whose values are in range; other lines are skipped.
static bool cache_lookup(const char *path, const std::string &key, int32_t &lm, int32_t &lb, int32_t &ch)
{
    if (!path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream in(line);
        std::string k;
        int32_t a, b, c;
        if (!(in >> k >> a >> b >> c) || k != key || !tuning_valid(a, b, c)) continue;
        lm = a;
        lb = b;
        ch = c;
        found = true;
    }
    return found;
}

namespace {
// Restores the context's settings unless the tuning completes, and owns the events.
struct TuneGuard {
    gss_ctx ctx;
    int32_t lm, lb, ch;
    bool prof, done = false;
    hipEvent_t a = nullptr, b = nullptr;
    explicit TuneGuard(gss_ctx c)
        : ctx(c), lm(c->local_max), lb(c->local_blocks), ch(c->local_chunk), prof(c->prof)
    {
    }
    ~TuneGuard()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        ctx->prof = prof;
        if (!done) {
            ctx->local_max = lm;
            ctx->local_blocks = lb;
            ctx->local_chunk = ch;
        }
    }
};
}  // namespace

gss_status autotune_impl(gss_ctx ctx, gss_tree t, const gss_params *p, uint8_t *const *masks,
                         int32_t *const *orders, const char *cache_path, int32_t *out_lm, int32_t *out_lb,
                         int32_t *out_ch, double *out_ms)
{
    const std::string key = tune_key(ctx, t, p);
    int32_t lm = ctx->local_max, lb = ctx->local_blocks, ch = ctx->local_chunk;
    if (cache_lookup(cache_path, key, lm, lb, ch)) {
        ctx->local_max = lm;
        ctx->local_blocks = lb;
        ctx->local_chunk = ch;
        if (out_lm) *out_lm = lm;
        if (out_lb) *out_lb = lb;
        if (out_ch) *out_ch = ch;
        if (out_ms) *out_ms = -1.0;
        return GSS_OK;
    }
    TuneGuard guard(ctx);
    HIP_OK(hipEventCreate(&guard.a));
    HIP_OK(hipEventCreate(&guard.b));
    ctx->prof = false;
    double best = 1e300;
    int32_t best_lm = ctx->local_max, best_lb = ctx->local_blocks, best_ch = ctx->local_chunk;
    auto time_setting = [&](int32_t m, int32_t bl, int32_t c, double &t_best) -> gss_status {
        ctx->local_max = m;
        ctx->local_blocks = bl;
        ctx->local_chunk = c;
        t_best = 1e300;
        for (int rep = 0; rep < 2; rep++) {
            HIP_OK(hipEventRecord(guard.a, ctx->stream));
            gss_status s = recover_batch_impl(ctx, t, p, masks, orders, nullptr);
            HIP_OK(hipEventRecord(guard.b, ctx->stream));
            HIP_OK(hipEventSynchronize(guard.b));
            if (s < 0) return s;
            float ms = 0.f;
            HIP_OK(hipEventElapsedTime(&ms, guard.a, guard.b));
            t_best = ms < t_best ? ms : t_best;
        }
        return GSS_OK;
    };
    // queue limit and workgroups first (chunk from the queue length), then the chunk
    const int32_t cand_lm[] = {64, 256, 1024};
    const int32_t cand_lb[] = {256, 1024, 4096};
    for (int32_t m : cand_lm)
        for (int32_t bl : cand_lb) {
            double tb;
            gss_status s = time_setting(m, bl, 0, tb);
            if (s < 0) return s;
            if (tb < best) {
                best = tb;
                best_lm = m;
                best_lb = bl;
                best_ch = 0;
            }
        }
    const int32_t cand_ch[] = {1, 4, 16, 64};
    const int32_t lm0 = best_lm, lb0 = best_lb;
    for (int32_t c : cand_ch) {
        double tb;
        gss_status s = time_setting(lm0, lb0, c, tb);
        if (s < 0) return s;
        if (tb < best) {
            best = tb;
            best_ch = c;
        }
    }
    ctx->local_max = best_lm;
    ctx->local_blocks = best_lb;
    ctx->local_chunk = best_ch;
    guard.done = true;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        if (f) f << key << " " << best_lm << " " << best_lb << " " << best_ch << "\n";
    }
    if (out_lm) *out_lm = best_lm;
    if (out_lb) *out_lb = best_lb;
    if (out_ch) *out_ch = best_ch;
    if (out_ms) *out_ms = best;
    return GSS_OK;
}
