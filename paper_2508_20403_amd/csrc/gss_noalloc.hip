// gss_noalloc.hip -- the allocation-free variant of gss_recover.
//
// Callers that cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid it) get gss_recover_noalloc: the same kernels, with every
// scratch buffer carved out of one file-scope device array instead of the context's
// pool.  Each device holds its own copy of the array, whose address is looked up once
// per device when a context is created there.  In host code the array's name is not a
// device address: only that looked-up address is ever passed to kernels or copies.
#include <mutex>

#include "gss_impl.h"

#define GSS_NOALLOC_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[GSS_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[GSS_NOALLOC_MAX_DEVICES];

// the device address of this device's scratch array (the device must be current)
void noalloc_scratch_init(int device)
{
    if (device < 0 || device >= GSS_NOALLOC_MAX_DEVICES)
        throw gss_error{GSS_ERR_ARG, "device index beyond the allocation-free scratch table"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        throw gss_error{GSS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    }
    g_scratch_ptr[device] = ptr;
}

void *noalloc_scratch(int device)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return (device >= 0 && device < GSS_NOALLOC_MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

// Scratch a recovery of this tree needs at the least: the per-edge arrays plus the
// buffers of a first prefix of about 1.25 K edges (a rounded-down estimate; the arena
// also stops a call that outgrows it later, with the same error).
static size_t noalloc_estimate(gss_ctx ctx, gss_tree t, const gss_params *p, int64_t K)
{
    const int64_t c = p->beta;
    const int64_t M = t->M;
    const int64_t P0 = std::min<int64_t>(M, K + K / 4 + 1024);
    const int64_t per_prefix = 130 + 8 * (c + 1) + 48 * (c + 1) * (c + 1);
    const int64_t lm = std::max<int32_t>(ctx->local_max, 1);
    const int64_t cand = std::min<int64_t>((int64_t)ctx->local_blocks * 4 * lm * (8 * (c + 1) + 12), (int64_t)256 << 20);
    return (size_t)(13 * (M + 1) + 4 * (M / 4096 + 2) + (int64_t)16384 * t->G + per_prefix * (P0 + 1) + cand);
}

gss_status recover_noalloc_impl(gss_ctx ctx, gss_tree t, const gss_params *p, uint8_t *mask, int32_t *order,
                                double *stretch, gss_info *info)
{
    char *base = (char *)noalloc_scratch(ctx->device);
    if (!base) throw gss_error{GSS_ERR_HIP, "no allocation-free scratch on this device"};
    const int64_t K = target_count(t, 0, p);
    const size_t need = noalloc_estimate(ctx, t, p, K);
    if (need > (size_t)GSS_NOALLOC_SCRATCH_BYTES)
        throw gss_error{GSS_ERR_OOM, "input too large for the allocation-free entry point: it needs about " +
                                         std::to_string(need >> 20) + " MiB of scratch, the limit is " +
                                         std::to_string((size_t)GSS_NOALLOC_SCRATCH_BYTES >> 20) +
                                         " MiB; use gss_recover"};
    struct ArenaScope {
        gss_ctx c;
        ArenaScope(gss_ctx ctx_, char *b) : c(ctx_)
        {
            c->arena = b;
            c->arena_size = GSS_NOALLOC_SCRATCH_BYTES;
            c->arena_off = 0;
            c->arena_peak = 0;
        }
        ~ArenaScope()
        {
            c->arena = nullptr;
            c->arena_size = c->arena_off = 0;
        }
    } scope(ctx, base);
    uint8_t *masks[1] = {mask};
    int32_t *orders[1] = {order};
    return recover_impl(ctx, t, p, masks, order ? orders : nullptr, stretch, info);
}
