// gss_mlp.hip -- learned cost model of LCA subtasks.
//
// A 12 -> 64 -> 64 -> 1 ReLU network predicts log2(cycles) of a subtask in the persistent
// recovery kernel from 12 subtask features.  The scheduler orders the work queue by the
// prediction (longest first); the recovery output never depends on it.
//   * inference: layers 1 and 2 on BF16 matrix cores (CDNA4's v_mfma_f32_16x16x32_bf16,
//     FP32 accumulation; lane l supplies row l % 16 and the eight K slots 8 (l / 16)..+7
//     of A, the same slots of B), one wavefront per 16 subtasks; layer 3 in FP32;
//   * training: FP32 mini-batch Adam, data parallel: a step's mini-batch is cut into
//     64-sample slices, one workgroup per slice runs forward, MSE loss and backward in
//     LDS and writes its share of the gradient, and a second kernel sums the shares in a
//     fixed order and applies Adam (deterministic; one workgroup and 64-sample batches
//     for small training sets);
//   * a gradient-only entry runs the same FP32 forward/backward on one batch (tests).
// Parameter layout (floats): W1[64][12] b1[64] W2[64][64] b2[64] W3[64] b3, then the
// feature normalisation mean[12] and std[12].
#include <cmath>

#include "gss_subtask.h"

#define HD 64
#define NF GSS_NFEAT
#define OFF_W1 0
#define OFF_B1 (HD * NF)
#define OFF_W2 (OFF_B1 + HD)
#define OFF_B2 (OFF_W2 + HD * HD)
#define OFF_W3 (OFF_B2 + HD)
#define OFF_B3 (OFF_W3 + HD)
#define NPARAM (OFF_B3 + 1)
#define OFF_MEAN NPARAM
#define OFF_STD (NPARAM + NF)
#define NTOTAL (NPARAM + 2 * NF)
#define TB 64  // training mini-batch

static_assert(NPARAM == 5057, "parameter count");

typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16x16 output tile += A (16 x 32) * B (32 x 16), BF16 operands given as bit patterns
__device__ __forceinline__ v4f mfma_bf16_k32(v8s a, v8s b, v4f acc)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), acc, 0, 0,
                                                   0);
}

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t b = __float_as_uint(f);
    uint32_t r = b + 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

// ------------------------------------------------------------------------------------
// BF16 copies of W1 (padded to 16 inputs) and W2 for the matrix cores
// ------------------------------------------------------------------------------------
__global__ void k_mlp_to_bf16(const float *__restrict__ w, uint16_t *__restrict__ wb)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < HD * 16) {
        int n = i / 16, k = i % 16;
        wb[i] = f2bf(k < NF ? w[OFF_W1 + n * NF + k] : 0.f);
    } else if (i < HD * 16 + HD * HD) {
        int j = i - HD * 16;
        wb[i] = f2bf(w[OFF_W2 + j]);
    }
}

// ------------------------------------------------------------------------------------
// inference: a block of 4 wavefronts handles 64 subtasks per iteration; with np given,
// only the first min(n, *np) rows (a count known on the device only)
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mlp_infer(const float *__restrict__ feat, int64_t n,
                                                   const int64_t *__restrict__ np,
                                                   const float *__restrict__ w, const uint16_t *__restrict__ wb,
                                                   float *__restrict__ out, int log_out)
{
    __shared__ float sh[4][16][HD + 1];
    if (np && *np < n) n = *np;
    const int lane = lane_id(), wv = threadIdx.x / GSS_WAVE;
    const int col = lane & 15, quad = lane >> 4;
    const uint16_t *wb1 = wb, *wb2 = wb + HD * 16;
    for (int64_t base = (int64_t)blockIdx.x * 64; base < n; base += (int64_t)gridDim.x * 64) {
        const int64_t r0 = base + wv * 16;
        // layer 1: A = normalised features (row = col, k = 8*quad..+7; inputs past the
        // twelve features are zero)
        v8s a;
        {
            int64_t r = r0 + col;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                int k = 8 * quad + i;
                float x = 0.f;
                if (r < n && k < NF) x = (feat[r * NF + k] - w[OFF_MEAN + k]) / w[OFF_STD + k];
                a[i] = (short)f2bf(x);
            }
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
            v8s b;
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int k = 8 * quad + i;
                b[i] = k < 16 ? (short)wb1[(16 * t + col) * 16 + k] : (short)0;
            }
            v4f acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma_bf16_k32(a, b, acc);
            // lane holds rows 4*quad+i, column 16t+col
#pragma unroll
            for (int i = 0; i < 4; i++) sh[wv][4 * quad + i][16 * t + col] = fmaxf(acc[i] + w[OFF_B1 + 16 * t + col], 0.f);
        }
        __syncthreads();
        // layer 2
        v4f acc2[4];
#pragma unroll
        for (int t = 0; t < 4; t++) {
            acc2[t] = (v4f){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kk = 0; kk < 2; kk++) {
                v8s a2, b2;
#pragma unroll
                for (int i = 0; i < 8; i++) {
                    a2[i] = (short)f2bf(sh[wv][col][32 * kk + 8 * quad + i]);
                    b2[i] = (short)wb2[(16 * t + col) * HD + 32 * kk + 8 * quad + i];
                }
                acc2[t] = mfma_bf16_k32(a2, b2, acc2[t]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; t++)
#pragma unroll
            for (int i = 0; i < 4; i++)
                sh[wv][4 * quad + i][16 * t + col] = fmaxf(acc2[t][i] + w[OFF_B2 + 16 * t + col], 0.f);
        __syncthreads();
        // layer 3 (FP32): row = col, four lanes split the 64 inputs
        float s = 0.f;
#pragma unroll
        for (int k = 0; k < 16; k++) s += sh[wv][col][16 * quad + k] * w[OFF_W3 + 16 * quad + k];
        s += __shfl_xor(s, 16, GSS_WAVE);
        s += __shfl_xor(s, 32, GSS_WAVE);
        const int64_t r = r0 + col;
        if (quad == 0 && r < n) {
            float y = s + w[OFF_B3];
            out[r] = log_out ? y : exp2f(fminf(y, 120.f));
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------
// training (FP32, one workgroup)
// ------------------------------------------------------------------------------------
// Activation rows are padded to HD + 1 floats and feature rows to NF + 1, so that lanes
// walking samples (stride one row) hit different LDS banks.
struct TrainLds {
    float w[NPARAM];
    float x[TB][NF + 1];
    float z1[TB][HD + 1];
    float z2[TB][HD + 1];
    float dy[TB];
    float y[TB];
};

// forward + backward of nb <= TB samples held in LDS.  The gradient is that of
// sum_b (yhat_b - y_b)^2 / denom, written to g[NPARAM] (global memory, fully overwritten);
// returns the sum of squared errors (thread 0).
__device__ float mlp_fwd_bwd(TrainLds &L, int nb, float denom, float *__restrict__ g)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    // z1 = x W1^T + b1  (lanes over samples)
    for (int e = tid; e < nb * HD; e += nt) {
        int h = e / nb, b = e % nb;
        float s = L.w[OFF_B1 + h];
        for (int k = 0; k < NF; k++) s += L.x[b][k] * L.w[OFF_W1 + h * NF + k];
        L.z1[b][h] = s;
    }
    __syncthreads();
    // z2 = relu(z1) W2^T + b2  (lanes over samples, weights broadcast)
    for (int e = tid; e < nb * HD; e += nt) {
        int h = e / nb, b = e % nb;
        float s = L.w[OFF_B2 + h];
        for (int k = 0; k < HD; k++) s += fmaxf(L.z1[b][k], 0.f) * L.w[OFF_W2 + h * HD + k];
        L.z2[b][h] = s;
    }
    __syncthreads();
    // y_hat, dy = 2 (y_hat - y) / denom
    for (int b = tid; b < nb; b += nt) {
        float s = L.w[OFF_B3];
        for (int k = 0; k < HD; k++) s += fmaxf(L.z2[b][k], 0.f) * L.w[OFF_W3 + k];
        L.dy[b] = 2.f * (s - L.y[b]) / denom;
        L.y[b] = (s - L.y[b]) * (s - L.y[b]);  // squared error, kept for the loss
    }
    __syncthreads();
    float sse = 0.f;
    if (tid == 0)
        for (int b = 0; b < nb; b++) sse += L.y[b];
    // gradients of layer 3
    for (int k = tid; k <= HD; k += nt) {
        float s = 0.f;
        for (int b = 0; b < nb; b++) s += L.dy[b] * (k < HD ? fmaxf(L.z2[b][k], 0.f) : 1.f);
        g[k < HD ? OFF_W3 + k : OFF_B3] = s;
    }
    __syncthreads();
    // dz2 = dy W3 * [z2 > 0]  (stored over z2; the ReLU mask is read before overwriting)
    for (int e = tid; e < nb * HD; e += nt) {
        int b = e / HD, h = e % HD;
        L.z2[b][h] = (L.z2[b][h] > 0.f) ? L.dy[b] * L.w[OFF_W3 + h] : 0.f;
    }
    __syncthreads();
    // gW2[h][k] = sum_b dz2[b][h] relu(z1[b][k]);  gb2[h] = sum_b dz2[b][h]
    for (int e = tid; e < HD * HD + HD; e += nt) {
        float s = 0.f;
        if (e < HD * HD) {
            int h = e / HD, k = e % HD;
            for (int b = 0; b < nb; b++) s += L.z2[b][h] * fmaxf(L.z1[b][k], 0.f);
            g[OFF_W2 + e] = s;
        } else {
            int h = e - HD * HD;
            for (int b = 0; b < nb; b++) s += L.z2[b][h];
            g[OFF_B2 + h] = s;
        }
    }
    __syncthreads();
    // dz1 = (dz2 W2) * [z1 > 0]  (stored over z1)
    for (int e = tid; e < nb * HD; e += nt) {
        int b = e / HD, k = e % HD;
        float s = 0.f;
        for (int h = 0; h < HD; h++) s += L.z2[b][h] * L.w[OFF_W2 + h * HD + k];
        L.z1[b][k] = (L.z1[b][k] > 0.f) ? s : 0.f;  // each element reads only its own z1
    }
    __syncthreads();
    // gW1[h][k] = sum_b dz1[b][h] x[b][k];  gb1[h] = sum_b dz1[b][h]
    for (int e = tid; e < HD * NF + HD; e += nt) {
        float s = 0.f;
        if (e < HD * NF) {
            int h = e / NF, k = e % NF;
            for (int b = 0; b < nb; b++) s += L.z1[b][h] * L.x[b][k];
            g[OFF_W1 + e] = s;
        } else {
            int h = e - HD * NF;
            for (int b = 0; b < nb; b++) s += L.z1[b][h];
            g[OFF_B1 + h] = s;
        }
    }
    __syncthreads();
    return sse;
}

// loads rows (start + b * stride) mod n, b < nb (normalised features, log2 targets) into LDS
__device__ void load_batch(TrainLds &L, const float *__restrict__ feat, const float *__restrict__ tgt,
                           const float *__restrict__ stats, int64_t n, int64_t start, int nb, int64_t stride)
{
    for (int e = threadIdx.x; e < nb * NF; e += blockDim.x) {
        int b = e / NF, k = e % NF;
        int64_t r = (start + (int64_t)b * stride) % n;
        L.x[b][k] = (feat[r * NF + k] - stats[k]) / stats[NF + k];
    }
    for (int b = threadIdx.x; b < nb; b += blockDim.x) L.y[b] = tgt[(start + (int64_t)b * stride) % n];
    __syncthreads();
}

// One training step, forward/backward part: workgroup q takes slice q of the step's
// mini-batch (rows (offset + (row0 + q * TB + b) * stride) mod n, b < TB, clipped to the
// rnb rows of the batch) and writes its gradient share gpart[q] and its squared-error
// sum sse[q].  The shares are scaled by the whole mini-batch size, so they sum to the
// mini-batch gradient.
__global__ __launch_bounds__(256) void k_mlp_step(const float *__restrict__ w, const float *__restrict__ feat,
                                                  const float *__restrict__ tgt, int64_t n, int64_t offset,
                                                  int64_t stride, int64_t row0, int32_t rnb,
                                                  float *__restrict__ gpart, float *__restrict__ sse)
{
    __shared__ TrainLds L;
    const int q = blockIdx.x;
    const int nb = min(TB, rnb - q * TB);
    float *g = gpart + (int64_t)q * NPARAM;
    if (nb <= 0) {
        for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) g[i] = 0.f;
        if (threadIdx.x == 0) sse[q] = 0.f;
        return;
    }
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) L.w[i] = w[i];
    load_batch(L, feat, tgt, w + OFF_MEAN, n, (offset + (row0 + (int64_t)q * TB) % n * stride) % n, nb, stride);
    const float e = mlp_fwd_bwd(L, nb, (float)rnb, g);
    if (threadIdx.x == 0) sse[q] = e;
}

// One training step, update part: g = sum of the nq shares in slice order, then Adam
// (step t >= 1) on every parameter; workgroup 0 adds the squared errors to loss[0].
__global__ __launch_bounds__(256) void k_mlp_adam(float *__restrict__ w, float *__restrict__ mom,
                                                  const float *__restrict__ gpart, const float *__restrict__ sse,
                                                  int32_t nq, int64_t t, float lr, float *__restrict__ loss)
{
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        float e = 0.f;
        for (int q = 0; q < nq; q++) e += sse[q];
        loss[0] += e;
    }
    if (i >= NPARAM) return;
    float gi = 0.f;
    for (int q = 0; q < nq; q++) gi += gpart[(int64_t)q * NPARAM + i];
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    const float m = b1 * mom[i] + (1.f - b1) * gi;
    const float v = b2 * mom[NPARAM + i] + (1.f - b2) * gi * gi;
    mom[i] = m;
    mom[NPARAM + i] = v;
    w[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// gradient of the batch MSE at the current weights (FP32), for checks against a CPU model
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ w, const float *__restrict__ xraw,
                                                  const float *__restrict__ tgt, int nb, float *__restrict__ g,
                                                  float *__restrict__ loss_out)
{
    __shared__ TrainLds L;
    for (int i = threadIdx.x; i < NPARAM; i += blockDim.x) L.w[i] = w[i];
    load_batch(L, xraw, tgt, w + OFF_MEAN, nb, 0, nb, 1);
    const float sse = mlp_fwd_bwd(L, nb, (float)nb, g);
    if (threadIdx.x == 0) *loss_out = sse / (float)nb;
}

// feature statistics (mean, std) and log2 targets of a training set
__global__ __launch_bounds__(256) void k_mlp_prepare(const float *__restrict__ feat, const double *__restrict__ cyc,
                                                     int64_t n, float *__restrict__ w, float *__restrict__ tgt,
                                                     int stats)
{
    __shared__ double s1[256], s2[256];
    for (int k = 0; k < NF && stats; k++) {
        double a = 0, b = 0;
        for (int64_t r = threadIdx.x; r < n; r += 256) {
            double x = feat[r * NF + k];
            a += x;
            b += x * x;
        }
        s1[threadIdx.x] = a;
        s2[threadIdx.x] = b;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) {
                s1[threadIdx.x] += s1[threadIdx.x + h];
                s2[threadIdx.x] += s2[threadIdx.x + h];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            double mean = s1[0] / (double)n;
            double var = s2[0] / (double)n - mean * mean;
            w[OFF_MEAN + k] = (float)mean;
            w[OFF_STD + k] = (float)sqrt(var > 1e-12 ? var : 1.0);
        }
        __syncthreads();
    }
    for (int64_t r = threadIdx.x; r < n; r += 256) tgt[r] = (float)log2(cyc[r] > 1.0 ? cyc[r] : 1.0);
}

// He-style initialisation from a counter-based generator (uniform in [-a, a])
__global__ void k_mlp_init(float *__restrict__ w, uint64_t seed)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= NPARAM) return;
    float fan = (i < OFF_B1) ? (float)NF : (i < OFF_W2) ? 0.f : (i < OFF_B2) ? (float)HD : (i < OFF_W3) ? 0.f
                                                                     : (i < OFF_B3) ? (float)HD : 0.f;
    if (fan == 0.f) {
        w[i] = 0.f;
        return;
    }
    uint64_t h = mix64(seed ^ (0xD1B54A32D192ED03ull * (uint64_t)(i + 1)));
    float u = (float)((h >> 40) & 0xffffff) / 16777216.f;  // [0,1)
    float a = sqrtf(6.f / fan);
    w[i] = (2.f * u - 1.f) * a;
}

// ------------------------------------------------------------------------------------
// host
// ------------------------------------------------------------------------------------
static void ensure_model(gss_ctx ctx)
{
    if (!ctx->mlp_w) {
        ctx->mlp_w = ctx->alloc<float>(NTOTAL);
        ctx->mlp_wbf16 = ctx->alloc<uint16_t>(HD * 16 + HD * HD);
    }
}

static void refresh_bf16(gss_ctx ctx)
{
    GSS_LAUNCH(k_mlp_to_bf16, dim3(grid_for(HD * 16 + HD * HD, 256)), dim3(256), 0, ctx->stream, ctx->mlp_w,
               (uint16_t *)ctx->mlp_wbf16);
}

void costmodel_predict(gss_ctx ctx, const float *feat, int64_t cap, const int64_t *d_nsub, float *pred)
{
    if (!ctx->model_ready) throw gss_error{GSS_ERR_ARG, "no cost model loaded"};
    if (cap <= 0) return;
    int blocks = (int)std::min<int64_t>((cap + 63) / 64, 2048);
    GSS_LAUNCH(k_mlp_infer, dim3(blocks), dim3(256), 0, ctx->stream, feat, cap, d_nsub, ctx->mlp_w,
               (const uint16_t *)ctx->mlp_wbf16, pred, 0);
}

void costmodel_predict_log2(gss_ctx ctx, const float *feat, int64_t n, float *out)
{
    if (!ctx->model_ready) throw gss_error{GSS_ERR_ARG, "no cost model loaded"};
    if (n <= 0) return;
    int blocks = (int)std::min<int64_t>((n + 63) / 64, 2048);
    GSS_LAUNCH(k_mlp_infer, dim3(blocks), dim3(256), 0, ctx->stream, feat, n, (const int64_t *)nullptr, ctx->mlp_w,
               (const uint16_t *)ctx->mlp_wbf16, out, 1);
}

void costmodel_load(gss_ctx ctx, const float *host_w)
{
    ensure_model(ctx);
    HIP_OK(hipMemcpyAsync(ctx->mlp_w, host_w, sizeof(float) * NTOTAL, hipMemcpyHostToDevice, ctx->stream));
    refresh_bf16(ctx);
    ctx->sync();
    ctx->model_ready = true;
}

void costmodel_save(gss_ctx ctx, float *host_w)
{
    if (!ctx->mlp_w) throw gss_error{GSS_ERR_ARG, "no cost model"};
    HIP_OK(hipMemcpyAsync(host_w, ctx->mlp_w, sizeof(float) * NTOTAL, hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
}

// Row order of epoch ep: row (offset + i * stride) mod n for i = 0..n-1, a permutation
// because the stride is made coprime to n.
static void epoch_order(uint64_t seed, int32_t ep, int64_t n, int64_t &offset, int64_t &stride)
{
    const uint64_t h = mix64(seed + 0x9E3779B97F4A7C15ull * (uint64_t)(ep + 1));
    stride = (int64_t)(h % (uint64_t)n) | 1;
    for (;;) {
        int64_t a = stride, b = n;
        while (b) {
            const int64_t t = a % b;
            a = b;
            b = t;
        }
        if (a == 1) break;
        stride = (stride + 2) % n;
        if (stride == 0) stride = 1;
    }
    offset = (int64_t)(mix64(h) % (uint64_t)n);
}

void costmodel_train(gss_ctx ctx, const float *host_feat, const double *host_cycles, int64_t n, int32_t epochs,
                     float lr, uint64_t seed, uint32_t flags, float *host_loss)
{
    if (n < 2 || epochs < 1) throw gss_error{GSS_ERR_ARG, "training needs at least 2 samples and 1 epoch"};
    const bool warm = (flags & GSS_TRAIN_WARM) != 0;
    if (warm && !ctx->model_ready) throw gss_error{GSS_ERR_ARG, "a warm start needs a loaded cost model"};
    hipStream_t st = ctx->stream;
    ensure_model(ctx);
    // slices per mini-batch: one for small sets, growing so that an epoch keeps at least
    // 256 steps, at most 64 (a 4096-sample mini-batch)
    const int32_t nq = (int32_t)std::max<int64_t>(1, std::min<int64_t>(64, n / (TB * 256)));
    const int64_t NB = (int64_t)nq * TB;
    const int64_t steps_per_epoch = (n + NB - 1) / NB;
    float *feat = ctx->alloc<float>(n * NF);
    double *cyc = ctx->alloc<double>(n);
    float *tgt = ctx->alloc<float>(n);
    float *mom = ctx->alloc<float>(2 * NPARAM);
    float *gpart = ctx->alloc<float>((int64_t)nq * NPARAM);
    float *sse = ctx->alloc<float>(nq);
    float *loss = ctx->alloc<float>(epochs);
    HIP_OK(hipMemcpyAsync(feat, host_feat, sizeof(float) * n * NF, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(cyc, host_cycles, sizeof(double) * n, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemsetAsync(mom, 0, sizeof(float) * 2 * NPARAM, st));
    HIP_OK(hipMemsetAsync(loss, 0, sizeof(float) * epochs, st));
    if (!warm) GSS_LAUNCH(k_mlp_init, dim3(grid_for(NPARAM, 256)), dim3(256), 0, st, ctx->mlp_w, seed);
    GSS_LAUNCH(k_mlp_prepare, dim3(1), dim3(256), 0, st, feat, cyc, n, ctx->mlp_w, tgt, warm ? 0 : 1);
    int64_t t = 0;
    for (int32_t ep = 0; ep < epochs; ep++) {
        int64_t offset, stride;
        epoch_order(seed, ep, n, offset, stride);
        for (int64_t s = 0; s < steps_per_epoch; s++) {
            const int32_t rnb = (int32_t)std::min<int64_t>(NB, n - s * NB);
            GSS_LAUNCH(k_mlp_step, dim3(nq), dim3(256), 0, st, ctx->mlp_w, feat, tgt, n, offset, stride, s * NB, rnb,
                       gpart, sse);
            GSS_LAUNCH(k_mlp_adam, dim3(grid_for(NPARAM, 256)), dim3(256), 0, st, ctx->mlp_w, mom, gpart, sse, nq,
                       ++t, lr, loss + ep);
        }
    }
    refresh_bf16(ctx);
    std::vector<float> lh(epochs);
    HIP_OK(hipMemcpyAsync(lh.data(), loss, sizeof(float) * epochs, hipMemcpyDeviceToHost, st));
    ctx->sync();
    if (host_loss)
        for (int32_t ep = 0; ep < epochs; ep++) host_loss[ep] = lh[ep] / (float)n;  // mean squared error
    ctx->model_ready = true;
    ctx->free(feat);
    ctx->free(cyc);
    ctx->free(tgt);
    ctx->free(mom);
    ctx->free(gpart);
    ctx->free(sse);
    ctx->free(loss);
}

void costmodel_grad(gss_ctx ctx, const float *host_x, const float *host_y, int32_t nb, float *host_g,
                    float *host_loss)
{
    if (nb < 1 || nb > TB) throw gss_error{GSS_ERR_ARG, "batch must hold 1..64 samples"};
    if (!ctx->mlp_w) throw gss_error{GSS_ERR_ARG, "no cost model"};
    hipStream_t st = ctx->stream;
    float *x = ctx->alloc<float>(nb * NF), *y = ctx->alloc<float>(nb), *g = ctx->alloc<float>(NPARAM);
    float *l = ctx->alloc<float>(1);
    HIP_OK(hipMemcpyAsync(x, host_x, sizeof(float) * nb * NF, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(y, host_y, sizeof(float) * nb, hipMemcpyHostToDevice, st));
    GSS_LAUNCH(k_mlp_grad, dim3(1), dim3(256), 0, st, ctx->mlp_w, x, y, nb, g, l);
    HIP_OK(hipMemcpyAsync(host_g, g, sizeof(float) * NPARAM, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(host_loss, l, sizeof(float), hipMemcpyDeviceToHost, st));
    ctx->sync();
    ctx->free(x);
    ctx->free(y);
    ctx->free(g);
    ctx->free(l);
}

// ------------------------------------------------------------------------------------
// trace of per-subtask features and cycles (training data)
// ------------------------------------------------------------------------------------
void trace_append(gss_ctx ctx, int64_t nsub, const int32_t *sub_ptr, const int32_t *sub_lca, int64_t P,
                  const float *feat, const uint64_t *cycles, const int32_t *queue, int32_t nlocal)
{
    if (!feat || !cycles || nlocal <= 0) return;
    std::vector<float> f((size_t)nsub * NF);
    std::vector<uint64_t> cy((size_t)nsub);
    std::vector<int32_t> ptr((size_t)nsub + 1), q((size_t)nlocal), lc((size_t)nsub);
    HIP_OK(hipMemcpyAsync(lc.data(), sub_lca, sizeof(int32_t) * lc.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(f.data(), feat, sizeof(float) * f.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(cy.data(), cycles, sizeof(uint64_t) * cy.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(ptr.data(), sub_ptr, sizeof(int32_t) * ptr.size(), hipMemcpyDeviceToHost, ctx->stream));
    HIP_OK(hipMemcpyAsync(q.data(), queue, sizeof(int32_t) * q.size(), hipMemcpyDeviceToHost, ctx->stream));
    ctx->sync();
    for (int32_t i = 0; i < nlocal; i++) {
        int32_t s = q[i];
        ctx->trace_feat.insert(ctx->trace_feat.end(), f.begin() + (size_t)s * NF, f.begin() + (size_t)(s + 1) * NF);
        ctx->trace_cycles.push_back((double)cy[s]);
        ctx->trace_size.push_back(ptr[s + 1] - ptr[s]);
        ctx->trace_lca.push_back(lc[s]);
        ctx->trace_plen.push_back(P);
    }
}

int64_t costmodel_nparam_total() { return NTOTAL; }
