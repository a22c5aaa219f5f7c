// gss_loose.hip -- one pass of the greedy under feGRASS's loose similarity (Def.
// "Similar edge (Loose)", eq. cond-loose-2) over a resolved prefix of the criticality
// order: the in-repo baseline that the strict condition is compared with (Sec. II-B,
// the multi-pass rule; Sec. III-A, the density-aware condition).
//
// Under the loose condition a recovered edge e = (u, v) marks every later off-tree edge
// with an endpoint in S_u or S_v, the balls of the constant radius c on the tree.  The
// relation "an endpoint of one edge lies within c tree hops of an endpoint of the other"
// is symmetric, so the serial pass (recover an unmarked edge, mark the later edges it
// covers) recovers the lexicographically first maximal independent set of that conflict
// graph in rank order.  Rounds of local decisions reach it exactly:
//   - an undecided edge with no undecided conflicting edge of lower rank is recovered
//     (edges recovered in the same round never conflict with each other),
//   - every undecided edge that conflicts with an edge recovered in the round is marked
//     (that edge ranks lower: otherwise the marked edge would have blocked it);
// each round decides at least the lowest undecided rank, and none depends on the
// rounds' count or on the order inside a round.
//
// Tree distance through common ancestors: hops(x, y) <= c exactly when some vertex z is
// the i-th ancestor of x and the j-th ancestor of y with i + j <= c (the lowest common
// ancestor is one when the distance is at most c; any such z bounds the distance).  So
// every undecided edge posts its rank at the cells (z, i) of the first c + 1 ancestors z
// of both endpoints, A keeping the lowest rank per cell, and reads the cells (z, j),
// j <= c - i, over the same ancestors; recovered edges set their cells of C the same way.
// In a batch the graphs' trees hang under a virtual root, which counts as above the root:
// edges of different graphs never conflict.
#include <climits>

#include "gss_impl.h"

namespace {

constexpr int LO_BLOCK = 256;

// prefix-edge states, as the candidate kernels of the recovery read them
constexpr uint8_t LO_UNDEC = 0, LO_CAND = 1, LO_MARK = 2, LO_NEW = 3;  // NEW: recovered this round

__global__ void k_lo_fill(int32_t *__restrict__ a, int64_t n, int32_t v)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// undecided edges post their rank at the ancestor cells of both endpoints
__global__ void k_lo_post(int64_t P, const uint8_t *__restrict__ state, const int32_t *__restrict__ ancU,
                          const int32_t *__restrict__ ancV, int32_t c, int32_t vroot, int32_t *__restrict__ A)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || state[p] != LO_UNDEC) return;
    for (int side = 0; side < 2; side++) {
        const int32_t *anc = side ? ancV : ancU;
        for (int i = 0; i <= c; i++) {
            const int32_t z = anc[(int64_t)i * P + p];
            if (z < 0 || z == vroot) break;  // above the root
            atomicMin(&A[(int64_t)z * (c + 1) + i], (int32_t)p);
        }
    }
}

// an undecided edge whose conflicting undecided edges all rank higher is recovered
__global__ void k_lo_decide(int64_t P, uint8_t *__restrict__ state, const int32_t *__restrict__ ancU,
                            const int32_t *__restrict__ ancV, int32_t c, int32_t vroot,
                            const int32_t *__restrict__ A, uint8_t *__restrict__ C)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P || state[p] != LO_UNDEC) return;
    int32_t low = INT_MAX;  // at most p: the edge reads its own post at (u, 0)
    for (int side = 0; side < 2; side++) {
        const int32_t *anc = side ? ancV : ancU;
        for (int i = 0; i <= c; i++) {
            const int32_t z = anc[(int64_t)i * P + p];
            if (z < 0 || z == vroot) break;
            const int32_t *cell = A + (int64_t)z * (c + 1);
            for (int j = 0; j <= c - i; j++) low = min(low, cell[j]);
        }
    }
    if (low != (int32_t)p) return;
    state[p] = LO_NEW;
    for (int side = 0; side < 2; side++) {
        const int32_t *anc = side ? ancV : ancU;
        for (int i = 0; i <= c; i++) {
            const int32_t z = anc[(int64_t)i * P + p];
            if (z < 0 || z == vroot) break;
            C[(int64_t)z * (c + 1) + i] = 1;
        }
    }
}

// clears this round's posts, settles the recovered edges, marks the undecided edges a
// recovered edge covers and counts the edges still undecided into rem[round & 1];
// rem[2] keeps the number of rounds that had an undecided edge
__global__ void k_lo_settle(int64_t P, uint8_t *__restrict__ state, const int32_t *__restrict__ ancU,
                            const int32_t *__restrict__ ancV, int32_t c, int32_t vroot, int32_t *__restrict__ A,
                            const uint8_t *__restrict__ C, unsigned long long *__restrict__ rem, int32_t round)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) rem[(round + 1) & 1] = 0;  // the next round's counter
    bool left = false, posted = false;
    if (p < P) {
        const uint8_t s = state[p];
        posted = s == LO_UNDEC || s == LO_NEW;
        if (posted) {  // the edges that posted this round
            bool covered = false;
            for (int side = 0; side < 2; side++) {
                const int32_t *anc = side ? ancV : ancU;
                for (int i = 0; i <= c; i++) {
                    const int32_t z = anc[(int64_t)i * P + p];
                    if (z < 0 || z == vroot) break;
                    A[(int64_t)z * (c + 1) + i] = INT_MAX;
                    if (s == LO_UNDEC) {
                        const uint8_t *cell = C + (int64_t)z * (c + 1);
                        for (int j = 0; j <= c - i; j++) covered |= cell[j] != 0;
                    }
                }
            }
            if (s == LO_NEW) state[p] = LO_CAND;
            else if (covered) state[p] = LO_MARK;
            else left = true;
        }
    }
    const uint64_t b = __ballot(left);
    if (lane_id() == 0 && b) atomicAdd(&rem[round & 1], (unsigned long long)__popcll(b));
    if (lane_id() == 0 && __ballot(posted)) atomicMax(&rem[2], (unsigned long long)round + 1);
}

}  // namespace

// Decides every edge of a prefix of P ranks (state[p] = 1 recovered, 2 marked) by the
// loose condition with radius c.  ancU/ancV: column i holds the i-th tree ancestor of the
// endpoints of rank p at [i * P + p], -1 above the root; n: vertices; vroot: a batch's
// virtual root (-1 for one graph).  Returns the rounds that had an undecided edge.
int64_t loose_greedy(gss_ctx ctx, int32_t n, int32_t vroot, int64_t P, int32_t c, const int32_t *ancU,
                     const int32_t *ancV, uint8_t *state)
{
    hipStream_t st = ctx->stream;
    fill_bytes(ctx, state, 0, (size_t)P + 1);
    if (P <= 0) return 0;
    const int64_t cells = (int64_t)n * (c + 1);
    int32_t *A = ctx->alloc<int32_t>(cells);
    uint8_t *C = ctx->alloc<uint8_t>(cells);
    unsigned long long *rem = ctx->alloc<unsigned long long>(3);
    GSS_LAUNCH(k_lo_fill, dim3(std::min<unsigned>(grid_for(cells, LO_BLOCK), 4096u)), dim3(LO_BLOCK), 0, st, A,
               cells, INT_MAX);
    fill_bytes(ctx, C, 0, (size_t)cells);
    fill_bytes(ctx, rem, 0, 3 * sizeof(unsigned long long));
    const dim3 g(grid_for(P, LO_BLOCK)), b(LO_BLOCK);
    // rounds are launched in growing groups; the undecided count is read after each group
    int64_t round = 0;
    unsigned long long h[3] = {0, 0, 0};
    for (int64_t group = 2;; group = std::min<int64_t>(2 * group, 64)) {
        for (int64_t r = 0; r < group; r++, round++) {
            GSS_LAUNCH(k_lo_post, g, b, 0, st, P, state, ancU, ancV, c, vroot, A);
            GSS_LAUNCH(k_lo_decide, g, b, 0, st, P, state, ancU, ancV, c, vroot, A, C);
            GSS_LAUNCH(k_lo_settle, g, b, 0, st, P, state, ancU, ancV, c, vroot, A, C, rem, (int32_t)round);
        }
        ctx->readback(h, rem, sizeof h);
        if (h[(round - 1) & 1] == 0) break;
    }
    HIP_OK(hipGetLastError());
    ctx->free(A);
    ctx->free(C);
    ctx->free(rem);
    return (int64_t)h[2];
}
