// gss_subtask.h -- LCA subtask engine: persistent work-queue kernel, grouping and features.
#pragma once
#include "gss_impl.h"

#define GSS_NFEAT 12          // features per subtask for the cost model
#define GSS_LOCAL_CAP 1024    // largest subtask the persistent kernel accepts
#define GSS_LANE_MAX 8        // queued subtasks this small are run by one lane each
enum : uint8_t { ST_UNDEC_ = 0, ST_CAND_ = 1, ST_MARK_ = 2 };

struct SubtaskArgs {
    int64_t P;                    // prefix length
    const int32_t *grp;           // ranks grouped by LCA, rank order inside a group
    const int32_t *sub_ptr;       // [nsub+1]
    const int32_t *queue;         // subtask ids in work order: nbig wavefront subtasks, then
                                  // the lane subtasks (at most GSS_LANE_MAX edges)
    int32_t nqueue;               // subtasks in the queue
    int32_t nbig;                 // wavefront subtasks at the front of the queue
    int32_t local_max;            // size limit of queued subtasks (<= GSS_LOCAL_CAP)
    int32_t chunk;                // queue entries taken per atomic on the head
    int32_t lpt_rounds;           // queue entries dealt to each wavefront before pulling
    unsigned int *queue_head;     // atomic pop counters: [0] wavefront part, [1] lane part
    const int32_t *ancU, *ancV;   // [(c+1) * P] ancestor chains per rank
    const int32_t *rdu, *rdv;     // depths of the endpoints per rank
    const uint8_t *rb;            // beta* per rank
    uint8_t *state;               // [P] out: recovered / marked
    uint64_t *cycles;             // [nsub] out: cycles spent per subtask (may be null)
    void *cand_scratch;           // per wavefront: local_max candidate descriptors
};

void launch_local_recover(gss_ctx ctx, int C, const SubtaskArgs &a, int blocks);
void launch_grouping_kernels(gss_ctx ctx, int64_t P, const uint64_t *glca, int32_t *head);
void launch_group_ptr(gss_ctx ctx, int64_t P, const uint64_t *glca, const int32_t *hid, int32_t *sub_ptr,
                      int32_t *sub_lca);
// nsubp: the subtask count in device memory; cap >= it: queue slots (keys past the count
// sort last)
void launch_subtask_keys(gss_ctx ctx, const int64_t *nsubp, int32_t cap, const int32_t *sub_ptr, int32_t local_max,
                         const float *pred, int cost_bits, uint64_t *qkey, int32_t *qval, int32_t *is_local,
                         int32_t *nlocal, int32_t *nsmall, unsigned long long *nglobal_edges);
void launch_join_list(gss_ctx ctx, int64_t P, const uint64_t *glca, const int32_t *hid, const int32_t *is_local,
                      const int32_t *grp, int32_t *glist);
void launch_subtask_features(gss_ctx ctx, const int64_t *nsubp, int32_t cap, const int32_t *sub_ptr,
                             const int32_t *sub_lca, const int32_t *grp, const int32_t *rdu, const int32_t *rdv,
                             const uint8_t *rb, const int32_t *ru, const int32_t *rv, const VRec *vrec, int64_t P,
                             int32_t local_max, float *feat);

// learned cost model (gss_mlp.hip): predicted cost per subtask from its features
// rows: min(cap, *d_nsub) (the subtask count in device memory)
void costmodel_predict(gss_ctx ctx, const float *feat, int64_t cap, const int64_t *d_nsub, float *pred);
// appends this call's per-subtask features, sizes and cycles to the context trace
void trace_append(gss_ctx ctx, int64_t nsub, const int32_t *sub_ptr, const int32_t *sub_lca, int64_t P,
                  const float *feat, const uint64_t *cycles, const int32_t *queue, int32_t nlocal);
void costmodel_predict_log2(gss_ctx ctx, const float *feat, int64_t n, float *out);
void costmodel_load(gss_ctx ctx, const float *host_w);
void costmodel_save(gss_ctx ctx, float *host_w);
void costmodel_train(gss_ctx ctx, const float *host_feat, const double *host_cycles, int64_t n, int32_t epochs,
                     float lr, uint64_t seed, uint32_t flags, float *host_loss);
void costmodel_grad(gss_ctx ctx, const float *host_x, const float *host_y, int32_t nb, float *host_g,
                    float *host_loss);
int64_t costmodel_nparam_total();
size_t local_desc_bytes(int C);
