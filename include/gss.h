/*
 * gss.h -- C ABI of the MI355X (gfx950) library for pdGRASS off-tree edge recovery.
 *
 * Problem (paper Sec. II-A, Sec. II-B, Alg. 1): given a weighted undirected graph
 * G=(V,E,w) and a spanning tree T of G, recover K = floor(alpha*|V|) off-tree edges so
 * that T plus the recovered edges is the sparsifier P (|V|-1+alpha|V| edges).  Off-tree
 * edges are ranked by stretch = w(e) * R_T(e), where R_T is the tree-path resistance
 * through the LCA (Def. "Resistance distance", eq. RT, resistive weight 1/w), in
 * descending order with ties broken by ascending edge id.  Walking that order, an
 * edge that is not marked is recovered, and it marks every later off-tree edge that is
 * strictly similar to it under its density-aware BFS step
 * beta* = min(dist(u,lca), dist(v,lca), c)  (eq. beta-new, Def. "Similar edge (Strict)").
 * If a pass over all edges recovers fewer than K edges, further passes run over the
 * unrecovered edges with all marks cleared (the multi-pass rule of Sec. II-B).
 *
 * Conventions
 *  - Unless stated otherwise every array argument is a DEVICE pointer owned by the
 *    caller; the library never frees or modifies caller arrays except the outputs.
 *  - Vertex ids are int32 in [0,n).  The edge id of {u,v} (u<v) is the rank of the
 *    CSR entry (u,v) among all entries with column > row, rows ascending, then columns
 *    ascending.  Per-edge arrays are indexed by edge id, length m = nnz/2.
 *  - Every call is stream-ordered on the context's HIP stream and returns after that
 *    stream has finished the call's work (host outputs are then valid).
 *  - No exception crosses the ABI: every function returns a gss_status.
 *  - One context must be used by one host thread at a time.
 */
#ifndef GSS_H
#define GSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t gss_status;
enum {
    GSS_OK = 0,
    GSS_SHORT = 1,            /* fewer than K off-tree edges exist; all were recovered   */
    GSS_ERR_ARG = -1,         /* bad argument: null pointer, n<1, malformed row_ptr,
                                 column index out of range, alpha not in [0,1], beta<0,
                                 beta > GSS_MAX_BETA                                      */
    GSS_ERR_NOT_SIMPLE = -2,  /* a row is not strictly increasing or holds a self-loop   */
    GSS_ERR_ASYM = -3,        /* (u,v) present without (v,u), or w(u,v) != w(v,u)         */
    GSS_ERR_WEIGHT = -4,      /* a weight is <= 0, NaN or infinite                        */
    GSS_ERR_NOT_TREE = -5,    /* parent[] out of range, not exactly one root, or a cycle */
    GSS_ERR_TREE_EDGE = -6,   /* some (x, parent[x]) is not an edge of G                  */
    GSS_ERR_RANGE = -7,       /* 1/w not a normal double, tree resistances need more than
                                 127 bits of fixed point, or a stretch is not finite      */
    GSS_ERR_HIP = -8,         /* a HIP runtime call failed (see gss_last_error)           */
    GSS_ERR_OOM = -9          /* device allocation failed                                 */
};
/* When several checks fail, the status reported is the first of: ARG, NOT_SIMPLE,
 * WEIGHT, ASYM, NOT_TREE, TREE_EDGE, RANGE. */

#define GSS_MAX_BETA 8        /* largest supported BFS-step constant c                     */

typedef struct gss_ctx_s *gss_ctx;    /* device, stream binding and scratch pool          */
typedef struct gss_tree_s *gss_tree;  /* prepared graph+tree; borrows the caller's CSR    */

/* CSR graph: symmetric, rows strictly increasing, no self-loops, w > 0 finite. */
typedef struct {
    int32_t n;                 /* number of vertices, >= 1                               */
    int64_t nnz;               /* number of stored entries (2m), < 2^31                  */
    const int32_t *row_ptr;    /* device [n+1]                                           */
    const int32_t *col;        /* device [nnz]                                           */
    const double *w;           /* device [nnz]                                           */
} gss_csr;

/* gss_params.flags */
#define GSS_F_MASK_TREE 1u     /* also set mask[] = 1 on tree edges (mask = sparsifier P) */
#define GSS_F_RECORD 2u        /* append per-subtask features and measured cycles of the work-
                                  queue kernel to the context trace (cost-model training data) */
#define GSS_F_STATS 4u         /* fill gss_info.n_subtasks / largest_subtask (an extra per-edge
                                  count; -1 in those fields otherwise)                     */
#define GSS_F_KEY_RT 8u        /* order the off-tree edges by the tree-path resistance R_T
                                  alone (the literal wording of Alg. 1 Step 2, "sort L based
                                  on resistances") instead of the stretch w*R_T; ties still
                                  by ascending id.  The stretch output is unchanged.  All
                                  graphs of a batch must agree on it.                     */
#define GSS_F_LOOSE 16u        /* feGRASS's loose similarity (Def. "Similar edge (Loose)",
                                  eq. cond-loose-2) instead of the strict one: a recovered
                                  edge marks every later off-tree edge with an endpoint
                                  within beta tree hops of either of its endpoints (the
                                  constant radius c = beta for every edge, not beta*).
                                  Passes repeat as under the strict condition (Sec. II-B).
                                  The in-repo baseline of the paper's comparison; the
                                  subtask schedule plays no part.  All graphs of a batch
                                  must agree on it.                                       */

/* gss_params.sched: order in which the subtask work queue is drained (never changes
 * the output).  GSS_SCHED_LEARNED without a loaded cost model falls back to the
 * edge-count order; gss_info.sched reports which one ran. */
enum { GSS_SCHED_EDGECOUNT = 0, GSS_SCHED_LEARNED = 1 };

typedef struct {
    double alpha;              /* fraction of |V| to recover, in [0,1]                   */
    int32_t beta;              /* BFS-step constant c >= 0 of eq. beta-new               */
    int32_t sched;             /* GSS_SCHED_*                                             */
    int64_t k_override;        /* >= 0: recover exactly this many; < 0: floor(alpha*n)   */
    uint32_t flags;            /* GSS_F_*                                                 */
    int32_t reserved;          /* must be 0                                               */
} gss_params;

typedef struct {
    int64_t m;                 /* undirected edges                                       */
    int64_t n_offtree;         /* M = m - n + 1                                          */
    int64_t k;                 /* target count K                                         */
    int64_t n_recovered;       /* min(K, M)                                              */
    int64_t n_subtasks;        /* distinct LCAs over all off-tree edges (GSS_F_STATS)    */
    int64_t largest_subtask;   /* edges sharing the most common LCA (GSS_F_STATS)        */
    int64_t prefix_len;        /* length of the criticality-order prefix resolved        */
    int64_t n_arcs;            /* strict-similarity pairs found inside that prefix       */
    int64_t n_join;            /* prefix edges in subtasks above the work-queue limit,
                                  resolved by the anchor hash join (all graphs of a batch) */
    int32_t passes;            /* passes that recovered at least one edge                */
    int32_t rounds;            /* dependency rounds used to resolve the prefix           */
    int32_t sched;             /* schedule that ran: GSS_SCHED_LEARNED only when it was
                                  asked for and a cost model is loaded; otherwise the
                                  edge-count order (the fallback)                        */
} gss_info;

/* Creates a context on `device` bound to `hip_stream` (a hipStream_t, may be NULL for
 * the default stream).  *out receives the handle.  Errors: ARG, HIP. */
gss_status gss_ctx_create(int device, void *hip_stream, gss_ctx *out);
/* Rebinds the context to another stream, after waiting for the work already queued on
 * the old one (a context's work must form a single stream order).  Errors: ARG, HIP. */
gss_status gss_ctx_set_stream(gss_ctx ctx, void *hip_stream);
/* Frees the context's device memory.  Trees built on it must be freed first. */
gss_status gss_ctx_destroy(gss_ctx ctx);

/* Tree preparation (Alg. 1 Step 1 set-up: the ancestor/LCA structure and the
 * root-to-node distances): validates g and parent (unless flags has
 * GSS_PREP_TRUSTED), enumerates edges, ranks the Euler tour and builds the preorder
 * range-minimum LCA structure, depths and the exact fixed-point root resistances.  parent: device [n], parent[root] = -1.
 * The tree keeps pointers to g's arrays; the caller keeps them alive and unchanged
 * until gss_tree_free.  Errors: ARG, NOT_SIMPLE, WEIGHT, ASYM, NOT_TREE, TREE_EDGE,
 * RANGE, HIP, OOM. */
#define GSS_PREP_TRUSTED 1u
gss_status gss_tree_prep(gss_ctx ctx, const gss_csr *g, const int32_t *parent, uint32_t flags,
                         gss_tree *out);
gss_status gss_tree_free(gss_tree tree);

/* Off-tree edge recovery (Alg. 1 Steps 1-4).
 *   mask    device uint8 [m]: 1 = recovered off-tree edge (and tree edges if
 *           GSS_F_MASK_TREE), 0 otherwise.  Required.
 *   order   device int32 [K] or NULL: recovered edge ids in recovery order.
 *   stretch device double [m] or NULL: stretch of every off-tree edge, 0 on tree edges.
 *   info    host or NULL.
 * Errors: ARG, RANGE, HIP, OOM.  Returns GSS_SHORT when M < K. */
gss_status gss_recover(gss_ctx ctx, gss_tree tree, const gss_params *params, uint8_t *mask,
                       int32_t *order, double *stretch, gss_info *info);

/* ---- allocation-free recovery -------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): gss_recover_noalloc computes exactly
 * what gss_recover computes, with the same arguments and outputs, but allocates nothing.
 * Its scratch is one static device array of GSS_NOALLOC_SCRATCH_BYTES bytes per device
 * (held from the first context on that device until the process ends); every call on a
 * device shares it, so calls that overlap on one device (other contexts or streams)
 * race and must be ordered by the caller.  The tree must come from gss_tree_prep.
 * Errors: as gss_recover; GSS_ERR_OOM with a message naming the limit when the input
 * needs more scratch than the array holds (checked before any kernel runs from the edge
 * count and K, and again as buffers are taken). */
#define GSS_NOALLOC_SCRATCH_BYTES 268435456
gss_status gss_recover_noalloc(gss_ctx ctx, gss_tree tree, const gss_params *params, uint8_t *mask,
                               int32_t *order, double *stretch, gss_info *info);

/* ---- batches: many graphs recovered by one pass of kernels -------------------------
 * gss_batch_prep copies nb graphs (host array of device CSRs, host array of device
 * parent arrays) into one disjoint union whose trees hang under a virtual root with
 * zero-resistance links, validates every graph as gss_tree_prep does, and prepares the
 * union once.  A graph with at least the batch split size of CSR entries (default 2^25,
 * gss_ctx_set_batch_split) fills the GPU by itself: it is prepared on its own, as by
 * gss_tree_prep, without a copy, and recovered by its own pass; so is a single graph
 * left over.  Edge ids, masks and orders stay per graph.  The caller keeps the arrays
 * alive and unchanged until gss_tree_free.  Errors: as gss_tree_prep. */
gss_status gss_batch_prep(gss_ctx ctx, int32_t nb, const gss_csr *graphs, const int32_t *const *parents,
                          uint32_t flags, gss_tree *out);
/* Recovers every graph of a batch tree: params, masks (device uint8 [m_g]) and orders
 * (device int32 [K_g], or NULL for the whole array or an entry) are host arrays of nb;
 * infos host [nb] or NULL.  All graphs must use the same beta and schedule.  Subtasks of
 * all graphs of the union share one work queue and one persistent launch; graphs prepared
 * on their own follow, one pass each.  Returns GSS_SHORT if any graph had fewer than K_g
 * off-tree edges. */
gss_status gss_recover_batch(gss_ctx ctx, gss_tree batch, const gss_params *params, uint8_t *const *masks,
                             int32_t *const *orders, gss_info *infos);
/* Autotuner of the work-queue settings (gss_ctx_set_tuning) for a tree (a single graph or
 * a batch) and its parameters: runs the recovery for each candidate setting (queue limit
 * local_max, workgroups local_blocks and queue chunk), timed with HIP events on the
 * context stream, keeps the fastest in the context and appends it to the text file
 * cache_path (NULL: no cache; an entry for the same device and workload is reused
 * without timing when its values pass the gss_ctx_set_tuning range checks; other entries
 * are ignored).  masks/orders as for gss_recover_batch (their contents are overwritten).
 * On an error the context keeps the settings it had before the call.  Outputs (host, may
 * be NULL): the chosen local_max, local_blocks and chunk and the best time in ms (-1
 * when taken from the cache). */
gss_status gss_autotune(gss_ctx ctx, gss_tree tree, const gss_params *params, uint8_t *const *masks,
                        int32_t *const *orders, const char *cache_path, int32_t *local_max, int32_t *local_blocks,
                        int32_t *chunk, double *best_ms);
/* Target count K of graph g of a tree under params p (one gss_params, as passed for that
 * graph): p->k_override when >= 0, else floor(alpha * n_g) with the product rounded to
 * double first (Sec. II-B: the sparsifier keeps alpha|V| off-tree edges).  This is the
 * length the order output of gss_recover / gss_recover_batch must have.  Returns -1 on a
 * bad argument. */
int64_t gss_target_count(gss_tree tree, int32_t g, const gss_params *p);
/* Number of graphs of a tree (1 for gss_tree_prep) and the edge count m_g of graph g. */
int32_t gss_tree_num_graphs(gss_tree tree);
int64_t gss_tree_graph_edges(gss_tree tree, int32_t g);

/* Diagnostics used by the parity tests (same kernels as the path above).
 *   depth  device int32 [n]; Dlo, Dhi device uint64 [n]: root resistance D(x) = (Dhi*2^64
 *   + Dlo) * 2^scale; scale host int32.  Any pointer may be NULL. */
gss_status gss_tree_export(gss_tree tree, int32_t *depth, uint64_t *Dlo, uint64_t *Dhi,
                           int32_t *scale);
/* Per-edge LCA (-1 on tree edges) and beta* (0 on tree edges) for BFS-step constant
 * beta; device int32 [m] each, either may be NULL. */
gss_status gss_edge_lca(gss_ctx ctx, gss_tree tree, int32_t beta, int32_t *lca, int32_t *bstar);

/* Returns the number of undirected edges m of a prepared tree, or -1. */
int64_t gss_tree_num_edges(gss_tree tree);

/* ---- subtask scheduling and the learned cost model --------------------------------
 * The recovery groups the resolved prefix of the criticality order into LCA subtasks
 * (paper: Lemma "strictly similar edges share their LCA", Alg. 1 Step 3).  Subtasks of at
 * most local_max edges are drained by a persistent work-queue kernel, one wavefront per
 * subtask; larger ones use a partitioned join on ancestor pairs.  The queue runs
 * longest-predicted first: by edge count (GSS_SCHED_EDGECOUNT), or by a 12-64-64-1 ReLU
 * network of 12 subtask features (GSS_SCHED_LEARNED, BF16 matrix-core inference).  The
 * order never changes the output.  Features of a subtask of S edges with LCA l:
 * log2(1+S); mean and max tree-path hop length d(u)+d(v)-2d(l); mean beta*; share of
 * beta* = 0; mean and max of deg_T(u)+deg_T(v); log2(1+deg_T(l)); log2(1+d(l));
 * S / (resolved prefix length); log2(1 + total path length); log2(1+S^2), all from exact
 * integer sums.  Only queued subtasks are ranked by cost, so only they are featurised and
 * predicted; the rows of larger subtasks are zero.  The target is
 * log2 of the cycles the work-queue kernel spent on the subtask.  Weights are
 * GSS_COSTMODEL_FLOATS floats: W1[64][12] b1[64] W2[64][64] b2[64] W3[64] b3, then the
 * feature mean[12] and standard deviation[12]. */
#define GSS_NFEAT 12
#define GSS_COSTMODEL_FLOATS 5081
#define GSS_COSTMODEL_PARAMS 5057

/* Diagnostics of the Euler-tour list ranking in gss_tree_prep.  Each level's buffers
 * have a capacity of about 1.3 times the expected ruler count; a level that outgrows it
 * is detected on the device and the ranking is repeated with twice (then four and eight
 * times) the capacities.  gss_ctx_set_rank_capacity divides the first attempt's
 * capacities by divisor (1..4; 1 is the default) so that tests can drive that retry;
 * the prepared tree is the same.  gss_tree_rank_attempts returns the number of
 * attempts the preparation of a tree took (the largest over a batch's parts), or -1. */
gss_status gss_ctx_set_rank_capacity(gss_ctx ctx, int32_t divisor);
/* Diagnostics of the short sorts of the recovery (a prefix of the criticality order, its
 * LCA grouping and the work queue; up to 524288 pairs).  They run as a sample sort: a
 * sorted sample gives bucket splitters, the pairs are counted and scattered into their
 * buckets, and one workgroup sorts each bucket, in LDS when it holds at most bucket_cap
 * pairs (0: the kernel's limit, 8192), otherwise in global memory.  radix = 1 sorts them
 * with the stable LSD radix sort of longer sorts instead.  Neither changes the output;
 * tests use them to drive every path.  Errors: ARG (radix not 0/1, bucket_cap 1 or
 * outside 0..8192). */
gss_status gss_ctx_set_sort(gss_ctx ctx, int32_t radix, int32_t bucket_cap);
int32_t gss_tree_rank_attempts(gss_tree tree);

/* Sets the batch split size (CSR entries, >= 0; 0 prepares every graph of a batch on its
 * own).  Errors: ARG. */
gss_status gss_ctx_set_batch_split(gss_ctx ctx, int64_t own_nnz);
/* Sets the work-queue limits: subtasks of at most local_max edges (0..1024; 0 sends every
 * subtask to the hash join) use the persistent kernel, which runs local_blocks (1..65536)
 * workgroups of four wavefronts; a wavefront takes chunk (1..64) queue entries per pop of
 * the queue head, or, with chunk = 0, about a sixteenth of its share of the queue (at
 * most 64).  Returns GSS_ERR_ARG outside those ranges. */
gss_status gss_ctx_set_tuning(gss_ctx ctx, int32_t local_max, int32_t local_blocks, int32_t chunk);
/* Copies up to cap rows of the context trace (host arrays feat[cap][12], cycles[cap],
 * size[cap], lca[cap] (the subtask's LCA vertex; in a batch, the vertex of the union),
 * prefix_len[cap] (the length of the criticality-order prefix the subtask was resolved
 * in); any may be NULL) and returns the number of rows held, or -1. */
int64_t gss_trace_read(gss_ctx ctx, float *feat, double *cycles, int32_t *size, int32_t *lca, int64_t *prefix_len,
                       int64_t cap);
gss_status gss_trace_clear(gss_ctx ctx);
/* Trains the cost model on the GPU (FP32 forward/backward and Adam kernels, data
 * parallel: each mini-batch is cut into 64-sample slices, one workgroup per slice, and
 * the slice gradients are summed in a fixed order, so training is deterministic) from
 * host arrays feat[n][12] and cycles[n]; the target is log2(cycles).  Mini-batches hold
 * 64 * clamp(n / 16384, 1, 64) samples; rows are visited in a seeded permutation per
 * epoch.  Adam: beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected, moments from zero.
 * flags: 0 starts from seeded random weights and the training set's feature mean and
 * standard deviation; GSS_TRAIN_WARM continues from the loaded weights and keeps their
 * normalisation (ARG if none is loaded).  loss: host [epochs] mean squared error per
 * epoch, or NULL. */
#define GSS_TRAIN_WARM 1u
gss_status gss_costmodel_train(gss_ctx ctx, const float *feat, const double *cycles, int64_t n, int32_t epochs,
                               float lr, uint64_t seed, uint32_t flags, float *loss);
/* Loads / saves the weights (host arrays of GSS_COSTMODEL_FLOATS floats). */
gss_status gss_costmodel_load(gss_ctx ctx, const float *weights);
gss_status gss_costmodel_save(gss_ctx ctx, float *weights);
/* BF16 inference: out[i] = predicted log2(cycles) of device feat[i][12], device out[n]. */
gss_status gss_costmodel_predict(gss_ctx ctx, const float *feat, int64_t n, float *out);
/* FP32 gradient of the mean squared error of host batch x[nb][12] (raw features), targets
 * y[nb] (1 <= nb <= 64) at the current weights: grad host [GSS_COSTMODEL_PARAMS]. */
gss_status gss_costmodel_grad(gss_ctx ctx, const float *x, const float *y, int32_t nb, float *grad, float *loss);

/* Live kernel timing (diagnostics): every launch of the selected kernels is bracketed by
 * HIP events on the context stream and the elapsed times are summed per kernel.
 * enable = 0 turns timing off; kernel_name NULL or "" selects every kernel.  Each call
 * clears the accumulated figures. */
gss_status gss_ctx_profile(gss_ctx ctx, int32_t enable, const char *kernel_name);
/* Reads accumulated entry idx: its kernel name (copied into buf, NUL-terminated), total
 * milliseconds, launch count, the algorithmic bytes of those launches (the least HBM
 * traffic each launch's step needs: inputs read once, outputs written once; 0 for kernels
 * without such a model) and the milliseconds of the latest launch.  Any output pointer
 * may be NULL.  Returns the number of entries, -1 on a bad argument. */
int32_t gss_ctx_profile_read(gss_ctx ctx, int32_t idx, char *buf, int32_t buflen, double *total_ms,
                             int64_t *launches, int64_t *alg_bytes, double *last_ms);

/* ---- spanning tree: the step before the recovery ----------------------------------
 * feGRASS's spanning tree (Sec. II-B "feGRASS Algorithm"; Def. "Effective weight",
 * eq. weff): root = the vertex of largest degree (the smallest id among ties); unweighted
 * breadth-first distances dist from it; per edge W_eff = w * log(max(deg u, deg v)) /
 * (dist u + dist v) (natural log, each operation rounded once); the maximum spanning
 * tree under the total order (W_eff descending, edge id ascending), rooted at root.
 * With flags = GSS_TREE_WEIGHT the order is by w itself (a maximum-weight spanning
 * tree; same root).  g: device CSR as for gss_tree_prep, and connected.  parent: device
 * int32 [n], receives the tree (-1 at the root), ready for gss_tree_prep; root: host
 * int32, receives the root; weff: device double [m] indexed by edge id (the ordering
 * weight of every edge), or NULL.  Errors: GSS_ERR_ARG (sizes, an unordered row, a
 * column out of range or on the diagonal, a graph that is not connected),
 * GSS_ERR_ASYM (an odd number of upper entries against nnz). */
#define GSS_TREE_WEIGHT 1u
gss_status gss_spanning_tree(gss_ctx ctx, const gss_csr *g, uint32_t flags, int32_t *parent, int32_t *root,
                             double *weff);

/* ---- memoized graph capture of recoveries ------------------------------------------
 * With enable = 1, gss_recover and gss_recover_batch remember each call's key: the tree,
 * the parameters, the output pointers and the context's settings (work-queue tuning,
 * sort settings, cost model).  The first call with a key runs eagerly and records every
 * value the host reads back; the second runs the same host code with the context stream
 * in capture mode, each read-back replaced by its recorded value plus a device-side
 * comparison with it, then launches the resulting HIP graph; every later call with the key
 * replays that graph: one launch and one host synchronisation.  Outputs and infos are
 * those of an eager call, since a recovery is a function of its key: a tree's arrays may
 * not change until gss_tree_free, which drops the tree's graphs.  Should a replayed value
 * ever differ from the recorded one, the graph is dropped and the call reruns eagerly.
 * Calls with GSS_F_RECORD, calls while kernel timing is on, and gss_recover_noalloc always
 * run eagerly.  At most 8 keys are kept per context (the oldest is dropped); each captured
 * key holds its own scratch arena (the recording call's peak) until dropped.  enable = 0
 * drops every graph.  Errors: GSS_ERR_ARG. */
gss_status gss_ctx_set_capture(gss_ctx ctx, int32_t enable);
/* Counts since the context was created: recording (eager) calls, captures, replays, and
 * host synchronisations of the context stream.  Any pointer may be NULL. */
gss_status gss_ctx_capture_stats(gss_ctx ctx, int64_t *records, int64_t *captures, int64_t *replays,
                                 int64_t *syncs);

/* Library-owned, static strings. */
const char *gss_status_str(gss_status s);
const char *gss_last_error(gss_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* GSS_H */
