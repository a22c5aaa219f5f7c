/*
 * gss_oracle.c -- plain serial CPU oracle for pdGRASS off-tree edge recovery.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The GPU library never links,
 * includes or calls it, and it shares no code, header or table with the GPU path.
 *
 * What it computes (paper: Sec. II-B, Sec. III-A, Sec. IV-B, Alg. 1):
 *   O1  validate the CSR graph, enumerate undirected edges (u<v); the edge id is the
 *       rank of (u,v) among the upper-triangle CSR entries (rows, then columns).
 *   O2  tree edges are {(x, parent x)}; all other edges are off-tree (Sec. II-B).
 *   O3  depth by BFS from the root over the tree.
 *   O4  resistive weight of each tree edge, t = RN(1/w)  (Def. "Resistance distance").
 *   O5  root-to-node resistance D(x) = sum of t on the root->x path, summed EXACTLY in
 *       128-bit fixed point at scale 2^s, s = (smallest exponent of any t) - 52.
 *   O6  LCA by binary lifting (the "skip table" of Alg. 1, Step 1).
 *   O7  R_T(u,v) = RN(D(u) + D(v) - 2 D(lca))  (eq. RT), stretch = RN(w * R_T),
 *       beta* = min(dist(u,lca), dist(v,lca), c)  (eq. beta-new; dist = tree hops).
 *   O8  criticality order pi: stretch descending, edge id ascending (Alg. 1 Step 2).
 *   O9  one serial greedy pass over pi: an unmarked edge is recovered, and every later
 *       undecided off-tree edge (u',v') with (u' in S_u and v' in S_v) or
 *       (u' in S_v and v' in S_u) is marked, where S_x is the beta*-hop BFS ball of x
 *       on the tree (Def. "Similar edge (Strict)", Def. "BFS step size").  Stop at
 *       K = floor(alpha*|V|) recovered edges.  If a pass ends short, a new pass runs
 *       over the unrecovered edges with all marks cleared (feGRASS multi-pass rule,
 *       Sec. II-B).
 *
 * Variants (bit flags, each from its own passage of the paper):
 *   ORC_KEY_RT   O8 sorts by the tree-path resistance R_T itself, the literal wording of
 *                Alg. 1 Step 2 ("sort L based on resistances"), instead of the stretch.
 *   ORC_LOOSE    O9 uses feGRASS's loose condition (Def. "Similar edge (Loose)", eq.
 *                cond-loose-2): with balls of the constant radius c around u and v, every
 *                later off-tree edge with EITHER endpoint in S_u or S_v is marked.  Passes
 *                repeat with marks cleared (the multi-pass rule of Sec. II-B).  The LCA
 *                lemma does not hold for it, so it has no subtask mode.
 *
 * Marking enumeration modes (must agree):
 *   ORC_MODE_INDEXED  -- scan the graph rows of every ball vertex except lca(e).
 *   ORC_MODE_BRUTE    -- test every later off-tree edge in pi.
 *   ORC_MODE_SUBTASK  -- group edges by LCA (Lemma "strictly similar edges share their
 *                        LCA"), run the greedy inside every group to completion, then
 *                        take candidates in pi order.  Used only to cross-check that the
 *                        subtask decomposition reaches the serial result.
 *
 * Floating point: FP64, round-to-nearest, no contraction (build with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef unsigned __int128 u128;

/* status codes (values are part of the library interface) */
enum {
    ORC_OK = 0, ORC_SHORT = 1,
    ORC_ERR_ARG = -1, ORC_ERR_NOT_SIMPLE = -2, ORC_ERR_ASYM = -3, ORC_ERR_WEIGHT = -4,
    ORC_ERR_NOT_TREE = -5, ORC_ERR_TREE_EDGE = -6, ORC_ERR_RANGE = -7, ORC_ERR_OOM = -9
};
enum { ORC_MODE_INDEXED = 0, ORC_MODE_BRUTE = 1, ORC_MODE_SUBTASK = 2 };
enum { ORC_KEY_RT = 1, ORC_LOOSE = 2 };

/* info[] slots */
enum {
    INF_M = 0, INF_NOFF, INF_K, INF_NREC, INF_PASSES, INF_NSUB, INF_LARGEST,
    INF_BALL_VERTS, INF_ROW_ENTRIES, INF_SCALE, INF_LEN
};

static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* index of `key` in the sorted row [lo,hi) of col, or -1 */
static int64_t find_in_row(const int32_t *col, int64_t lo, int64_t hi, int32_t key)
{
    const int64_t end = hi;
    while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (col[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && col[lo] == key) ? lo : -1;
}

/* ---------------------------------------------------------------------------------- */
/* state shared by the steps of one run                                                */
/* ---------------------------------------------------------------------------------- */
typedef struct {
    int32_t n;
    const int32_t *row_ptr, *col;
    const double *w;
    const int32_t *parent;
    int64_t nnz, m, M;
    int32_t root, c;
    int32_t variant;           /* ORC_KEY_RT | ORC_LOOSE */
    /* edges */
    int32_t *eu, *ev;          /* [m] */
    double *ew;                /* [m] */
    int32_t *eid_entry;        /* [nnz] edge id of each CSR entry */
    uint8_t *is_tree;          /* [m] */
    int32_t *off;              /* [M] off-tree edge ids in id order */
    /* tree */
    int32_t *cptr, *clist;     /* children CSR */
    int32_t *depth;            /* [n] */
    u128 *D;                   /* [n] fixed-point root resistance */
    int32_t scale;             /* s: D is in units of 2^s */
    int32_t **up; int32_t levels;
    /* per edge */
    int32_t *lca, *bstar;      /* [m] */
    double *stretch;           /* [m] */
    double *res;               /* [m] R_T of each off-tree edge */
    int32_t *pi;               /* [M] */
    int32_t *rank_of;          /* [m] */
} run_t;

static void run_free(run_t *r)
{
    free(r->eu); free(r->ev); free(r->ew); free(r->eid_entry); free(r->is_tree); free(r->off);
    free(r->cptr); free(r->clist); free(r->depth); free(r->D);
    if (r->up) { for (int i = 0; i < r->levels; i++) free(r->up[i]); free(r->up); }
    free(r->lca); free(r->bstar); free(r->stretch); free(r->res); free(r->pi); free(r->rank_of);
}

/* O1: validation and edge enumeration */
static int step_edges(run_t *r)
{
    const int32_t n = r->n, *rp = r->row_ptr, *col = r->col;
    const double *w = r->w;
    if (n < 1 || !rp || !col || !w || !r->parent) return ORC_ERR_ARG;
    if (rp[0] != 0) return ORC_ERR_ARG;
    for (int32_t u = 0; u < n; u++)
        if (rp[u + 1] < rp[u]) return ORC_ERR_ARG;
    r->nnz = rp[n];
    for (int64_t k = 0; k < r->nnz; k++)
        if (col[k] < 0 || col[k] >= n) return ORC_ERR_ARG;
    for (int32_t u = 0; u < n; u++)
        for (int64_t k = rp[u]; k < rp[u + 1]; k++) {
            if (col[k] == u) return ORC_ERR_NOT_SIMPLE;
            if (k > rp[u] && col[k] <= col[k - 1]) return ORC_ERR_NOT_SIMPLE;
        }
    for (int64_t k = 0; k < r->nnz; k++)
        if (!isfinite(w[k]) || !(w[k] > 0.0)) return ORC_ERR_WEIGHT;
    for (int32_t u = 0; u < n; u++)
        for (int64_t k = rp[u]; k < rp[u + 1]; k++) {
            int32_t v = col[k];
            int64_t j = find_in_row(col, rp[v], rp[v + 1], u);
            if (j < 0 || w[j] != w[k]) return ORC_ERR_ASYM;
        }
    r->m = r->nnz / 2;
    r->eu = malloc(sizeof(int32_t) * (size_t)(r->m + 1));
    r->ev = malloc(sizeof(int32_t) * (size_t)(r->m + 1));
    r->ew = malloc(sizeof(double) * (size_t)(r->m + 1));
    r->eid_entry = malloc(sizeof(int32_t) * (size_t)(r->nnz + 1));
    if (!r->eu || !r->ev || !r->ew || !r->eid_entry) return ORC_ERR_OOM;
    int64_t id = 0;
    for (int32_t u = 0; u < n; u++)
        for (int64_t k = rp[u]; k < rp[u + 1]; k++) {
            int32_t v = col[k];
            if (v > u) {
                r->eu[id] = u; r->ev[id] = v; r->ew[id] = w[k];
                r->eid_entry[k] = (int32_t)id;
                id++;
            } else {
                /* (v,u) with v<u was numbered while scanning row v */
                int64_t j = find_in_row(col, rp[v], rp[v + 1], u);
                r->eid_entry[k] = r->eid_entry[j];
            }
        }
    return ORC_OK;
}

/* O2-O5: tree checks, depth, exact root resistance */
static int step_tree(run_t *r)
{
    const int32_t n = r->n, *par = r->parent, *rp = r->row_ptr, *col = r->col;
    int32_t roots = 0;
    r->root = -1;
    for (int32_t x = 0; x < n; x++) {
        if (par[x] == -1) { roots++; r->root = x; }
        else if (par[x] < 0 || par[x] >= n || par[x] == x) return ORC_ERR_NOT_TREE;
    }
    if (roots != 1) return ORC_ERR_NOT_TREE;
    r->cptr = calloc((size_t)n + 1, sizeof(int32_t));
    r->clist = malloc(sizeof(int32_t) * (size_t)(n > 1 ? n - 1 : 1));
    r->depth = malloc(sizeof(int32_t) * (size_t)n);
    r->D = malloc(sizeof(u128) * (size_t)n);
    int32_t *fill = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *queue = malloc(sizeof(int32_t) * (size_t)n);
    if (!r->cptr || !r->clist || !r->depth || !r->D || !fill || !queue) {
        free(fill); free(queue); return ORC_ERR_OOM;
    }
    for (int32_t x = 0; x < n; x++)
        if (par[x] >= 0) r->cptr[par[x] + 1]++;
    for (int32_t x = 0; x < n; x++) r->cptr[x + 1] += r->cptr[x];
    memcpy(fill, r->cptr, sizeof(int32_t) * (size_t)(n + 1));
    for (int32_t x = 0; x < n; x++)
        if (par[x] >= 0) r->clist[fill[par[x]]++] = x;
    /* BFS from the root: every vertex must be reached exactly once */
    int32_t head = 0, tail = 0;
    queue[tail++] = r->root;
    r->depth[r->root] = 0;
    while (head < tail) {
        int32_t x = queue[head++];
        for (int32_t k = r->cptr[x]; k < r->cptr[x + 1]; k++) {
            int32_t y = r->clist[k];
            r->depth[y] = r->depth[x] + 1;
            queue[tail++] = y;
        }
    }
    free(fill);
    if (tail != n) { free(queue); return ORC_ERR_NOT_TREE; }
    /* tree edges must be edges of G */
    r->is_tree = calloc((size_t)r->m + 1, 1);
    double *tw = malloc(sizeof(double) * (size_t)n);
    if (!r->is_tree || !tw) { free(queue); free(tw); return ORC_ERR_OOM; }
    for (int32_t x = 0; x < n; x++) {
        if (x == r->root) continue;
        int64_t k = find_in_row(col, rp[x], rp[x + 1], par[x]);
        if (k < 0) { free(queue); free(tw); return ORC_ERR_TREE_EDGE; }
        r->is_tree[r->eid_entry[k]] = 1;
        tw[x] = r->w[k];
    }
    /* O4: t = RN(1/w); the fixed-point scale needs normal, finite terms */
    int emin = INT32_MAX, emax = INT32_MIN;
    double *t = tw; /* reuse storage: t[x] replaces w(x,parent x) */
    for (int32_t x = 0; x < n; x++) {
        if (x == r->root) continue;
        t[x] = 1.0 / tw[x];
        if (!isnormal(t[x])) { free(queue); free(tw); return ORC_ERR_RANGE; }
        int e = ilogb(t[x]);
        if (e < emin) emin = e;
        if (e > emax) emax = e;
    }
    if (n == 1) { emin = 0; emax = 0; }
    if (emax - emin > 74) { free(queue); free(tw); return ORC_ERR_RANGE; }
    r->scale = emin - 52;
    /* O5: exact sums along root paths, in BFS order (parents before children) */
    const u128 limit = ((u128)1) << 127;
    u128 total = 0;
    r->D[r->root] = 0;
    for (int32_t i = 1; i < n; i++) {
        int32_t x = queue[i];
        int e = ilogb(t[x]);
        uint64_t mant = (uint64_t)ldexp(t[x], 52 - e);   /* exact: 53-bit integer */
        u128 T = ((u128)mant) << (e - emin);
        if (T >= limit - total) { free(queue); free(tw); return ORC_ERR_RANGE; }
        total += T;
        r->D[x] = r->D[par[x]] + T;
    }
    free(queue);
    free(tw);
    /* off-tree list in id order */
    r->M = r->m - (n - 1);
    r->off = malloc(sizeof(int32_t) * (size_t)(r->M + 1));
    if (!r->off) return ORC_ERR_OOM;
    int64_t j = 0;
    for (int64_t e = 0; e < r->m; e++)
        if (!r->is_tree[e]) r->off[j++] = (int32_t)e;
    return ORC_OK;
}

/* O6: binary lifting table */
static int step_lifting(run_t *r)
{
    int32_t maxd = 0;
    for (int32_t x = 0; x < r->n; x++)
        if (r->depth[x] > maxd) maxd = r->depth[x];
    int L = 1;
    while ((1 << L) <= maxd) L++;
    r->levels = L;
    r->up = calloc((size_t)L, sizeof(int32_t *));
    if (!r->up) return ORC_ERR_OOM;
    for (int k = 0; k < L; k++) {
        r->up[k] = malloc(sizeof(int32_t) * (size_t)r->n);
        if (!r->up[k]) return ORC_ERR_OOM;
    }
    for (int32_t x = 0; x < r->n; x++)
        r->up[0][x] = (r->parent[x] < 0) ? x : r->parent[x];
    for (int k = 1; k < L; k++)
        for (int32_t x = 0; x < r->n; x++)
            r->up[k][x] = r->up[k - 1][r->up[k - 1][x]];
    return ORC_OK;
}

static int32_t lca_query(const run_t *r, int32_t a, int32_t b)
{
    if (r->depth[a] < r->depth[b]) { int32_t t = a; a = b; b = t; }
    int32_t diff = r->depth[a] - r->depth[b];
    for (int k = 0; k < r->levels; k++)
        if ((diff >> k) & 1) a = r->up[k][a];
    if (a == b) return a;
    for (int k = r->levels - 1; k >= 0; k--)
        if (r->up[k][a] != r->up[k][b]) { a = r->up[k][a]; b = r->up[k][b]; }
    return r->up[0][a];
}

/* O7: LCA, resistance, stretch and beta* of every off-tree edge */
static int step_stretch(run_t *r)
{
    r->lca = malloc(sizeof(int32_t) * (size_t)(r->m + 1));
    r->bstar = malloc(sizeof(int32_t) * (size_t)(r->m + 1));
    r->stretch = malloc(sizeof(double) * (size_t)(r->m + 1));
    r->res = malloc(sizeof(double) * (size_t)(r->m + 1));
    if (!r->lca || !r->bstar || !r->stretch || !r->res) return ORC_ERR_OOM;
    for (int64_t e = 0; e < r->m; e++) { r->lca[e] = -1; r->bstar[e] = 0; r->stretch[e] = 0.0; r->res[e] = 0.0; }
    for (int64_t j = 0; j < r->M; j++) {
        int32_t e = r->off[j], u = r->eu[e], v = r->ev[e];
        int32_t l = lca_query(r, u, v);
        u128 Rfix = (r->D[u] - r->D[l]) + (r->D[v] - r->D[l]);
        double R = ldexp((double)Rfix, r->scale);       /* one correctly rounded conversion */
        double s = r->ew[e] * R;
        if (!isfinite(R) || !isfinite(s)) return ORC_ERR_RANGE;
        int32_t du = r->depth[u] - r->depth[l], dv = r->depth[v] - r->depth[l];
        int32_t b = du < dv ? du : dv;
        if (r->c < b) b = r->c;
        r->lca[e] = l; r->bstar[e] = b; r->stretch[e] = s; r->res[e] = R;
    }
    return ORC_OK;
}

/* O8: criticality order (key: the stretch, or R_T with ORC_KEY_RT) */
static const run_t *g_sort_run;
static int cmp_pi(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    const double *key = (g_sort_run->variant & ORC_KEY_RT) ? g_sort_run->res : g_sort_run->stretch;
    double sa = key[a], sb = key[b];
    if (sa > sb) return -1;
    if (sa < sb) return 1;
    return (a < b) ? -1 : (a > b);
}

static int step_sort(run_t *r)
{
    r->pi = malloc(sizeof(int32_t) * (size_t)(r->M + 1));
    r->rank_of = malloc(sizeof(int32_t) * (size_t)(r->m + 1));
    if (!r->pi || !r->rank_of) return ORC_ERR_OOM;
    memcpy(r->pi, r->off, sizeof(int32_t) * (size_t)r->M);
    g_sort_run = r;
    qsort(r->pi, (size_t)r->M, sizeof(int32_t), cmp_pi);
    for (int64_t e = 0; e < r->m; e++) r->rank_of[e] = -1;
    for (int64_t i = 0; i < r->M; i++) r->rank_of[r->pi[i]] = (int32_t)i;
    return ORC_OK;
}

/* beta-hop BFS ball on the tree; fills list and stamps, returns its size */
static int64_t tree_ball(const run_t *r, int32_t src, int32_t radius, int32_t *stamp, int32_t cur,
                         int32_t *list, int32_t *dist)
{
    int64_t head = 0, tail = 0;
    list[tail++] = src; stamp[src] = cur; dist[0] = 0;
    while (head < tail) {
        int32_t x = list[head];
        int32_t d = dist[head];
        head++;
        if (d == radius) continue;
        int32_t p = r->parent[x];
        if (p >= 0 && stamp[p] != cur) { stamp[p] = cur; list[tail] = p; dist[tail] = d + 1; tail++; }
        for (int32_t k = r->cptr[x]; k < r->cptr[x + 1]; k++) {
            int32_t y = r->clist[k];
            if (stamp[y] != cur) { stamp[y] = cur; list[tail] = y; dist[tail] = d + 1; tail++; }
        }
    }
    return tail;
}

typedef struct {
    int32_t *stampU, *stampV, *listU, *listV, *distU, *distV;
    int32_t cur;
    int64_t ball_verts, row_entries;
} balls_t;

static int balls_init(balls_t *b, int32_t n)
{
    b->stampU = calloc((size_t)n, sizeof(int32_t));
    b->stampV = calloc((size_t)n, sizeof(int32_t));
    b->listU = malloc(sizeof(int32_t) * (size_t)n);
    b->listV = malloc(sizeof(int32_t) * (size_t)n);
    b->distU = malloc(sizeof(int32_t) * (size_t)n);
    b->distV = malloc(sizeof(int32_t) * (size_t)n);
    b->cur = 0; b->ball_verts = 0; b->row_entries = 0;
    return (b->stampU && b->stampV && b->listU && b->listV && b->distU && b->distV) ? ORC_OK
                                                                                    : ORC_ERR_OOM;
}

static void balls_free(balls_t *b)
{
    free(b->stampU); free(b->stampV); free(b->listU); free(b->listV); free(b->distU); free(b->distV);
}

/* is off-tree edge f strictly similar to the edge whose balls are currently stamped? */
static inline int similar_now(const run_t *r, const balls_t *b, int32_t f)
{
    int32_t x = r->eu[f], y = r->ev[f];
    return (b->stampU[x] == b->cur && b->stampV[y] == b->cur) ||
           (b->stampV[x] == b->cur && b->stampU[y] == b->cur);
}

/* loosely similar (eq. cond-loose-2): an endpoint of f lies in S_u or in S_v */
static inline int loose_now(const balls_t *b, const run_t *r, int32_t f)
{
    int32_t x = r->eu[f], y = r->ev[f];
    return b->stampU[x] == b->cur || b->stampV[x] == b->cur || b->stampU[y] == b->cur || b->stampV[y] == b->cur;
}

/* O9 in the two global modes */
static int step_greedy_global(run_t *r, int mode, int64_t K, uint8_t *rec_pass, int32_t *order,
                              int64_t *nrec_out, int32_t *passes_out, balls_t *b)
{
    uint8_t *marked = malloc((size_t)r->m + 1);
    if (!marked) return ORC_ERR_OOM;
    int64_t nrec = 0;
    int32_t passes = 0;
    while (nrec < K) {
        memset(marked, 0, (size_t)r->m + 1);
        int64_t got = 0;
        for (int64_t i = 0; i < r->M && nrec < K; i++) {
            int32_t e = r->pi[i];
            if (rec_pass[e] || marked[e]) continue;
            rec_pass[e] = (uint8_t)(passes + 1 > 255 ? 255 : passes + 1);
            order[nrec++] = e;
            got++;
            int32_t u = r->eu[e], v = r->ev[e], l = r->lca[e], beta = r->bstar[e];
            const int loose = (r->variant & ORC_LOOSE) != 0;
            if (loose) beta = r->c;  /* feGRASS: the constant BFS step c */
            b->cur++;
            int64_t nu = tree_ball(r, u, beta, b->stampU, b->cur, b->listU, b->distU);
            int64_t nv = tree_ball(r, v, beta, b->stampV, b->cur, b->listV, b->distV);
            b->ball_verts += nu + nv;
            if (loose && mode == ORC_MODE_BRUTE) {
                for (int64_t j = i + 1; j < r->M; j++) {
                    int32_t f = r->pi[j];
                    if (!rec_pass[f] && loose_now(b, r, f)) marked[f] = 1;
                }
            } else if (loose) {
                /* every off-tree edge incident to a vertex of S_u or S_v */
                for (int side = 0; side < 2; side++) {
                    const int32_t *list = side ? b->listV : b->listU;
                    int64_t cnt = side ? nv : nu;
                    for (int64_t q = 0; q < cnt; q++) {
                        int32_t x = list[q];
                        for (int64_t k = r->row_ptr[x]; k < r->row_ptr[x + 1]; k++) {
                            int32_t f = r->eid_entry[k];
                            b->row_entries++;
                            if (r->is_tree[f]) continue;
                            if (r->rank_of[f] > i && !rec_pass[f]) marked[f] = 1;
                        }
                    }
                }
            } else if (mode == ORC_MODE_BRUTE) {
                for (int64_t j = i + 1; j < r->M; j++) {
                    int32_t f = r->pi[j];
                    if (!rec_pass[f] && similar_now(r, b, f)) marked[f] = 1;
                }
            } else {
                for (int side = 0; side < 2; side++) {
                    const int32_t *list = side ? b->listV : b->listU;
                    const int32_t *other = side ? b->stampU : b->stampV;
                    int64_t cnt = side ? nv : nu;
                    for (int64_t q = 0; q < cnt; q++) {
                        int32_t x = list[q];
                        if (x == l) continue;
                        for (int64_t k = r->row_ptr[x]; k < r->row_ptr[x + 1]; k++) {
                            int32_t f = r->eid_entry[k];
                            b->row_entries++;
                            if (r->is_tree[f] || other[r->col[k]] != b->cur) continue;
                            if (r->rank_of[f] > i && !rec_pass[f]) marked[f] = 1;
                        }
                    }
                }
            }
        }
        if (got == 0) break;
        passes++;
    }
    free(marked);
    *nrec_out = nrec;
    *passes_out = passes;
    return ORC_OK;
}

/* O9 via LCA subtasks (cross-check mode) */
static int step_greedy_subtask(run_t *r, int64_t K, uint8_t *rec_pass, int32_t *order,
                               int64_t *nrec_out, int32_t *passes_out, balls_t *b)
{
    int32_t n = r->n;
    int64_t M = r->M;
    int32_t *gptr = calloc((size_t)n + 1, sizeof(int32_t));
    int32_t *gfill = malloc(sizeof(int32_t) * ((size_t)n + 1));
    int32_t *grp = malloc(sizeof(int32_t) * ((size_t)M + 1));
    uint8_t *marked = malloc((size_t)r->m + 1);
    uint8_t *cand = malloc((size_t)r->m + 1);
    if (!gptr || !gfill || !grp || !marked || !cand) {
        free(gptr); free(gfill); free(grp); free(marked); free(cand); return ORC_ERR_OOM;
    }
    /* stable counting sort of pi by LCA: each group keeps pi order */
    for (int64_t i = 0; i < M; i++) gptr[r->lca[r->pi[i]] + 1]++;
    for (int32_t x = 0; x < n; x++) gptr[x + 1] += gptr[x];
    memcpy(gfill, gptr, sizeof(int32_t) * ((size_t)n + 1));
    for (int64_t i = 0; i < M; i++) grp[gfill[r->lca[r->pi[i]]]++] = r->pi[i];
    int64_t nrec = 0;
    int32_t passes = 0;
    while (nrec < K) {
        memset(marked, 0, (size_t)r->m + 1);
        memset(cand, 0, (size_t)r->m + 1);
        for (int32_t l = 0; l < n; l++) {
            for (int32_t a = gptr[l]; a < gptr[l + 1]; a++) {
                int32_t e = grp[a];
                if (rec_pass[e] || marked[e]) continue;
                cand[e] = 1;
                b->cur++;
                tree_ball(r, r->eu[e], r->bstar[e], b->stampU, b->cur, b->listU, b->distU);
                tree_ball(r, r->ev[e], r->bstar[e], b->stampV, b->cur, b->listV, b->distV);
                for (int32_t q = a + 1; q < gptr[l + 1]; q++) {
                    int32_t f = grp[q];
                    if (!rec_pass[f] && similar_now(r, b, f)) marked[f] = 1;
                }
            }
        }
        int64_t got = 0;
        for (int64_t i = 0; i < M && nrec < K; i++) {
            int32_t e = r->pi[i];
            if (cand[e] && !rec_pass[e]) {
                rec_pass[e] = (uint8_t)(passes + 1 > 255 ? 255 : passes + 1);
                order[nrec++] = e;
                got++;
            }
        }
        if (got == 0) break;
        passes++;
    }
    free(gptr); free(gfill); free(grp); free(marked); free(cand);
    *nrec_out = nrec;
    *passes_out = passes;
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------- */
/* public entry point                                                                  */
/* ---------------------------------------------------------------------------------- */

/* Number of undirected edges a valid input has (nnz/2); sizes the per-edge outputs. */
int64_t orc_num_edges(int32_t n, const int32_t *row_ptr)
{
    if (n < 1 || !row_ptr) return -1;
    return (int64_t)row_ptr[n] / 2;
}

/*
 * Runs O1-O10.  Every output pointer may be NULL.
 *   mask[m]       1 = recovered off-tree edge
 *   order[K]      recovered edge ids in recovery order (K = floor(alpha*n) or k_override)
 *   pass_of[m]    pass in which the edge was recovered (0 = not recovered)
 *   stretch[m], lca[m], bstar[m]: per edge (tree edges: 0, -1, 0)
 *   eu[m], ev[m], is_tree[m]: enumerated edges
 *   depth[n]; Dlo[n], Dhi[n]: the 128-bit fixed-point root resistance; rank_of[m]
 *   info[INF_LEN]; times[4] = step 1 (tree+LCA+stretch), step 2 (sort),
 *   step 3 (grouping count), step 4 (greedy), seconds.
 *   variant: ORC_KEY_RT and/or ORC_LOOSE (0: the method as the paper states it).
 */
int orc_recover(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *w,
                const int32_t *parent, double alpha, int32_t c, int64_t k_override, int32_t mode,
                int32_t variant, uint8_t *mask, int32_t *order, uint8_t *pass_of, double *stretch,
                int32_t *lca, int32_t *bstar, int32_t *eu, int32_t *ev, uint8_t *is_tree, int32_t *depth,
                uint64_t *Dlo, uint64_t *Dhi, int32_t *rank_of, int64_t *info, double *times)
{
    run_t r;
    memset(&r, 0, sizeof r);
    r.n = n; r.row_ptr = row_ptr; r.col = col; r.w = w; r.parent = parent; r.c = c; r.variant = variant;
    if (!(alpha >= 0.0 && alpha <= 1.0) || c < 0 || mode < 0 || mode > 2) return ORC_ERR_ARG;
    if ((variant & ~(ORC_KEY_RT | ORC_LOOSE)) || ((variant & ORC_LOOSE) && mode == ORC_MODE_SUBTASK))
        return ORC_ERR_ARG;
    double t0 = now_s();
    int st = step_edges(&r);
    if (st == ORC_OK) st = step_tree(&r);
    if (st == ORC_OK) st = step_lifting(&r);
    if (st == ORC_OK) st = step_stretch(&r);
    double t1 = now_s();
    if (st == ORC_OK) st = step_sort(&r);
    double t2 = now_s();
    if (st != ORC_OK) { run_free(&r); return st; }

    /* Step 3 statistics: LCA groups */
    int64_t nsub = 0, largest = 0;
    {
        int32_t *cnt = calloc((size_t)n, sizeof(int32_t));
        if (!cnt) { run_free(&r); return ORC_ERR_OOM; }
        for (int64_t j = 0; j < r.M; j++) cnt[r.lca[r.off[j]]]++;
        for (int32_t x = 0; x < n; x++)
            if (cnt[x]) { nsub++; if (cnt[x] > largest) largest = cnt[x]; }
        free(cnt);
    }
    double t3 = now_s();

    int64_t K = (k_override >= 0) ? k_override : (int64_t)floor(alpha * (double)n);
    uint8_t *rec_pass = calloc((size_t)r.m + 1, 1);
    int32_t *ord = malloc(sizeof(int32_t) * (size_t)(K + 1));
    balls_t b;
    memset(&b, 0, sizeof b);
    if (!rec_pass || !ord || balls_init(&b, n) != ORC_OK) {
        free(rec_pass); free(ord); balls_free(&b); run_free(&r); return ORC_ERR_OOM;
    }
    int64_t nrec = 0;
    int32_t passes = 0;
    if (mode == ORC_MODE_SUBTASK) st = step_greedy_subtask(&r, K, rec_pass, ord, &nrec, &passes, &b);
    else st = step_greedy_global(&r, mode, K, rec_pass, ord, &nrec, &passes, &b);
    double t4 = now_s();
    if (st == ORC_OK) {
        if (mask) for (int64_t e = 0; e < r.m; e++) mask[e] = rec_pass[e] ? 1 : 0;
        if (pass_of) memcpy(pass_of, rec_pass, (size_t)r.m);
        if (order) memcpy(order, ord, sizeof(int32_t) * (size_t)nrec);
        if (stretch) memcpy(stretch, r.stretch, sizeof(double) * (size_t)r.m);
        if (lca) memcpy(lca, r.lca, sizeof(int32_t) * (size_t)r.m);
        if (bstar) memcpy(bstar, r.bstar, sizeof(int32_t) * (size_t)r.m);
        if (eu) memcpy(eu, r.eu, sizeof(int32_t) * (size_t)r.m);
        if (ev) memcpy(ev, r.ev, sizeof(int32_t) * (size_t)r.m);
        if (is_tree) memcpy(is_tree, r.is_tree, (size_t)r.m);
        if (depth) memcpy(depth, r.depth, sizeof(int32_t) * (size_t)n);
        if (Dlo || Dhi)
            for (int32_t x = 0; x < n; x++) {
                if (Dlo) Dlo[x] = (uint64_t)r.D[x];
                if (Dhi) Dhi[x] = (uint64_t)(r.D[x] >> 64);
            }
        if (rank_of) memcpy(rank_of, r.rank_of, sizeof(int32_t) * (size_t)r.m);
        if (info) {
            info[INF_M] = r.m; info[INF_NOFF] = r.M; info[INF_K] = K; info[INF_NREC] = nrec;
            info[INF_PASSES] = passes; info[INF_NSUB] = nsub; info[INF_LARGEST] = largest;
            info[INF_BALL_VERTS] = b.ball_verts; info[INF_ROW_ENTRIES] = b.row_entries;
            info[INF_SCALE] = r.scale;
        }
        if (times) { times[0] = t1 - t0; times[1] = t2 - t1; times[2] = t3 - t2; times[3] = t4 - t3; }
        st = (nrec < K) ? ORC_SHORT : ORC_OK;
    }
    free(rec_pass); free(ord); balls_free(&b); run_free(&r);
    return st;
}
