/*
 * gss_oracle_tree.c -- plain serial CPU oracle for feGRASS's spanning tree, the step
 * before the recovery (Sec. II-B "feGRASS Algorithm", Def. "Effective weight", eq. weff).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite loads this library (built together with
 * gss_oracle.c); the GPU library never links, includes or calls it, and it shares no
 * code, header or table with the GPU path.
 *
 * What it computes:
 *   T1  deg(x) = number of neighbours of x in G; root = the vertex of largest degree,
 *       the smallest id among ties (the definition names "the vertex with the maximum
 *       degree"; ties are not discussed).
 *   T2  dist_G(root, x), the unweighted distance, by breadth-first search in G.
 *   T3  for every edge e = (u, v):
 *         W_eff(e) = RN( RN(w_e * log(max(deg u, deg v))) / (dist u + dist v) )
 *       with the natural logarithm (eq. weff; any base scales every W_eff alike and
 *       leaves the tree unchanged).  Edge ids as in gss_oracle.c: the rank of (u, v),
 *       u < v, among the upper-triangle CSR entries.
 *   T4  the maximum spanning tree under the total order (W_eff descending, edge id
 *       ascending), by Kruskal's algorithm with union-find (a total order makes the
 *       maximum spanning tree unique).
 *   T5  parent[] of that tree rooted at root, by breadth-first search over its edges.
 * With plain != 0 the order in T4 is by w itself (a maximum-weight spanning tree).
 *
 * Returns 0, or -1 for bad arguments or a graph that is not connected.
 * Floating point: FP64, round-to-nearest, no contraction (built with -ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t u, v;
    int64_t id;
    double weff;
} tedge_t;

static int cmp_weff(const void *pa, const void *pb)
{
    const tedge_t *a = (const tedge_t *)pa, *b = (const tedge_t *)pb;
    if (a->weff > b->weff) return -1;
    if (a->weff < b->weff) return 1;
    return (a->id < b->id) ? -1 : (a->id > b->id); /* ties: smaller edge id first */
}

static int32_t uf_find(int32_t *up, int32_t x)
{
    int32_t r = x;
    while (up[r] != r) r = up[r];
    while (up[x] != r) {
        int32_t nx = up[x];
        up[x] = r;
        x = nx;
    }
    return r;
}

int orc_spanning_tree(int32_t n, const int32_t *row_ptr, const int32_t *col, const double *w, int plain,
                      int32_t *parent, int32_t *root_out, double *weff_out, int32_t *dist_out)
{
    if (n < 1 || !row_ptr || !parent || !root_out) return -1;
    /* T1 */
    int32_t root = 0;
    for (int32_t x = 1; x < n; x++)
        if (row_ptr[x + 1] - row_ptr[x] > row_ptr[root + 1] - row_ptr[root]) root = x;
    /* T2 */
    int32_t *dist = malloc(sizeof(int32_t) * (size_t)n), *queue = malloc(sizeof(int32_t) * (size_t)n);
    if (!dist || !queue) {
        free(dist);
        free(queue);
        return -1;
    }
    for (int32_t x = 0; x < n; x++) dist[x] = -1;
    int64_t qh = 0, qt = 0;
    dist[root] = 0;
    queue[qt++] = root;
    while (qh < qt) {
        int32_t x = queue[qh++];
        for (int64_t k = row_ptr[x]; k < row_ptr[x + 1]; k++) {
            int32_t y = col[k];
            if (y < 0 || y >= n) {
                free(dist);
                free(queue);
                return -1;
            }
            if (dist[y] < 0) {
                dist[y] = dist[x] + 1;
                queue[qt++] = y;
            }
        }
    }
    if (qt != n) { /* not connected */
        free(dist);
        free(queue);
        return -1;
    }
    /* T3: edges in id order */
    int64_t m = 0;
    for (int32_t x = 0; x < n; x++)
        for (int64_t k = row_ptr[x]; k < row_ptr[x + 1]; k++)
            if (col[k] > x) m++;
    tedge_t *e = malloc(sizeof(tedge_t) * (size_t)(m + 1));
    int32_t *up = malloc(sizeof(int32_t) * (size_t)n);
    if (!e || !up) {
        free(dist);
        free(queue);
        free(e);
        free(up);
        return -1;
    }
    int64_t id = 0;
    for (int32_t x = 0; x < n; x++)
        for (int64_t k = row_ptr[x]; k < row_ptr[x + 1]; k++) {
            int32_t y = col[k];
            if (y <= x) continue;
            int32_t dx = row_ptr[x + 1] - row_ptr[x], dy = row_ptr[y + 1] - row_ptr[y];
            double lg = log((double)(dx > dy ? dx : dy));
            double num = w[k] * lg;
            e[id].u = x;
            e[id].v = y;
            e[id].id = id;
            e[id].weff = plain ? w[k] : num / (double)(dist[x] + dist[y]);
            if (weff_out) weff_out[id] = e[id].weff;
            id++;
        }
    /* T4 */
    qsort(e, (size_t)m, sizeof(tedge_t), cmp_weff);
    for (int32_t x = 0; x < n; x++) up[x] = x;
    /* tree adjacency, built as the edges are taken: head[x] -> list of (next, nbr) */
    int32_t *head = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *nxt = malloc(sizeof(int32_t) * 2 * (size_t)(n > 1 ? n - 1 : 1));
    int32_t *nbr = malloc(sizeof(int32_t) * 2 * (size_t)(n > 1 ? n - 1 : 1));
    if (!head || !nxt || !nbr) {
        free(dist);
        free(queue);
        free(e);
        free(up);
        free(head);
        free(nxt);
        free(nbr);
        return -1;
    }
    for (int32_t x = 0; x < n; x++) head[x] = -1;
    int32_t taken = 0;
    for (int64_t i = 0; i < m && taken < n - 1; i++) {
        int32_t a = uf_find(up, e[i].u), b = uf_find(up, e[i].v);
        if (a == b) continue;
        up[a] = b;
        nbr[2 * taken] = e[i].v;
        nxt[2 * taken] = head[e[i].u];
        head[e[i].u] = 2 * taken;
        nbr[2 * taken + 1] = e[i].u;
        nxt[2 * taken + 1] = head[e[i].v];
        head[e[i].v] = 2 * taken + 1;
        taken++;
    }
    /* T5 */
    for (int32_t x = 0; x < n; x++) parent[x] = -2;
    parent[root] = -1;
    qh = qt = 0;
    queue[qt++] = root;
    while (qh < qt) {
        int32_t x = queue[qh++];
        for (int32_t h = head[x]; h >= 0; h = nxt[h]) {
            int32_t y = nbr[h];
            if (parent[y] == -2) {
                parent[y] = x;
                queue[qt++] = y;
            }
        }
    }
    if (dist_out) memcpy(dist_out, dist, sizeof(int32_t) * (size_t)n);
    *root_out = root;
    free(dist);
    free(queue);
    free(e);
    free(up);
    free(head);
    free(nxt);
    free(nbr);
    return 0;
}
