/*
 * Brute-force embedding enumerator — test infrastructure only (a pin for the oracle).
 *
 * Enumerates, one by one, the injective homomorphisms phi : T -> G of a tree template (the
 * labelled non-induced embeddings of Section 2, "Subgraph-counting problem"), optionally keeping
 * only the colourful ones (every template vertex gets a different colour, Section 2.1). It shares
 * nothing with the dynamic program in oracle.c: it walks the template in BFS order from the chosen
 * root and extends a partial map one vertex at a time.
 *
 *   per_vertex[v] = number of maps with phi(root) = v   (optional)
 *   *total        = sum over v
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define BR_MAXK 16

typedef struct {
    int k;
    int order[BR_MAXK];   /* BFS order from the root */
    int parent[BR_MAXK];  /* parent of order[i] in the rooted template (-1 for the root) */
    const int64_t* row_ptr;
    const int32_t* col;
    const uint8_t* colours;
} bctx;

static uint64_t extend(const bctx* c, int depth, int32_t* img, uint32_t used_colours) {
    if (depth == c->k) return 1;
    const int x = c->order[depth];
    const int32_t pv = img[c->parent[x]];
    uint64_t total = 0;
    for (int64_t e = c->row_ptr[pv]; e < c->row_ptr[pv + 1]; ++e) {
        const int32_t w = c->col[e];
        int clash = 0;
        for (int i = 0; i < depth; ++i)
            if (img[c->order[i]] == w) { clash = 1; break; }
        if (clash) continue;
        uint32_t cw = 0;
        if (c->colours) {
            cw = 1u << c->colours[w];
            if (used_colours & cw) continue;
        }
        img[x] = w;
        total += extend(c, depth + 1, img, used_colours | cw);
    }
    return total;
}

int orc_brute_count(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint8_t* colours,
                    int k, const int32_t* tedges, int root, uint64_t* per_vertex, uint64_t* total,
                    int threads) {
    if (k < 1 || k > BR_MAXK || root < 0 || root >= k) return -1;
    int adj[BR_MAXK][BR_MAXK], deg[BR_MAXK];
    memset(deg, 0, sizeof(deg));
    for (int i = 0; i < k - 1; ++i) {
        int u = tedges[2 * i], v = tedges[2 * i + 1];
        if (u < 0 || v < 0 || u >= k || v >= k || u == v) return -1;
        adj[u][deg[u]++] = v;
        adj[v][deg[v]++] = u;
    }
    bctx c;
    c.k = k;
    c.row_ptr = row_ptr;
    c.col = col;
    c.colours = colours;
    int seen[BR_MAXK] = {0}, head = 0, tail = 0;
    c.order[tail++] = root;
    seen[root] = 1;
    c.parent[root] = -1;
    while (head < tail) {
        int x = c.order[head++];
        for (int j = 0; j < deg[x]; ++j) {
            int y = adj[x][j];
            if (!seen[y]) { seen[y] = 1; c.parent[y] = x; c.order[tail++] = y; }
        }
    }
    if (tail != k) return -1;
    if (threads > 0) omp_set_num_threads(threads);
    uint64_t sum = 0;
#pragma omp parallel for schedule(dynamic, 8) reduction(+ : sum)
    for (int64_t v = 0; v < n; ++v) {
        int32_t img[BR_MAXK];
        img[root] = (int32_t)v;
        uint32_t cu = colours ? (1u << colours[v]) : 0u;
        uint64_t cnt = extend(&c, 1, img, cu);
        if (per_vertex) per_vertex[v] = cnt;
        sum += cnt;
    }
    *total = sum;
    return 0;
}

/* number of automorphisms of T by enumerating injective homomorphisms T -> T (small k only) */
int orc_brute_aut(int k, const int32_t* tedges, uint64_t* aut) {
    int64_t row_ptr[BR_MAXK + 1];
    int32_t col[2 * BR_MAXK];
    int64_t e = 0;
    for (int v = 0; v < k; ++v) {
        row_ptr[v] = e;
        for (int u = 0; u < k; ++u)
            for (int i = 0; i < k - 1; ++i)
                if ((tedges[2 * i] == v && tedges[2 * i + 1] == u) ||
                    (tedges[2 * i] == u && tedges[2 * i + 1] == v))
                    col[e++] = u;
    }
    row_ptr[k] = e;
    return orc_brute_count(k, row_ptr, col, NULL, k, tedges, 0, NULL, aut, 1);
}
