/*
 * Colour-coding ORACLE — test infrastructure only.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load this library. The
 * product path (the HIP library under paper_1804_09764_amd/) never links, loads or calls it, and
 * the two share no code, headers or tables.
 *
 * What it computes (paper, Section 2.1 "The Color-coding Technique", Eq. 1 and Algorithm 1):
 *
 *   For a tree template T on k vertices, a graph G and a colouring col : V -> {0..k-1}, the
 *   dynamic program computes C(v, T_i, S): the number of colourful embeddings of the rooted
 *   sub-template T_i with its root mapped to v that use exactly the colour set S (|S| = |T_i|).
 *   Cutting the edge (root(T_i), u) splits T_i into the active part T_i' (keeps the root) and the
 *   passive part T_i'' (rooted at u), and
 *
 *       C(v, T_i, S) = sum_{u in N(v)} sum_{S = S1 (disjoint) S2, |S1| = |T_i'|} C(v, T_i', S1) * C(u, T_i'', S2)
 *
 *   down to single vertices, where C(v, T_1, {c}) = [col(v) = c] (Section 2.1, the recursive
 *   partition of the template in Figure 1(a)). The total over v at the full template is the number
 *   of colourful embeddings for one colouring (Algorithm 1, Eq. 3 before its k^k/k! scaling).
 *
 * Readings taken here, where the paper leaves a choice open:
 *   - The over-counting divisor d of Eq. 1 is not applied: the program counts labelled maps
 *     (injective homomorphisms phi : T -> G with col o phi injective), an exact integer. The
 *     estimate divides by |Aut(T)| once at the end.
 *   - Colours are 0..k-1 (the paper writes 1..k); exactly k colours.
 *   - The random colouring, where it is drawn here rather than passed in, is the counter-based
 *     hash described at orc_colour.
 *
 * Arithmetic: tables hold IEEE double (the counts are integers, exact below 2^53); every entry's
 * sum of products is accumulated in x87 long double with Neumaier compensation, so that each entry
 * is the exact sum rounded once to double. Below 2^53 every entry is exact.
 *
 * Colour sets are bitmasks over k colours; a set's index is its position among the sets of the
 * same size listed in increasing numeric order of the mask (colex order).
 *
 * Loop order follows Eq. 1 literally: for each centre vertex v and set S, the sum runs over the
 * neighbours u and, inside, over the splits of S. Nothing is pre-summed or fused.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define ORC_MAXK 16

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -3 };

static int64_t binom_i(int n, int r) {
    if (r < 0 || r > n) return 0;
    int64_t b = 1;
    for (int i = 1; i <= r; ++i) b = b * (n - r + i) / i;
    return b;
}

static int popcount32(uint32_t x) {
    int c = 0;
    while (x) { x &= x - 1; ++c; }
    return c;
}

/* position of every mask among the masks of the same popcount, in increasing numeric order */
static int32_t* make_rank(int k) {
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) << k);
    int32_t next[ORC_MAXK + 1];
    if (!rank) return NULL;
    memset(next, 0, sizeof(next));
    for (uint32_t m = 0; m < (1u << k); ++m) rank[m] = next[popcount32(m)]++;
    return rank;
}

static inline void neumaier_add(long double* sum, long double* comp, long double t) {
    long double y = *sum + t;
    long double as = *sum < 0 ? -*sum : *sum;
    long double at = t < 0 ? -t : t;
    if (as >= at) *comp += (*sum - y) + t;
    else          *comp += (t - y) + *sum;
    *sum = y;
}

/* ---------------------------------------------------------------------------------------------
 * Random colouring (Algorithm 1, "pick a colour uniformly at random").
 * Counter-based: h = mix64(mix64(seed + G*(iter+1)) + H*(v+1)), colour = floor(k * h / 2^64),
 * where mix64 is the SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014) and
 * G = 0x9E3779B97F4A7C15, H = 0xD1B54A32D192ED03. The range reduction is Lemire's
 * multiply-shift (ACM TOMACS 2019).
 * ------------------------------------------------------------------------------------------- */
static uint64_t orc_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

int orc_colour(uint64_t seed, uint64_t iter, int64_t n, int k, uint8_t* out) {
    if (k < 1 || k > ORC_MAXK || n < 0) return ORC_EINVAL;
    const uint64_t G = 0x9E3779B97F4A7C15ULL, H = 0xD1B54A32D192ED03ULL;
    uint64_t base = orc_mix64(seed + G * (iter + 1));
    for (int64_t v = 0; v < n; ++v) {
        uint64_t h = orc_mix64(base + H * (uint64_t)(v + 1));
        out[v] = (uint8_t)(((unsigned __int128)h * (unsigned)k) >> 64);
    }
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------------
 * One application of Eq. 1 at a split of sizes (s, a, p = s - a), for nv centre vertices.
 *   act : nv x C(k,a)   row i = C(v_i, T', .)
 *   pas : rows x C(k,p) row u = C(u, T'', .)
 *   nbr_ptr/nbr : the neighbours of centre i are the pas rows nbr[nbr_ptr[i] .. nbr_ptr[i+1])
 *   out : nv x C(k,s)
 * ------------------------------------------------------------------------------------------- */
int orc_step(int k, int s, int a, int64_t nv, const int64_t* nbr_ptr, const int32_t* nbr,
             const double* act, const double* pas, double* out, int threads) {
    const int p = s - a;
    if (k < 1 || k > ORC_MAXK || a < 1 || p < 1 || s > k || nv < 0) return ORC_EINVAL;
    const int64_t ws = binom_i(k, s), wa = binom_i(k, a), wp = binom_i(k, p);
    const int64_t np = binom_i(s, a);
    int32_t* rank = make_rank(k);
    uint32_t* smask = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)ws);
    int32_t* pair_a = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ws * np));
    int32_t* pair_p = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ws * np));
    if (!rank || !smask || !pair_a || !pair_p) {
        free(rank); free(smask); free(pair_a); free(pair_p);
        return ORC_ENOMEM;
    }
    int64_t cnt = 0;
    for (uint32_t m = 0; m < (1u << k); ++m)
        if (popcount32(m) == s) smask[cnt++] = m;
    /* every split S = S1 + S2 with |S1| = a, listed by walking the sub-masks of S */
    for (int64_t r = 0; r < ws; ++r) {
        const uint32_t S = smask[r];
        int64_t j = 0;
        for (uint32_t sub = S;; sub = (sub - 1) & S) {
            if (popcount32(sub) == a) {
                pair_a[r * np + j] = rank[sub];
                pair_p[r * np + j] = rank[S & ~sub];
                ++j;
            }
            if (sub == 0) break;
        }
    }
    if (threads > 0) omp_set_num_threads(threads);
    /* every (centre, colour set) entry is one independent task: a single high-degree centre is
       spread over the threads, and each entry's sum is accumulated in the same order as ever */
#pragma omp parallel for collapse(2) schedule(dynamic, 16)
    for (int64_t i = 0; i < nv; ++i) {
        for (int64_t r = 0; r < ws; ++r) {
            const double* arow = act + i * wa;
            long double sum = 0.0L, comp = 0.0L;
            for (int64_t e = nbr_ptr[i]; e < nbr_ptr[i + 1]; ++e) {
                const double* prow = pas + (int64_t)nbr[e] * wp;
                for (int64_t j = 0; j < np; ++j) {
                    long double t = (long double)arow[pair_a[r * np + j]] *
                                    (long double)prow[pair_p[r * np + j]];
                    neumaier_add(&sum, &comp, t);
                }
            }
            out[i * ws + r] = (double)(sum + comp);
        }
    }
    free(rank); free(smask); free(pair_a); free(pair_p);
    return ORC_OK;
}

/* ---------------------------------------------------------------------------------------------
 * Template handling: validation, rooting, the oracle's own partition rule.
 * ------------------------------------------------------------------------------------------- */
typedef struct {
    int k;
    int deg[ORC_MAXK];
    int adj[ORC_MAXK][ORC_MAXK];
    int parent[ORC_MAXK];
    uint32_t kids[ORC_MAXK];  /* children bitmask in the rooted tree */
    int size[ORC_MAXK];       /* subtree size */
    int rule;
} otree;

static int tree_load(otree* t, int k, const int32_t* edges) {
    if (k < 1 || k > ORC_MAXK) return ORC_EINVAL;
    memset(t, 0, sizeof(*t));
    t->k = k;
    for (int i = 0; i < k - 1; ++i) {
        int u = edges[2 * i], v = edges[2 * i + 1];
        if (u < 0 || v < 0 || u >= k || v >= k || u == v) return ORC_EINVAL;
        for (int j = 0; j < t->deg[u]; ++j)
            if (t->adj[u][j] == v) return ORC_EINVAL;
        t->adj[u][t->deg[u]++] = v;
        t->adj[v][t->deg[v]++] = u;
    }
    /* connected? */
    int seen[ORC_MAXK] = {0}, stack[ORC_MAXK], sp = 0, cnt = 0;
    stack[sp++] = 0; seen[0] = 1;
    while (sp) {
        int x = stack[--sp]; ++cnt;
        for (int j = 0; j < t->deg[x]; ++j)
            if (!seen[t->adj[x][j]]) { seen[t->adj[x][j]] = 1; stack[sp++] = t->adj[x][j]; }
    }
    return cnt == k ? ORC_OK : ORC_EINVAL;
}

static int tree_root(otree* t, int x, int p) {
    t->parent[x] = p;
    t->kids[x] = 0;
    t->size[x] = 1;
    for (int j = 0; j < t->deg[x]; ++j) {
        int y = t->adj[x][j];
        if (y == p) continue;
        t->kids[x] |= 1u << y;
        t->size[x] += tree_root(t, y, x);
    }
    return t->size[x];
}

/* rule 0: cut the child with the largest subtree (ties: larger label);
 * rule 1: cut the child with the smallest subtree (ties: smaller label). */
static int pick_child(const otree* t, uint32_t kids) {
    int best = -1;
    for (int c = 0; c < t->k; ++c) {
        if (!(kids >> c & 1u)) continue;
        if (best < 0) { best = c; continue; }
        if (t->rule == 0) {
            if (t->size[c] > t->size[best] || (t->size[c] == t->size[best] && c > best)) best = c;
        } else {
            if (t->size[c] < t->size[best] || (t->size[c] == t->size[best] && c < best)) best = c;
        }
    }
    return best;
}

typedef struct {
    int64_t n;
    const int64_t* row_ptr;
    const int32_t* col;
    const uint8_t* colours;
    int threads;
    int err;
} ograph;

/* table of the sub-template made of root r and the subtrees of the children in `kids` */
static double* solve(const otree* t, const ograph* g, int r, uint32_t kids, int* size_out) {
    const int k = t->k;
    if (kids == 0) {
        double* leaf = (double*)calloc((size_t)g->n * k, sizeof(double));
        if (!leaf) return NULL;
        for (int64_t v = 0; v < g->n; ++v) leaf[v * k + g->colours[v]] = 1.0;  /* rank({c}) = c */
        *size_out = 1;
        return leaf;
    }
    int c = pick_child(t, kids);
    int a_sz = 0, p_sz = 0;
    double* A = solve(t, g, r, kids & ~(1u << c), &a_sz);
    if (!A) return NULL;
    double* P = solve(t, g, c, t->kids[c], &p_sz);
    if (!P) { free(A); return NULL; }
    int s = a_sz + p_sz;
    double* out = (double*)malloc(sizeof(double) * (size_t)g->n * (size_t)binom_i(k, s));
    if (!out) { free(A); free(P); return NULL; }
    int rc = orc_step(k, s, a_sz, g->n, g->row_ptr, g->col, A, P, out, g->threads);
    free(A);
    free(P);
    if (rc != ORC_OK) { free(out); return NULL; }
    *size_out = s;
    return out;
}

/*
 * Colourful labelled embeddings for one colouring.
 *   per_vertex[v] (optional) = C(v, T rooted at `root`, [k])
 *   *X = sum over v, accumulated in long double with compensation
 * root < 0 selects the rule's default (rule 0: largest label, rule 1: smallest label).
 */
int orc_count(int64_t n, const int64_t* row_ptr, const int32_t* col, const uint8_t* colours, int k,
              const int32_t* tedges, int root, int rule, double* per_vertex, long double* X,
              int threads) {
    otree t;
    if (rule != 0 && rule != 1) return ORC_EINVAL;
    int rc = tree_load(&t, k, tedges);
    if (rc != ORC_OK) return rc;
    for (int64_t v = 0; v < n; ++v)
        if (colours[v] >= k) return ORC_EINVAL;
    t.rule = rule;
    if (root < 0) root = (rule == 0) ? k - 1 : 0;
    if (root >= k) return ORC_EINVAL;
    tree_root(&t, root, -1);
    ograph g = {n, row_ptr, col, colours, threads, 0};
    int sz = 0;
    double* top = solve(&t, &g, root, t.kids[root], &sz);
    if (!top) return ORC_ENOMEM;
    long double sum = 0.0L, comp = 0.0L;
    for (int64_t v = 0; v < n; ++v) {
        if (per_vertex) per_vertex[v] = top[v];
        neumaier_add(&sum, &comp, (long double)top[v]);
    }
    *X = sum + comp;
    free(top);
    return ORC_OK;
}

/*
 * |Aut(T)| as the number of colourful injective homomorphisms of T into itself under the identity
 * colouring: an injective map from T's vertices to T's vertices that keeps all k-1 edges is a
 * bijection onto the edge set, i.e. an automorphism, and the identity colouring makes every
 * injective map colourful.
 */
int orc_aut(int k, const int32_t* tedges, long double* aut) {
    otree t;
    int rc = tree_load(&t, k, tedges);
    if (rc != ORC_OK) return rc;
    /* CSR of T itself */
    int64_t row_ptr[ORC_MAXK + 1];
    int32_t col[2 * ORC_MAXK];
    uint8_t colours[ORC_MAXK];
    int64_t e = 0;
    for (int v = 0; v < k; ++v) {
        row_ptr[v] = e;
        /* sorted neighbour list */
        for (int u = 0; u < k; ++u)
            for (int j = 0; j < t.deg[v]; ++j)
                if (t.adj[v][j] == u) col[e++] = u;
        colours[v] = (uint8_t)v;
    }
    row_ptr[k] = e;
    return orc_count(k, row_ptr, col, colours, k, tedges, -1, 0, NULL, aut, 1);
}

/* Table-3-style bookkeeping is a planner concern of the GPU library, not the oracle's. */

/* mean_b(X_b) * k^k / k! / |Aut(T)|, evaluated in long double (Algorithm 1, Eq. 3 and the
 * colourful probability k!/k^k of Section 2.1). */
int orc_estimate(int k, long double aut, const long double* X, int64_t B, long double* est) {
    if (k < 1 || B < 1 || aut <= 0) return ORC_EINVAL;
    long double m = 0.0L, c = 0.0L;
    for (int64_t b = 0; b < B; ++b) neumaier_add(&m, &c, X[b]);
    m = (m + c) / (long double)B;
    long double scale = 1.0L;
    for (int i = 1; i <= k; ++i) scale *= (long double)k / (long double)i;
    *est = m * scale / aut;
    return ORC_OK;
}

int orc_threads(void) { return omp_get_max_threads(); }
