/*
 * Seeded synthetic graph generator (input side only).
 *
 * Builds the R-MAT graphs the benchmarks and tests run on: ef * 2^scale edge draws, each edge
 * choosing one quadrant per bit level with probabilities (a, b, c, 1-a-b-c), a seeded bijective
 * relabelling of the vertex ids (so that hubs are not clustered at low ids), self-loop removal,
 * symmetrisation and de-duplication, and sorted CSR rows (int64 row offsets, int32 columns).
 * Isolated vertices are kept, so n = 2^scale.
 *
 * This file holds no colour-coding arithmetic. It is shared, as an input generator, by the oracle
 * tests and by the GPU tests and benchmark; inputs/__init__.py has a numpy twin of the same edge
 * draw (used to cross-check this file at small scales).
 *
 * Random numbers: counter-based. mix64 is the finaliser of SplitMix64 (Steele, Lea and Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014). The draw for bit level l of
 * edge e is the upper 32 bits of mix64(mix64(seed + G*(e+1)) + H*(l+1)).
 *
 * Two-phase C API so that the caller (numpy) owns the output arrays:
 *   gen_rmat_build(...)  -> opaque handle, reports n and nnz
 *   gen_rmat_fill(h, row_ptr, col)  copies the CSR out
 *   gen_free(h)
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <omp.h>

#define GEN_G 0x9E3779B97F4A7C15ULL
#define GEN_H 0xD1B54A32D192ED03ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

typedef struct {
    int scale;
    uint64_t mask, p1, q1, p2, q2;
    int shift;
    uint32_t ta, tb, tc;
    uint64_t seed;
} rmat_params;

static inline uint64_t perm(const rmat_params* P, uint64_t x) {
    x = (x * P->p1 + P->q1) & P->mask;
    x ^= x >> P->shift;
    x = (x * P->p2 + P->q2) & P->mask;
    x ^= x >> P->shift;
    return x;
}

/* one edge draw; returns 0 for a self-loop */
static inline int draw(const rmat_params* P, uint64_t e, uint32_t* src, uint32_t* dst) {
    uint64_t base = mix64(P->seed + GEN_G * (e + 1));
    uint64_t s = 0, d = 0;
    for (int l = 0; l < P->scale; ++l) {
        uint32_t r = (uint32_t)(mix64(base + GEN_H * (uint64_t)(l + 1)) >> 32);
        uint64_t bs, bd;
        if (r < P->ta)      { bs = 0; bd = 0; }
        else if (r < P->tb) { bs = 0; bd = 1; }
        else if (r < P->tc) { bs = 1; bd = 0; }
        else                { bs = 1; bd = 1; }
        s = (s << 1) | bs;
        d = (d << 1) | bd;
    }
    s = perm(P, s);
    d = perm(P, d);
    *src = (uint32_t)s;
    *dst = (uint32_t)d;
    return s != d;
}

typedef struct {
    int64_t n, nnz;
    int64_t* raw_off;   /* n+1 offsets into raw */
    int32_t* raw;       /* per-row sorted, unique prefix of length uniq[v] */
    int64_t* uniq;
} gen_handle;

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

void gen_rmat_params(int scale, double a, double b, double c, uint64_t seed, uint64_t out[8]) {
    /* exposes the derived constants so the numpy twin can be checked against them */
    out[0] = (uint64_t)floor(a * 4294967296.0);
    out[1] = (uint64_t)floor((a + b) * 4294967296.0);
    out[2] = (uint64_t)floor((a + b + c) * 4294967296.0);
    out[3] = mix64(seed + 1) | 1ULL;
    out[4] = mix64(seed + 2);
    out[5] = mix64(seed + 3) | 1ULL;
    out[6] = mix64(seed + 4);
    out[7] = (uint64_t)((scale + 1) / 2);
}

void* gen_rmat_build(int scale, int64_t edge_factor, double a, double b, double c, uint64_t seed,
                     int threads, int64_t* n_out, int64_t* nnz_out) {
    if (scale < 1 || scale > 30 || edge_factor < 1) return NULL;
    if (threads <= 0) threads = omp_get_max_threads();
    rmat_params P;
    uint64_t k8[8];
    gen_rmat_params(scale, a, b, c, seed, k8);
    P.scale = scale;
    P.mask = (1ULL << scale) - 1;
    P.ta = (uint32_t)k8[0]; P.tb = (uint32_t)k8[1]; P.tc = (uint32_t)k8[2];
    P.p1 = k8[3]; P.q1 = k8[4]; P.p2 = k8[5]; P.q2 = k8[6];
    P.shift = (int)k8[7];
    P.seed = seed;

    const int64_t n = (int64_t)1 << scale;
    const uint64_t E = (uint64_t)edge_factor << scale;
    const int T = threads;

    gen_handle* h = (gen_handle*)calloc(1, sizeof(gen_handle));
    int64_t* cnt = (int64_t*)calloc((size_t)T * (size_t)n, sizeof(int64_t));  /* per-thread degrees */
    int64_t* off = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!h || !cnt || !off) { free(h); free(cnt); free(off); return NULL; }
    h->n = n;

    /* pass 1: each thread counts the endpoints of its own contiguous range of edge draws */
#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num();
        const uint64_t lo = E * (uint64_t)t / (uint64_t)T, hi = E * (uint64_t)(t + 1) / (uint64_t)T;
        int64_t* my = cnt + (size_t)t * (size_t)n;
        for (uint64_t e = lo; e < hi; ++e) {
            uint32_t s, d;
            if (draw(&P, e, &s, &d)) { my[s]++; my[d]++; }
        }
    }
    /* row offsets, and per-thread write cursors (thread t writes after threads < t) */
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) {
        int64_t acc = off[v];
        for (int t = 0; t < T; ++t) {
            int64_t x = cnt[(size_t)t * (size_t)n + (size_t)v];
            cnt[(size_t)t * (size_t)n + (size_t)v] = acc;
            acc += x;
        }
        off[v + 1] = acc;
    }
    const int64_t raw_n = off[n];
    int32_t* raw = (int32_t*)malloc((size_t)(raw_n > 0 ? raw_n : 1) * sizeof(int32_t));
    if (!raw) { free(off); free(cnt); free(h); return NULL; }

    /* pass 2: the same draws, scattered through the thread's own cursors (no atomics) */
#pragma omp parallel num_threads(T)
    {
        const int t = omp_get_thread_num();
        const uint64_t lo = E * (uint64_t)t / (uint64_t)T, hi = E * (uint64_t)(t + 1) / (uint64_t)T;
        int64_t* cur = cnt + (size_t)t * (size_t)n;
        for (uint64_t e = lo; e < hi; ++e) {
            uint32_t s, d;
            if (draw(&P, e, &s, &d)) {
                raw[cur[s]++] = (int32_t)d;
                raw[cur[d]++] = (int32_t)s;
            }
        }
    }
    free(cnt);
    int64_t* uniq = (int64_t*)malloc(((size_t)n + 1) * sizeof(int64_t));
    if (!uniq) { free(raw); free(off); free(h); return NULL; }
    /* sort + unique per row */
#pragma omp parallel for schedule(dynamic, 256) num_threads(T)
    for (int64_t v = 0; v < n; ++v) {
        int32_t* r = raw + off[v];
        int64_t len = off[v + 1] - off[v];
        if (len > 1) qsort(r, (size_t)len, sizeof(int32_t), cmp_i32);
        int64_t u = 0;
        for (int64_t i = 0; i < len; ++i)
            if (i == 0 || r[i] != r[i - 1]) r[u++] = r[i];
        uniq[v] = u;
    }
    int64_t nnz = 0;
    for (int64_t v = 0; v < n; ++v) nnz += uniq[v];
    h->raw_off = off;
    h->raw = raw;
    h->uniq = uniq;
    h->nnz = nnz;
    *n_out = n;
    *nnz_out = nnz;
    return h;
}

int gen_rmat_fill(void* hv, int64_t* row_ptr, int32_t* col, int threads) {
    gen_handle* h = (gen_handle*)hv;
    if (!h) return -1;
    if (threads <= 0) threads = omp_get_max_threads();
    const int64_t n = h->n;
    row_ptr[0] = 0;
    for (int64_t v = 0; v < n; ++v) row_ptr[v + 1] = row_ptr[v] + h->uniq[v];
#pragma omp parallel for schedule(dynamic, 1024) num_threads(threads)
    for (int64_t v = 0; v < n; ++v)
        memcpy(col + row_ptr[v], h->raw + h->raw_off[v], (size_t)h->uniq[v] * sizeof(int32_t));
    return 0;
}

void gen_free(void* hv) {
    gen_handle* h = (gen_handle*)hv;
    if (!h) return;
    free(h->raw_off);
    free(h->raw);
    free(h->uniq);
    free(h);
}

/* raw edge draws (before relabel filtering) for cross-checking the numpy twin at small sizes */
int gen_rmat_draws(int scale, double a, double b, double c, uint64_t seed, uint64_t e0, uint64_t count,
                   uint32_t* src, uint32_t* dst, uint8_t* keep) {
    rmat_params P;
    uint64_t k8[8];
    gen_rmat_params(scale, a, b, c, seed, k8);
    P.scale = scale;
    P.mask = (1ULL << scale) - 1;
    P.ta = (uint32_t)k8[0]; P.tb = (uint32_t)k8[1]; P.tc = (uint32_t)k8[2];
    P.p1 = k8[3]; P.q1 = k8[4]; P.p2 = k8[5]; P.q2 = k8[6];
    P.shift = (int)k8[7];
    P.seed = seed;
    for (uint64_t i = 0; i < count; ++i) keep[i] = (uint8_t)draw(&P, e0 + i, &src[i], &dst[i]);
    return 0;
}
