// Host side of the C ABI declared in include/cc.h: plans, graphs, colouring, plain and packed counts,
// estimates and measurement; argument checking, workspace layouts, work lists and launch sequences.
// Multi-template counts are in cc_multi.cpp, instance batches in cc_batch.cpp.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "cc_host.h"
#include "cc_internal.h"

namespace cc {
namespace host {

thread_local std::string g_err;

cc_status fail(cc_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

cc_status hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return CC_EDEVICE;
}

void resolve_tuning(int64_t nnz, const cc_tuning* t, int32_t* thr, int32_t* chunk, int32_t* cols = nullptr) {
    int32_t c = (t && t->chunk > 0) ? t->chunk : (nnz >= ((int64_t)1 << 28) ? 2048 : 512);
    c = (c + 63) / 64 * 64;
    int32_t h = (t && t->hub_threshold > 0) ? t->hub_threshold : 2 * c;
    if (h < c) h = c;
    *thr = h;
    *chunk = c;
    if (cols) *cols = t ? t->cols_per_lane : 0;
}

struct GraphLayout {
    size_t flags_off, light_off, range_off, chunk_off, hub_off, total;
};

constexpr int kRangeRows = 64;  // at most this many light rows per range task

GraphLayout graph_layout(int64_t n, int64_t nnz, int32_t thr, int32_t chunk) {
    GraphLayout L;
    const int64_t max_hubs = nnz / ((int64_t)thr + 1) + 1;
    const int64_t max_chunks = nnz / chunk + max_hubs;
    L.flags_off = 0;
    L.light_off = 256;
    L.range_off = align256(L.light_off + (size_t)n * sizeof(int32_t));
    L.chunk_off = align256(L.range_off + (size_t)(n + 1) * sizeof(int32_t));
    L.hub_off = align256(L.chunk_off + (size_t)max_chunks * sizeof(cc::ChunkItem));
    L.total = align256(L.hub_off + (size_t)max_hubs * sizeof(cc::HubItem));
    return L;
}

// Colour classes per projected pass of each split (0: the split reads the passive table itself).
// Auto: a split is projected when its projected rows hold at least 30 % fewer 128-byte lines than
// a centre reads from a stored row (measured on R-MAT 23 / edge factor 256: projected rows stream
// about 10 % slower, so the 462-entry rows of 12-vertex templates, 16 lines instead of 21.7, gain
// 16 %, while the 330-entry rows, 14 instead of 17.5, lose 3 %) and the lines it saves on the
// neighbour reads exceed twice the bytes of making the copies (each pass reads the table once;
// every vertex writes one row per other colour); a pass takes as many classes as fit in the table
// arena's size.
std::vector<int> projection_plan(const cc_plan* P, const cc_graph* G, int64_t n_pad) {
    std::vector<int> g(P->splits.size(), 0);
    const int k = P->k;
    const int mode = G->proj_classes;
    if (mode < 0 || G->n == 0) return g;
    const double arena_bytes = (double)P->arena_cols * (double)n_pad * sizeof(double);
    for (size_t i = 0; i < P->splits.size(); ++i) {
        const cc::Split& sp = P->splits[i];
        if (sp.Wn <= 0) continue;
        const double per_class = (double)n_pad * sp.Wn_pad * sizeof(double);
        int cls;
        if (mode > 0) {
            cls = std::min(mode, k);
        } else {
            cls = (int)std::max(1.0, std::min((double)k, std::floor(arena_bytes / per_class)));
            const int passes = (k + cls - 1) / cls;
            if (sp.lines_need < 1.2 * (sp.Wn_pad / 16.0)) continue;
            const double saved = (double)G->nnz * (k - 1) / k * 128.0 * (sp.lines_need - sp.Wn_pad / 16.0);
            const double cost = (double)G->n * sizeof(double) *
                                ((double)passes * cc::pad_stride(sp.Wp) + (double)(k - 1) * sp.Wn_pad);
            if (!(saved > 2.0 * cost)) continue;
        }
        const int passes = (k + cls - 1) / cls;
        g[i] = (k + passes - 1) / passes;  // the same number of classes in every pass, give or take one
    }
    return g;
}

struct CountLayout {
    size_t arena_off, partial_off, root_off, red_off, ecol_off, proj_off, total;
    int64_t n_pad;
    std::vector<int> proj;  // classes per projected pass of each split (0: none)
};

// arena_cols: the table arena's width in columns of n_pad doubles (-1: the plan's own);
// proj_cap: at most this many colour classes per projected pass (0: no projection; -1: no cap)
CountLayout count_layout(const cc_plan* P, const cc_graph* G, int64_t arena_cols = -1, int proj_cap = -1) {
    CountLayout L;
    L.n_pad = pad32(G->n);
    L.arena_off = 0;
    if (arena_cols < 0) arena_cols = P->arena_cols;
    L.partial_off = align256((size_t)arena_cols * (size_t)L.n_pad * sizeof(double));
    L.root_off = align256(L.partial_off + (size_t)G->n_chunks * (size_t)P->max_stride_N * sizeof(double));
    L.red_off = align256(L.root_off + (size_t)std::max<int64_t>(G->n, 1) * sizeof(double));
    L.ecol_off = align256(L.red_off + 1024 * sizeof(double));
    L.proj_off = align256(L.ecol_off + (size_t)std::max<int64_t>(G->nnz, 1));
    L.proj = projection_plan(P, G, L.n_pad);
    if (proj_cap >= 0)
        for (int& c : L.proj) c = std::min(c, proj_cap);
    size_t proj_bytes = 0;
    for (size_t i = 0; i < P->splits.size(); ++i)
        proj_bytes = std::max(proj_bytes, (size_t)L.proj[i] * (size_t)L.n_pad * (size_t)P->splits[i].Wn_pad * sizeof(double));
    L.total = align256(L.proj_off + proj_bytes);
    return L;
}

// workspace of a packed count with B colourings per row
PackedLayout packed_layout(const cc_plan* P, const cc_graph* G, int32_t B) {
    PackedLayout L;
    L.n_pad = pad32(G->n);
    const int64_t cols = cc::packed_arena(P, B, &L.col_off);
    L.stride.resize(P->tables.size());
    L.bstep.resize(P->tables.size());
    for (size_t t = 0; t < P->tables.size(); ++t) {
        const int64_t W = P->tables[t].W;
        L.stride[t] = cc::packed_wide(W) ? cc::packed_stride(W) : cc::packed_stride((int64_t)B * W);
        L.bstep[t] = cc::packed_wide(W) ? L.n_pad * cc::packed_stride(W) : W;
    }
    int64_t nst = 1;
    for (const auto& sp : P->splits) nst = std::max(nst, cc::packed_stride((int64_t)B * sp.Cf));
    L.nstride = nst;
    L.arena_off = 0;
    L.partial_off = align256((size_t)cols * (size_t)L.n_pad * sizeof(double));
    L.root_off = align256(L.partial_off + (size_t)G->n_chunks * (size_t)nst * sizeof(double));
    L.colour_off = align256(L.root_off + (size_t)std::max<int64_t>(G->n, 1) * (size_t)B * sizeof(double));
    L.red_off = align256(L.colour_off + (size_t)std::max<int64_t>(G->n, 1) * (size_t)B);
    L.total = align256(L.red_off + (size_t)cc::packed_reduce_blocks(G->n) * (size_t)B * sizeof(double));
    return L;
}

// arguments of split `sp` of plan P on graph G for one colouring; tables live in `arena`
// everything of a split's arguments except where its tables live
cc::StepParams base_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, const uint8_t* colour,
                           double* partial, double* root_out) {
    cc::StepParams h{};
    h.row_ptr = G->row_ptr;
    h.col = G->col;
    h.colour = colour;
    h.ecol = nullptr;
    h.cstride = 1;
    h.light = G->light;
    h.light_start = G->light_start;
    h.chunks = G->chunks;
    h.hubs = G->hubs;
    h.n_light = G->n_light;
    h.n_ranges = G->n_ranges;
    h.n_chunks = G->n_chunks;
    h.n_hubs = G->n_hubs;
    h.O = root_out;
    h.ostride = 1;
    const uint8_t* cdev = (const uint8_t*)P->dev;
    h.partial = partial;
    h.nstride = P->max_stride_N;
    h.fold = sp.fold_off >= 0 ? (const uint16_t*)(cdev + sp.fold_off) : nullptr;
    h.split = sp.split_off >= 0 ? (const uint32_t*)(cdev + sp.split_off) : nullptr;
    h.mask = sp.mask_off >= 0 ? (const uint16_t*)(cdev + sp.mask_off) : nullptr;
    h.cols_per_lane = G->cols_per_lane;
    h.cls_mask = cc::kAllClasses;
    h.class_stride = 0;
    h.tile_doubles = G->packed_tile;
    h.k = P->k;
    h.s = sp.s;
    h.a = sp.a;
    h.p = sp.p;
    h.Wa = sp.Wa;
    h.Wp = sp.Wp;
    h.Ws = sp.Ws;
    h.Nw = sp.Nw;
    h.npairs = sp.npairs;
    h.a_off = cc::split_a_off(sp.Nw);
    h.stage_a = cc::split_stage_a(sp.Nw, sp.Wa, sp.a) ? 1 : 0;
    h.lds_wave = cc::split_lds_wave(sp.Nw, sp.Wa, sp.a);
    return h;
}

cc::StepParams step_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, const uint8_t* colour,
                           double* arena, int64_t n_pad, double* partial, double* root_out) {
    cc::StepParams h = base_params(P, G, sp, colour, partial, root_out);
    if (sp.pas >= 0) {
        const cc::Table& t = P->tables[sp.pas];
        h.P = arena + t.col_off * n_pad;
        h.pstride = t.stride;
    }
    if (sp.act >= 0) {
        const cc::Table& t = P->tables[sp.act];
        h.A = arena + t.col_off * n_pad;
        h.astride = t.stride;
    }
    if (sp.out >= 0) {
        const cc::Table& t = P->tables[sp.out];
        h.O = arena + t.col_off * n_pad;
        h.ostride = t.stride;
    }
    return h;
}

// the same split over the packed layout (B colourings per row, colours as [v][b])
cc::StepParams packed_step_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, PIds t,
                                  const uint8_t* colour, double* arena, const PackedLayout& L, double* partial,
                                  double* root_out, int32_t B) {
    cc::StepParams h = base_params(P, G, sp, colour, partial, root_out);
    if (t.pas >= 0) {
        h.P = arena + L.col_off[(size_t)t.pas] * L.n_pad;
        h.pstride = L.stride[(size_t)t.pas];
    }
    if (t.act >= 0) {
        h.A = arena + L.col_off[(size_t)t.act] * L.n_pad;
        h.astride = L.stride[(size_t)t.act];
    }
    if (t.out >= 0) {
        h.O = arena + L.col_off[(size_t)t.out] * L.n_pad;
        h.ostride = L.stride[(size_t)t.out];
    } else {
        h.O = root_out;
        h.ostride = B;
    }
    h.nstride = L.nstride;
    const uint8_t* cdev = (const uint8_t*)P->dev;
    h.B = B;
    h.Cf = sp.Cf;
    h.fullmap = sp.full_off >= 0 ? (const uint16_t*)(cdev + sp.full_off) : nullptr;
    h.emap = (const uint16_t*)(cdev + sp.emap_off);
    cc::packed_tile(&h);
    return h;
}

// split `sp` of a packed count for colouring b alone, with the one-colouring kernels: the tables
// are the packed ones offset to colouring b's entry blocks; colours_bn is the caller's [B][n]
// colour array (colouring b's colours are contiguous there, a small, cache-resident array)
cc::StepParams packed_one_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, PIds t,
                                 const uint8_t* colours_bn, double* arena, const PackedLayout& L, double* partial,
                                 double* root_out, int32_t B, int32_t b) {
    cc::StepParams h = base_params(P, G, sp, colours_bn + (int64_t)b * G->n, partial, root_out);
    if (t.pas >= 0) {
        h.P = arena + L.col_off[(size_t)t.pas] * L.n_pad + (int64_t)b * L.bstep[(size_t)t.pas];
        h.pstride = L.stride[(size_t)t.pas];
    }
    if (t.act >= 0) {
        h.A = arena + L.col_off[(size_t)t.act] * L.n_pad + (int64_t)b * L.bstep[(size_t)t.act];
        h.astride = L.stride[(size_t)t.act];
    }
    if (t.out >= 0) {
        h.O = arena + L.col_off[(size_t)t.out] * L.n_pad + (int64_t)b * L.bstep[(size_t)t.out];
        h.ostride = L.stride[(size_t)t.out];
    } else {
        h.O = root_out + b;
        h.ostride = B;
    }
    return h;
}

// every split of the plan that runs the packed kernels fits their LDS (one wavefront's slice and
// the maps)
bool packed_fits(const cc_plan* P, int32_t B) {
    for (const auto& sp : P->splits) {
        if (!cc::packed_kernel_split(sp)) continue;
        cc::StepParams h{};
        h.k = P->k;
        h.a = sp.a;
        h.p = sp.p;
        h.Wa = sp.Wa;
        h.Wp = sp.Wp;
        h.Nw = sp.Nw;
        h.Ws = sp.Ws;
        h.npairs = sp.npairs;
        h.Cf = sp.Cf;
        h.B = B;
        cc::packed_tile(&h);
        if (cc::packed_lds_bytes(h, 1) > 64 * 1024) return false;
    }
    return true;
}

}  // namespace host
}  // namespace cc

using namespace cc::host;

extern "C" {

const char* cc_last_error(void) { return g_err.c_str(); }

cc_status cc_plan_create(int32_t k, const int32_t* edges_host, int32_t root, uint32_t flags, cc_plan** out) {
    if (!out) return fail(CC_EINVAL, "out is NULL");
    *out = nullptr;
    cc_plan* P = new (std::nothrow) cc_plan();
    if (!P) return fail(CC_ENOMEM, "plan allocation failed");
    std::string err;
    cc_status st;
    try {
        st = cc::plan_build(k, edges_host, root, flags, P, &err);
    } catch (const std::bad_alloc&) {
        st = CC_ENOMEM;
        err = "host allocation failed while planning";
    } catch (...) {
        st = CC_EINTERNAL;
        err = "planner failed";
    }
    if (st != CC_OK) {
        delete P;
        return fail(st, err);
    }
    *out = P;
    g_err.clear();
    return CC_OK;
}

cc_status cc_plan_info_get(const cc_plan* P, cc_plan_info* o) {
    if (!P || !o) return fail(CC_EINVAL, "NULL argument");
    o->k = P->k;
    o->root = P->root;
    o->n_splits = (int32_t)P->splits.size();
    o->aut = P->aut;
    o->units_per_edge = P->units_per_edge;
    o->table3_memory = P->t3_memory;
    o->table3_compute = P->t3_compute;
    o->gather_doubles_per_edge = P->gather_per_edge;
    o->combine_fma_per_vertex = P->combine_per_vertex;
    o->peak_live_columns = P->peak_live_cols;
    o->device_bytes = P->consts.size();
    return CC_OK;
}

cc_status cc_plan_split_get(const cc_plan* P, int32_t i, int32_t* s, int32_t* a, int32_t* p) {
    if (!P || !s || !a || !p) return fail(CC_EINVAL, "NULL argument");
    if (i < 0 || i >= (int32_t)P->splits.size()) return fail(CC_ERANGE, "split index out of range");
    *s = P->splits[i].s;
    *a = P->splits[i].a;
    *p = P->splits[i].p;
    return CC_OK;
}

cc_status cc_plan_bind_device(cc_plan* P, void* dev, size_t bytes, void* stream) {
    if (!P || !dev) return fail(CC_EINVAL, "NULL argument");
    if (bytes < P->consts.size()) return fail(CC_ENOSPC, "device buffer smaller than info.device_bytes");
    hipError_t e = hipMemcpyAsync(dev, P->consts.data(), P->consts.size(), hipMemcpyHostToDevice,
                                  (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(plan constants)");
    e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize(plan constants)");
    P->dev = dev;
    P->dev_bytes = bytes;
    return CC_OK;
}

void cc_plan_destroy(cc_plan* P) { delete P; }

cc_status cc_plan_split_maps(const cc_plan* P, int32_t i, cc_split_maps* o) {
    if (!P || !o) return fail(CC_EINVAL, "NULL argument");
    if (i < 0 || i >= (int32_t)P->splits.size()) return fail(CC_ERANGE, "split index out of range");
    const cc::Split& sp = P->splits[(size_t)i];
    o->act = sp.act;
    o->pas = sp.pas;
    o->out = sp.out;
    o->split_off = sp.split_off;
    o->fold_off = sp.fold_off;
    o->mask_off = sp.mask_off;
    o->full_off = sp.full_off;
    o->emap_off = sp.emap_off;
    o->proj_src_off = sp.proj_src_off;
    o->proj_fold_off = sp.proj_fold_off;
    o->Wn = sp.Wn;
    return CC_OK;
}

cc_status cc_plan_constants_get(const cc_plan* P, void* host, size_t bytes) {
    if (!P || (!host && !P->consts.empty())) return fail(CC_EINVAL, "NULL argument");
    if (bytes < P->consts.size()) return fail(CC_ENOSPC, "buffer smaller than the plan's constants");
    if (!P->consts.empty()) std::memcpy(host, P->consts.data(), P->consts.size());
    return CC_OK;
}

cc_status cc_entry_order(int32_t k, int32_t m, int32_t* order, int64_t n) {
    if (k < 1 || k > cc::kMaxK) return fail(CC_ERANGE, "k out of range");
    if (m < 0 || m > k - 1) return fail(CC_ERANGE, "m out of range");
    if (!order) return fail(CC_EINVAL, "order is NULL");
    if (n != cc::binom(k - 1, m)) return fail(CC_EINVAL, "n must be C(k-1, m)");
    try {
        const std::vector<int> o = cc::entry_order(k - 1, m);
        for (int64_t i = 0; i < n; ++i) order[i] = o[(size_t)i];
    } catch (const std::bad_alloc&) {
        return fail(CC_ENOMEM, "host allocation failed");
    }
    return CC_OK;
}

cc_status cc_profile_enable(cc_plan* P, int32_t enable) {
    if (!P) return fail(CC_EINVAL, "NULL plan");
    for (auto& v : P->prof_events)
        for (void* e : v) (void)hipEventDestroy((hipEvent_t)e);
    P->prof_events.assign(P->splits.size(), {});
    P->prof_launches.assign(P->splits.size(), 0);
    P->profiling = enable != 0;
    return CC_OK;
}

cc_status cc_profile_read(cc_plan* P, int32_t n, double* gather_ms, double* finish_ms, int64_t* launches) {
    if (!P) return fail(CC_EINVAL, "NULL plan");
    if (n < 0 || n > (int32_t)P->splits.size()) return fail(CC_ERANGE, "n out of range");
    if (P->prof_events.size() != P->splits.size()) {
        P->prof_events.assign(P->splits.size(), {});
        P->prof_launches.assign(P->splits.size(), 0);
    }
    cc_status st = CC_OK;
    for (int32_t i = 0; i < (int32_t)P->splits.size(); ++i) {
        double g = 0.0, f = 0.0;
        auto& ev = P->prof_events[(size_t)i];
        for (size_t j = 0; j + 3 <= ev.size(); j += 3) {
            hipEvent_t a = (hipEvent_t)ev[j], b = (hipEvent_t)ev[j + 1], c = (hipEvent_t)ev[j + 2];
            float t1 = 0.f, t2 = 0.f;
            hipError_t e = hipEventSynchronize(c);
            if (e == hipSuccess) e = hipEventElapsedTime(&t1, a, b);
            if (e == hipSuccess) e = hipEventElapsedTime(&t2, b, c);
            if (e != hipSuccess) st = hip_fail(e, "profile events");
            g += t1;
            f += t2;
        }
        if (i < n) {
            if (gather_ms) gather_ms[i] = g;
            if (finish_ms) finish_ms[i] = f;
            if (launches) launches[i] = P->prof_launches[(size_t)i];
        }
        for (void* e : ev) (void)hipEventDestroy((hipEvent_t)e);
        ev.clear();
        P->prof_launches[(size_t)i] = 0;
    }
    return st;
}

cc_plan::~cc_plan() {
    for (auto& v : prof_events)
        for (void* e : v) (void)hipEventDestroy((hipEvent_t)e);
}

cc_status cc_graph_workspace_bytes(int64_t n, int64_t nnz, const cc_tuning* tuning, size_t* bytes) {
    if (!bytes || n < 0 || nnz < 0) return fail(CC_EINVAL, "bad argument");
    if (n >= ((int64_t)1 << 31)) return fail(CC_ERANGE, "n must be below 2^31");
    int32_t thr, chunk;
    resolve_tuning(nnz, tuning, &thr, &chunk);
    *bytes = graph_layout(n, nnz, thr, chunk).total;
    return CC_OK;
}

cc_status cc_graph_prepare(int64_t n, int64_t nnz, const int64_t* row_ptr_dev, const int32_t* col_dev,
                           void* ws_dev, size_t ws_bytes, const cc_tuning* tuning, uint32_t flags,
                           void* stream, cc_graph** out) {
    if (!out) return fail(CC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 0 || nnz < 0 || !row_ptr_dev || (nnz > 0 && !col_dev) || !ws_dev)
        return fail(CC_EINVAL, "bad graph arguments");
    if (n >= ((int64_t)1 << 31)) return fail(CC_ERANGE, "n must be below 2^31");
    int32_t thr, chunk, cols;
    resolve_tuning(nnz, tuning, &thr, &chunk, &cols);
    if (tuning && (tuning->proj_classes < -1 || tuning->proj_classes > CC_MAX_K))
        return fail(CC_EINVAL, "proj_classes must be -1, 0 or 1..16");
    if (tuning && tuning->packed_tile != 0 && tuning->packed_tile != 128 && tuning->packed_tile != 256 &&
        tuning->packed_tile != 512)
        return fail(CC_EINVAL, "packed_tile must be 0, 128, 256 or 512");
    if (cols != 0 && cols != 1 && cols != 2 && cols != 4 && cols != 8 && cols != 16)
        return fail(CC_EINVAL, "cols_per_lane must be 0, 1, 2, 4, 8 or 16");
    GraphLayout L = graph_layout(n, nnz, thr, chunk);
    if (ws_bytes < L.total) return fail(CC_ENOSPC, "graph workspace too small");
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)ws_dev;
    unsigned* dflags = (unsigned*)(ws + L.flags_off);
    hipError_t e;
    // row offsets are checked on the host first, so that the validation kernel only follows
    // offsets that stay inside col
    std::vector<int64_t> rp((size_t)n + 1);
    e = hipMemcpyAsync(rp.data(), row_ptr_dev, sizeof(int64_t) * (size_t)(n + 1), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "row offset readback");
    if (rp[0] != 0 || rp[n] != nnz) return fail(CC_EINVAL, "row_ptr[0] must be 0 and row_ptr[n] = nnz");
    for (int64_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v]) return fail(CC_EINVAL, "row offsets decrease");
    if (!(flags & CC_GRAPH_TRUST)) {
        e = cc::launch_fill_u32(dflags, 1, 0u, st);
        if (e != hipSuccess) return hip_fail(e, "validation launch");
        e = cc::launch_validate(row_ptr_dev, col_dev, n, nnz, dflags, st);
        if (e != hipSuccess) return hip_fail(e, "validation launch");
        unsigned hf = 0;
        e = hipMemcpyAsync(&hf, dflags, sizeof(unsigned), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "validation readback");
        if (hf) {
            std::string m = "CSR validation failed:";
            if (hf & 1u) m += " column out of range;";
            if (hf & 2u) m += " self-loop;";
            if (hf & 4u) m += " unsorted or duplicate entries;";
            if (hf & 8u) m += " not symmetric;";
            return fail(CC_EINVAL, m);
        }
    }
    std::vector<int32_t> light;
    std::vector<cc::ChunkItem> chunks;
    std::vector<cc::HubItem> hubs;
    int64_t maxdeg = 0;
    light.reserve((size_t)n);
    for (int64_t v = 0; v < n; ++v) {
        const int64_t d = rp[v + 1] - rp[v];
        maxdeg = std::max(maxdeg, d);
        if (d > thr) {
            cc::HubItem h;
            h.v = (int32_t)v;
            h.first_chunk = (int64_t)chunks.size();
            for (int64_t b = rp[v]; b < rp[v + 1]; b += chunk) {
                cc::ChunkItem c;
                c.beg = b;
                c.v = (int32_t)v;
                c.len = (int32_t)std::min<int64_t>(chunk, rp[v + 1] - b);
                chunks.push_back(c);
            }
            h.n_chunks = (int32_t)(chunks.size() - h.first_chunk);
            hubs.push_back(h);
        } else {
            light.push_back((int32_t)v);
        }
    }
    // heaviest rows first so that long items start early
    std::stable_sort(light.begin(), light.end(), [&](int32_t a, int32_t b) {
        return (rp[a + 1] - rp[a]) > (rp[b + 1] - rp[b]);
    });
    // light ranges: consecutive light rows (heaviest first) totalling at most `chunk` entries
    // (a single heavier row forms its own range) and at most kRangeRows rows
    std::vector<int32_t> starts;
    starts.reserve(light.size() / 8 + 2);
    {
        int64_t acc = 0, cnt = 0;
        for (size_t i = 0; i < light.size(); ++i) {
            const int64_t d = rp[light[i] + 1] - rp[light[i]];
            if (cnt == 0 || acc + d > chunk || cnt == kRangeRows) {
                starts.push_back((int32_t)i);
                acc = 0;
                cnt = 0;
            }
            acc += d;
            ++cnt;
        }
        starts.push_back((int32_t)light.size());
    }
    cc_graph* G = new (std::nothrow) cc_graph();
    if (!G) return fail(CC_ENOMEM, "graph allocation failed");
    G->n = n;
    G->nnz = nnz;
    G->max_degree = maxdeg;
    G->row_ptr = row_ptr_dev;
    G->col = col_dev;
    G->light = (int32_t*)(ws + L.light_off);
    G->light_start = (int32_t*)(ws + L.range_off);
    G->n_ranges = (int64_t)starts.size() - 1;
    G->chunks = (cc::ChunkItem*)(ws + L.chunk_off);
    G->hubs = (cc::HubItem*)(ws + L.hub_off);
    G->n_light = (int64_t)light.size();
    G->n_chunks = (int64_t)chunks.size();
    G->n_hubs = (int64_t)hubs.size();
    G->hub_threshold = thr;
    G->chunk = chunk;
    G->cols_per_lane = cols;
    G->proj_classes = tuning ? tuning->proj_classes : 0;
    G->packed_tile = tuning ? tuning->packed_tile : 0;
    e = hipGetDevice(&G->device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&G->n_cu, hipDeviceAttributeMultiprocessorCount, G->device);
    if (e == hipSuccess && !light.empty())
        e = hipMemcpyAsync(G->light, light.data(), light.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(G->light_start, starts.data(), starts.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !chunks.empty())
        e = hipMemcpyAsync(G->chunks, chunks.data(), chunks.size() * sizeof(cc::ChunkItem), hipMemcpyHostToDevice, st);
    if (e == hipSuccess && !hubs.empty())
        e = hipMemcpyAsync(G->hubs, hubs.data(), hubs.size() * sizeof(cc::HubItem), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete G;
        return hip_fail(e, "graph work-list upload");
    }
    *out = G;
    return CC_OK;
}

cc_status cc_graph_info_get(const cc_graph* G, cc_graph_info* o) {
    if (!G || !o) return fail(CC_EINVAL, "NULL argument");
    o->n = G->n;
    o->nnz = G->nnz;
    o->max_degree = G->max_degree;
    o->n_light = G->n_light;
    o->n_hubs = G->n_hubs;
    o->n_chunks = G->n_chunks;
    o->hub_threshold = G->hub_threshold;
    o->chunk = G->chunk;
    o->cols_per_lane = G->cols_per_lane;
    o->proj_classes = G->proj_classes;
    o->packed_tile = G->packed_tile;
    return CC_OK;
}

void cc_graph_release(cc_graph* G) { delete G; }

cc_status cc_color(const cc_graph* G, int32_t k, uint64_t seed, uint64_t first_iter, int32_t B,
                   uint8_t* colours_dev, void* stream) {
    if (!G || (!colours_dev && B > 0 && G->n > 0)) return fail(CC_EINVAL, "NULL argument");
    if (k < 1 || k > CC_MAX_K) return fail(CC_ERANGE, "k must be in [1, 16]");
    if (B < 0) return fail(CC_EINVAL, "B must be >= 0");
    hipError_t e = cc::launch_colour(seed, first_iter, G->n, k, B, colours_dev, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "colour launch");
    return CC_OK;
}

cc_status cc_count_workspace_bytes(const cc_plan* P, const cc_graph* G, size_t* bytes) {
    if (!P || !G || !bytes) return fail(CC_EINVAL, "NULL argument");
    *bytes = count_layout(P, G).total;
    return CC_OK;
}

cc_status cc_count_projection(const cc_plan* P, const cc_graph* G, int32_t* classes, int32_t n) {
    if (!P || !G || !classes) return fail(CC_EINVAL, "NULL argument");
    if (n < (int32_t)P->splits.size()) return fail(CC_EINVAL, "classes holds fewer entries than the plan has splits");
    const std::vector<int> g = projection_plan(P, G, pad32(G->n));
    for (size_t i = 0; i < g.size(); ++i) classes[i] = g[i];
    return CC_OK;
}

}  // extern "C"

namespace {

// Splits [0, last] of plan P for one colouring on `st`: the per-entry neighbour colours, then
// every split's gather + combine and cut-row finish, timed per split while profiling.
// Where each table of a count lives when some tables are parked in host memory over an idle
// stretch (cc_count_budget): a parked table t holds columns off_a[t] from its production to split
// g0[t] (its last use before the stretch, or its production), is copied to the caller's host
// buffer at host_off[t] after split g0[t], and comes back into columns off_b[t] just before split
// g1[t] (its next use), where it stays until its last use. Unparked tables hold off_a for their
// whole life (off_b = off_a).
struct Placement {
    std::vector<int64_t> off_a, off_b;
    std::vector<int> parked, g0, g1;
    std::vector<size_t> host_off;
    uint8_t* host = nullptr;
    // columns of table t for split j
    int64_t off(size_t t, int j) const { return (parked[t] && j >= g1[t]) ? off_b[t] : off_a[t]; }
};

hipError_t run_splits(const cc_plan* P, const cc_graph* G, const uint8_t* colour, const CountLayout& L, uint8_t* ws,
                      double* root_out, int64_t last, hipStream_t st, const Placement* PL = nullptr) {
    double* arena = (double*)(ws + L.arena_off);
    double* partial = (double*)(ws + L.partial_off);
    uint8_t* ecol = ws + L.ecol_off;
    // every split reads the colour of each CSR entry's vertex: gathered once per colouring into a
    // sequential array instead of once per split at random
    hipError_t e = cc::launch_edge_colours(G->col, colour, G->nnz, ecol, st);
    const cc_plan* plan = P;
    // a projected split: per pass, copy the needed entries of every passive row for the pass's
    // centre colours, then run the pass's centres on the copies; the cut rows finish at the end
    auto projected = [&](const cc::Split& sp, const cc::StepParams& h, int cls, hipEvent_t mid) -> hipError_t {
        const uint8_t* cdev = (const uint8_t*)plan->dev;
        const int k = plan->k;
        cc::StepParams hp = h;
        hp.P = (const double*)(ws + L.proj_off);
        hp.pstride = sp.Wn_pad;
        hp.Wp = sp.Wn;
        hp.fold = (const uint16_t*)(cdev + sp.proj_fold_off);
        hp.mask = (const uint16_t*)(cdev + sp.proj_mask_off);
        hp.class_stride = L.n_pad * sp.Wn_pad;
        hipError_t err = hipSuccess;
        for (int c0 = 0; err == hipSuccess && c0 < k; c0 += cls) {
            const int c1 = std::min(k, c0 + cls);
            uint32_t m = ((1u << c1) - 1u) & ~((1u << c0) - 1u);
            if (c0 == 0) m |= cc::kAnyInvalid;
            err = cc::launch_project(h.P, h.pstride, sp.Wp, colour, G->n, k, (const uint16_t*)(cdev + sp.proj_src_off),
                                     sp.Wn, sp.Wn_pad, hp.class_stride, m & ((1u << k) - 1u),
                                     (double*)(ws + L.proj_off), st);
            hp.cls_mask = m;
            if (err == hipSuccess) err = cc::launch_split_tasks(hp, G->n_cu, st);
        }
        if (err == hipSuccess && mid) err = hipEventRecord(mid, st);
        if (err == hipSuccess) err = cc::launch_hub_finish(h, G->n_cu, st);
        return err;
    };
    // bytes of one table's rows (vertex-major, n rows of its stride)
    auto table_bytes = [&](int t) { return (size_t)G->n * (size_t)P->tables[(size_t)t].stride * sizeof(double); };
    for (int64_t i = 0; e == hipSuccess && i <= last; ++i) {
        const cc::Split& sp = P->splits[(size_t)i];
        cc::StepParams h = step_params(P, G, sp, colour, arena, L.n_pad, partial, root_out);
        h.ecol = ecol;
        if (PL) {
            // parked tables read again by this split come back from host memory
            for (size_t t = 0; e == hipSuccess && t < P->tables.size(); ++t)
                if (PL->parked[t] && PL->g1[t] == (int)i)
                    e = hipMemcpyAsync(arena + PL->off_b[t] * L.n_pad, PL->host + PL->host_off[t], table_bytes((int)t),
                                       hipMemcpyHostToDevice, st);
            if (sp.act >= 0) h.A = arena + PL->off((size_t)sp.act, (int)i) * L.n_pad;
            if (sp.pas >= 0) h.P = arena + PL->off((size_t)sp.pas, (int)i) * L.n_pad;
            if (sp.out >= 0) h.O = arena + PL->off((size_t)sp.out, (int)i) * L.n_pad;
        }
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        if (P->profiling) {
            for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipEventCreate(&ev[q]);
            if (e == hipSuccess) e = hipEventRecord(ev[0], st);
        }
        const int cls = L.proj[(size_t)i];
        if (e == hipSuccess && cls > 0) e = projected(sp, h, cls, P->profiling ? ev[1] : nullptr);
        else if (e == hipSuccess) e = cc::launch_split(h, G->n_cu, st, P->profiling ? ev[1] : nullptr);
        if (e == hipSuccess && P->profiling) {
            e = hipEventRecord(ev[2], st);
            auto& pe = P->prof_events[(size_t)i];
            pe.push_back(ev[0]);
            pe.push_back(ev[1]);
            pe.push_back(ev[2]);
            P->prof_launches[(size_t)i] += 1;
        }
        // a table parked after this split goes to host memory now; its device columns are reused
        // by later splits only after the copy (the stream orders them)
        for (size_t t = 0; e == hipSuccess && PL && t < P->tables.size(); ++t)
            if (PL->parked[t] && PL->g0[t] == (int)i)
                e = hipMemcpyAsync(PL->host + PL->host_off[t], arena + PL->off_a[t] * L.n_pad, table_bytes((int)t),
                                   hipMemcpyDeviceToHost, st);
    }
    return e;
}

// Tables parked in host memory so that a count fits a device budget. Each table lives over an
// interval of splits (from the split that writes it to its last reader); parking it over an idle
// stretch (between two consecutive uses, the write counting as one) splits that interval in two.
// Columns are assigned to the intervals largest first, each at the lowest offset free over its
// whole interval. While that arena exceeds the budget, the largest table idle at the split where
// the resident columns peak is parked over that stretch (one stretch per table).
struct BudgetLayout {
    CountLayout L;
    Placement PL;
    int64_t arena_cols = 0, unbounded_cols = 0;
    int parked = 0;
    size_t host_bytes = 0;
    bool fits = false;
};

BudgetLayout budget_layout(const cc_plan* P, const cc_graph* G, size_t budget) {
    BudgetLayout B;
    const size_t nt = P->tables.size(), ns = P->splits.size();
    // the splits that write and read each table, in order
    std::vector<std::vector<int>> events(nt);
    for (size_t j = 0; j < ns; ++j) {
        const cc::Split& sp = P->splits[j];
        for (int t : {sp.out, sp.act, sp.pas})
            if (t >= 0 && (events[(size_t)t].empty() || events[(size_t)t].back() != (int)j))
                events[(size_t)t].push_back((int)j);
    }
    Placement& PL = B.PL;
    PL.parked.assign(nt, 0);
    PL.g0.assign(nt, -1);
    PL.g1.assign(nt, -1);
    auto stride = [&](size_t t) { return (int64_t)P->tables[t].stride; };
    struct Iv {
        int64_t len;
        int s, e;
        size_t t;
        bool second;
    };
    // offsets for the current parking choice; returns the arena width
    auto place = [&]() -> int64_t {
        std::vector<Iv> iv;
        for (size_t t = 0; t < nt; ++t) {
            if (events[t].empty()) continue;
            if (PL.parked[t]) {
                iv.push_back({stride(t), events[t].front(), PL.g0[t], t, false});
                iv.push_back({stride(t), PL.g1[t], events[t].back(), t, true});
            } else {
                iv.push_back({stride(t), events[t].front(), events[t].back(), t, false});
            }
        }
        std::stable_sort(iv.begin(), iv.end(), [](const Iv& a, const Iv& b) {
            return a.len != b.len ? a.len > b.len : a.s < b.s;
        });
        std::vector<std::pair<const Iv*, int64_t>> placed;
        int64_t width = 0;
        PL.off_a.assign(nt, 0);
        PL.off_b.assign(nt, 0);
        for (const Iv& x : iv) {
            std::vector<std::pair<int64_t, int64_t>> busy;  // columns taken over x's splits
            for (auto& pr : placed)
                if (std::max(pr.first->s, x.s) <= std::min(pr.first->e, x.e)) busy.push_back({pr.second, pr.first->len});
            std::sort(busy.begin(), busy.end());
            int64_t off = 0;
            for (auto& b : busy) {
                if (b.first - off >= x.len) break;
                off = std::max(off, b.first + b.second);
            }
            placed.push_back({&x, off});
            width = std::max(width, off + x.len);
            if (x.second) PL.off_b[x.t] = off;
            else PL.off_a[x.t] = off;
        }
        for (size_t t = 0; t < nt; ++t)
            if (!PL.parked[t]) PL.off_b[t] = PL.off_a[t];
        return width;
    };
    B.unbounded_cols = P->arena_cols;
    int proj_cap = -1;  // the projected rows' scratch shrinks once nothing more can be parked
    for (;;) {
        B.arena_cols = place();
        B.L = count_layout(P, G, B.arena_cols, proj_cap);
        if (B.L.total <= budget) {
            B.fits = true;
            break;
        }
        // the split where the most columns are resident
        int64_t best_live = -1;
        int jstar = 0;
        for (size_t j = 0; j < ns; ++j) {
            int64_t live = 0;
            for (size_t t = 0; t < nt; ++t) {
                if (events[t].empty()) continue;
                const int J = (int)j;
                const bool res = PL.parked[t] ? ((events[t].front() <= J && J <= PL.g0[t]) ||
                                                 (PL.g1[t] <= J && J <= events[t].back()))
                                              : (events[t].front() <= J && J <= events[t].back());
                if (res) live += stride(t);
            }
            if (live > best_live) {
                best_live = live;
                jstar = (int)j;
            }
        }
        // the largest unparked table resident but idle there: two consecutive events around jstar
        int pick = -1, pg0 = -1, pg1 = -1;
        for (size_t t = 0; t < nt; ++t) {
            if (PL.parked[t]) continue;
            const std::vector<int>& ev = events[t];
            for (size_t q = 0; q + 1 < ev.size(); ++q)
                if (ev[q] < jstar && jstar < ev[q + 1] && (pick < 0 || stride(t) > stride((size_t)pick))) {
                    pick = (int)t;
                    pg0 = ev[q];
                    pg1 = ev[q + 1];
                }
        }
        if (pick < 0) {
            // nothing idle at the peak: fewer colour classes per projected pass, then none
            int most = 0;
            for (int c : B.L.proj) most = std::max(most, c);
            if (most == 0) break;  // the budget cannot be met
            proj_cap = most / 2;
            continue;
        }
        PL.parked[(size_t)pick] = 1;
        PL.g0[(size_t)pick] = pg0;
        PL.g1[(size_t)pick] = pg1;
        ++B.parked;
    }
    PL.host_off.assign(nt, 0);
    for (size_t t = 0; t < nt; ++t)
        if (PL.parked[t]) {
            PL.host_off[t] = B.host_bytes;
            B.host_bytes = align256(B.host_bytes + (size_t)G->n * (size_t)stride(t) * sizeof(double));
        }
    return B;
}

}  // namespace

extern "C" {

cc_status cc_count(const cc_plan* P, const cc_graph* G, const uint8_t* colours_dev, int32_t B, void* ws_dev,
                   size_t ws_bytes, double* X_dev, double* vertex_dev, void* stream) {
    if (!P || !G) return fail(CC_EINVAL, "NULL plan or graph");
    if (B < 0) return fail(CC_EINVAL, "B must be >= 0");
    if (B == 0) return CC_OK;
    if (!X_dev || !ws_dev || (G->n > 0 && !colours_dev)) return fail(CC_EINVAL, "NULL buffer");
    if (!P->splits.empty() && !P->dev) return fail(CC_EINVAL, "plan not bound to device memory");
    CountLayout L = count_layout(P, G);
    if (ws_bytes < L.total) return fail(CC_ENOSPC, "count workspace too small");
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)ws_dev;
    double* red = (double*)(ws + L.red_off);
    const int64_t n = G->n;
    hipError_t e = hipSuccess;
    for (int32_t b = 0; b < B; ++b) {
        double* root_out = vertex_dev ? vertex_dev + (int64_t)b * n : (double*)(ws + L.root_off);
        if (n == 0) {
            e = cc::launch_fill_f64(X_dev + b, 1, 0.0, st);
            if (e != hipSuccess) return hip_fail(e, "fill");
            continue;
        }
        const uint8_t* colour = colours_dev + (int64_t)b * n;
        if (P->splits.empty()) {
            // k = 1: every vertex roots exactly one map
            e = cc::launch_fill_f64(root_out, n, 1.0, st);
        } else {
            e = run_splits(P, G, colour, L, ws, root_out, (int64_t)P->splits.size() - 1, st);
        }
        if (e == hipSuccess) e = cc::launch_reduce(root_out, n, red, X_dev + b, st);
        if (e != hipSuccess) return hip_fail(e, "count launch");
    }
    return CC_OK;
}

cc_status cc_count_budget_plan(const cc_plan* P, const cc_graph* G, size_t device_budget, cc_budget_info* o) {
    if (!P || !G || !o) return fail(CC_EINVAL, "NULL argument");
    const BudgetLayout Bl = budget_layout(P, G, device_budget);
    o->workspace_bytes = Bl.L.total;
    o->host_bytes = Bl.host_bytes;
    o->parked_tables = Bl.parked;
    o->proj_classes = 0;
    for (int c : Bl.L.proj) o->proj_classes = std::max(o->proj_classes, c);
    o->arena_columns = Bl.arena_cols;
    o->unbounded_columns = Bl.unbounded_cols;
    if (!Bl.fits) return fail(CC_ENOSPC, "the count does not fit this device budget even with tables parked in host memory");
    return CC_OK;
}

cc_status cc_count_budget(const cc_plan* P, const cc_graph* G, const uint8_t* colours_dev, int32_t B,
                          size_t device_budget, void* ws_dev, size_t ws_bytes, void* host_buf, size_t host_bytes,
                          double* X_dev, double* vertex_dev, void* stream) {
    if (!P || !G) return fail(CC_EINVAL, "NULL plan or graph");
    if (B < 0) return fail(CC_EINVAL, "B must be >= 0");
    if (B == 0) return CC_OK;
    if (!X_dev || !ws_dev || (G->n > 0 && !colours_dev)) return fail(CC_EINVAL, "NULL buffer");
    if (!P->splits.empty() && !P->dev) return fail(CC_EINVAL, "plan not bound to device memory");
    BudgetLayout Bl = budget_layout(P, G, device_budget);
    if (!Bl.fits) return fail(CC_ENOSPC, "the count does not fit this device budget even with tables parked in host memory");
    if (ws_bytes < Bl.L.total) return fail(CC_ENOSPC, "count workspace too small");
    if (Bl.host_bytes > 0 && (!host_buf || host_bytes < Bl.host_bytes))
        return fail(CC_ENOSPC, "host buffer for the parked tables too small");
    Bl.PL.host = (uint8_t*)host_buf;
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)ws_dev;
    double* red = (double*)(ws + Bl.L.red_off);
    const int64_t n = G->n;
    hipError_t e = hipSuccess;
    for (int32_t b = 0; b < B; ++b) {
        double* root_out = vertex_dev ? vertex_dev + (int64_t)b * n : (double*)(ws + Bl.L.root_off);
        if (n == 0) {
            e = cc::launch_fill_f64(X_dev + b, 1, 0.0, st);
            if (e != hipSuccess) return hip_fail(e, "fill");
            continue;
        }
        const uint8_t* colour = colours_dev + (int64_t)b * n;
        if (P->splits.empty()) e = cc::launch_fill_f64(root_out, n, 1.0, st);
        else e = run_splits(P, G, colour, Bl.L, ws, root_out, (int64_t)P->splits.size() - 1, st, &Bl.PL);
        if (e == hipSuccess) e = cc::launch_reduce(root_out, n, red, X_dev + b, st);
        if (e != hipSuccess) return hip_fail(e, "budgeted count launch");
    }
    return CC_OK;
}

cc_status cc_count_inspect(const cc_plan* P, const cc_graph* G, const uint8_t* colours_dev, int32_t last,
                           void* ws_dev, size_t ws_bytes, double* vertex_dev, void* stream) {
    if (!P || !G) return fail(CC_EINVAL, "NULL plan or graph");
    if (last < 0 || last >= (int32_t)P->splits.size()) return fail(CC_ERANGE, "split index out of range");
    if (!ws_dev || (G->n > 0 && !colours_dev)) return fail(CC_EINVAL, "NULL buffer");
    if (P->splits[(size_t)last].out == -2 && !vertex_dev && G->n > 0)
        return fail(CC_EINVAL, "the last split writes the root counts: vertex_dev is needed");
    if (!P->dev) return fail(CC_EINVAL, "plan not bound to device memory");
    CountLayout L = count_layout(P, G);
    if (ws_bytes < L.total) return fail(CC_ENOSPC, "count workspace too small");
    if (G->n == 0) return CC_OK;
    hipError_t e = run_splits(P, G, colours_dev, L, (uint8_t*)ws_dev, vertex_dev, last, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "inspection count launch");
    return CC_OK;
}

cc_status cc_plan_table_get(const cc_plan* P, const cc_graph* G, int32_t table, cc_table_desc* o) {
    if (!P || !G || !o) return fail(CC_EINVAL, "NULL argument");
    if (table < 0 || table >= (int32_t)P->tables.size()) return fail(CC_ERANGE, "table id out of range");
    const cc::Table& t = P->tables[(size_t)table];
    const CountLayout L = count_layout(P, G);
    o->size = t.size;
    o->width = t.W;
    o->stride = t.stride;
    o->offset = (int64_t)L.arena_off + t.col_off * L.n_pad * (int64_t)sizeof(double);
    return CC_OK;
}

cc_status cc_count_packed_workspace_bytes(const cc_plan* P, const cc_graph* G, int32_t B, size_t* bytes) {
    if (!P || !G || !bytes) return fail(CC_EINVAL, "NULL argument");
    if (B < 1 || B > CC_MAX_PACKED) return fail(CC_ERANGE, "B must be in [1, CC_MAX_PACKED]");
    *bytes = packed_layout(P, G, B).total;
    return CC_OK;
}

cc_status cc_count_packed(const cc_plan* P, const cc_graph* G, const uint8_t* colours_dev, int32_t B, void* ws_dev,
                          size_t ws_bytes, double* X_dev, double* vertex_dev, void* stream) {
    if (!P || !G) return fail(CC_EINVAL, "NULL plan or graph");
    if (B < 1 || B > CC_MAX_PACKED) return fail(CC_ERANGE, "B must be in [1, CC_MAX_PACKED]");
    if (!X_dev || !ws_dev || (G->n > 0 && !colours_dev)) return fail(CC_EINVAL, "NULL buffer");
    if (!P->splits.empty() && !P->dev) return fail(CC_EINVAL, "plan not bound to device memory");
    if (!packed_fits(P, B)) return fail(CC_ERANGE, "template too large for the packed layout (use cc_count)");
    PackedLayout L = packed_layout(P, G, B);
    if (ws_bytes < L.total) return fail(CC_ENOSPC, "count workspace too small");
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)ws_dev;
    const int64_t n = G->n;
    hipError_t e = hipSuccess;
    if (n == 0) {
        e = cc::launch_fill_f64(X_dev, B, 0.0, st);
        if (e != hipSuccess) return hip_fail(e, "fill");
        return CC_OK;
    }
    double* arena = (double*)(ws + L.arena_off);
    double* partial = (double*)(ws + L.partial_off);
    double* root_out = vertex_dev ? vertex_dev : (double*)(ws + L.root_off);
    uint8_t* cpk = ws + L.colour_off;
    double* red = (double*)(ws + L.red_off);
    e = cc::launch_transpose_colours(colours_dev, n, B, cpk, st);
    if (e == hipSuccess && P->splits.empty()) e = cc::launch_fill_f64(root_out, n * B, 1.0, st);
    for (size_t i = 0; e == hipSuccess && i < P->splits.size(); ++i) {
        const cc::Split& sp = P->splits[i];
        // wide rows run the one-colouring kernels colouring after colouring (they share the
        // chunk-partial scratch, so they run in stream order); each launch pair is timed alone
        const bool packed_k = cc::packed_kernel_split(sp);
        for (int32_t b = 0; e == hipSuccess && b < (packed_k ? 1 : B); ++b) {
            hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
            if (P->profiling) {
                for (int q = 0; q < 3 && e == hipSuccess; ++q) e = hipEventCreate(&ev[q]);
                if (e == hipSuccess) e = hipEventRecord(ev[0], st);
            }
            if (e == hipSuccess) {
                if (packed_k) {
                    cc::StepParams h = packed_step_params(P, G, sp, own_ids(sp), cpk, arena, L, partial, root_out, B);
                    e = cc::launch_packed_split(h, G->n_cu, st, P->profiling ? ev[1] : nullptr);
                } else {
                    cc::StepParams h =
                        packed_one_params(P, G, sp, own_ids(sp), colours_dev, arena, L, partial, root_out, B, b);
                    e = cc::launch_split(h, G->n_cu, st, P->profiling ? ev[1] : nullptr);
                }
            }
            if (e == hipSuccess && P->profiling) {
                e = hipEventRecord(ev[2], st);
                auto& pe = P->prof_events[i];
                pe.push_back(ev[0]);
                pe.push_back(ev[1]);
                pe.push_back(ev[2]);
                P->prof_launches[i] += 1;
            }
        }
    }
    if (e == hipSuccess) e = cc::launch_reduce_packed(root_out, n, B, red, X_dev, st);
    if (e != hipSuccess) return hip_fail(e, "packed count launch");
    return CC_OK;
}

cc_status cc_stream_check(void* stream) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "stream check");
    return CC_OK;
}

static long double scale_factor(const cc_plan* P) {
    long double s = 1.0L;
    for (int i = 1; i <= P->k; ++i) s *= (long double)P->k / (long double)i;  // k^k / k!
    return s / (long double)P->aut;
}

cc_status cc_estimate(const cc_plan* P, const double* X_host, int32_t B, double* estimate, double* std_err) {
    if (!P || !X_host || !estimate) return fail(CC_EINVAL, "NULL argument");
    if (B < 1) return fail(CC_EINVAL, "B must be >= 1");
    long double m = 0.0L;
    for (int32_t b = 0; b < B; ++b) m += (long double)X_host[b];
    m /= (long double)B;
    long double var = 0.0L;
    for (int32_t b = 0; b < B; ++b) {
        long double d = (long double)X_host[b] - m;
        var += d * d;
    }
    const long double f = scale_factor(P);
    *estimate = (double)(m * f);
    if (std_err) *std_err = (B > 1) ? (double)(sqrtl(var / (long double)(B - 1) / (long double)B) * f) : 0.0;
    return CC_OK;
}

cc_status cc_estimate_median_of_means(const cc_plan* P, const double* X_host, int32_t B, int32_t groups,
                                      double* estimate) {
    if (!P || !X_host || !estimate) return fail(CC_EINVAL, "NULL argument");
    if (groups < 1 || B < groups || B % groups) return fail(CC_EINVAL, "B must be a positive multiple of groups");
    const int32_t per = B / groups;
    std::vector<long double> means((size_t)groups);
    for (int32_t g = 0; g < groups; ++g) {
        long double m = 0.0L;
        for (int32_t i = 0; i < per; ++i) m += (long double)X_host[g * per + i];
        means[(size_t)g] = m / (long double)per;
    }
    std::sort(means.begin(), means.end());
    long double med = (groups % 2) ? means[(size_t)groups / 2]
                                   : 0.5L * (means[(size_t)groups / 2 - 1] + means[(size_t)groups / 2]);
    *estimate = (double)(med * scale_factor(P));
    return CC_OK;
}

cc_status cc_iterations(int32_t k, double epsilon, double delta, int64_t* per_group, int32_t* groups) {
    if (!per_group || !groups) return fail(CC_EINVAL, "NULL argument");
    if (k < 1 || k > CC_MAX_K) return fail(CC_ERANGE, "k must be in [1, 16]");
    if (!(epsilon > 0.0 && epsilon < 1.0) || !(delta > 0.0 && delta < 1.0))
        return fail(CC_ERANGE, "epsilon and delta must be in (0, 1)");
    const long double s = ceill(4.0L * expl((long double)k) / ((long double)epsilon * (long double)epsilon));
    if (s > 4.0e18L) return fail(CC_ERANGE, "per-group sample size too large");
    const long double t = ceill(8.0L * logl(1.0L / (long double)delta));
    *per_group = (int64_t)s;
    *groups = t < 1.0L ? 1 : (int32_t)t;
    return CC_OK;
}

}  // extern "C"
