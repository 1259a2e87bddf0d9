// Multi-template packed counts (cc_multi_*, cc_count_packed_multi): several templates of one size
// over the same colourings, the table of each distinct rooted sub-template computed once.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <functional>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "cc_host.h"
#include "cc_internal.h"

using namespace cc::host;

namespace {

// workspace of a packed multi-template count: the steps' allocation sequence replayed over the
// shared tables
PackedLayout multi_layout(const cc_multi* M, const cc_graph* G, int32_t B) {
    PackedLayout L;
    L.n_pad = pad32(G->n);
    const size_t nt = M->table_W.size();
    L.col_off.assign(nt, 0);
    L.stride.resize(nt);
    L.bstep.resize(nt);
    for (size_t t = 0; t < nt; ++t) {
        const int64_t W = M->table_W[t];
        L.stride[t] = cc::packed_wide(W) ? cc::packed_stride(W) : cc::packed_stride((int64_t)B * W);
        L.bstep[t] = cc::packed_wide(W) ? L.n_pad * cc::packed_stride(W) : W;
    }
    // first-fit over columns, in step order
    std::vector<std::pair<int64_t, int64_t>> used;
    int64_t peak = 0, nst = 1;
    for (const auto& st : M->steps) {
        const cc::Split& sp = M->plans[(size_t)st.plan]->splits[(size_t)st.split];
        nst = std::max(nst, cc::packed_stride((int64_t)B * sp.Cf));
        if (st.out >= 0) {
            const int64_t len = cc::packed_cols(M->table_W[(size_t)st.out], B);
            std::sort(used.begin(), used.end());
            int64_t off = 0;
            for (auto& u : used) {
                if (u.first - off >= len) break;
                off = std::max(off, u.first + u.second);
            }
            used.push_back({off, len});
            peak = std::max(peak, off + len);
            L.col_off[(size_t)st.out] = off;
        }
        for (int g : st.release)
            for (size_t i = 0; i < used.size(); ++i)
                if (used[i].first == L.col_off[(size_t)g]) {
                    used.erase(used.begin() + (long)i);
                    break;
                }
    }
    L.nstride = nst;
    L.arena_off = 0;
    L.partial_off = align256((size_t)peak * (size_t)L.n_pad * sizeof(double));
    L.root_off = align256(L.partial_off + (size_t)G->n_chunks * (size_t)nst * sizeof(double));
    L.colour_off = align256(L.root_off + (size_t)std::max<int64_t>(G->n, 1) * (size_t)B * sizeof(double));
    L.red_off = align256(L.colour_off + (size_t)std::max<int64_t>(G->n, 1) * (size_t)B);
    L.total = align256(L.red_off + (size_t)cc::packed_reduce_blocks(G->n) * (size_t)B * sizeof(double));
    return L;
}

}  // namespace

extern "C" {

cc_status cc_multi_create(int32_t n_plans, const cc_plan* const* plans, cc_multi** out) {
    if (!out) return fail(CC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_plans < 1 || !plans) return fail(CC_EINVAL, "need at least one plan");
    for (int32_t i = 0; i < n_plans; ++i) {
        if (!plans[i]) return fail(CC_EINVAL, "NULL plan");
        if (plans[i]->k != plans[0]->k) return fail(CC_EINVAL, "all plans of a multi-template count need the same k");
    }
    cc_multi* M = new (std::nothrow) cc_multi();
    if (!M) return fail(CC_ENOMEM, "allocation failed");
    try {
        M->k = plans[0]->k;
        M->plans.assign(plans, plans + n_plans);
        std::map<std::string, int> key_to_g;
        for (int32_t p = 0; p < n_plans; ++p) {
            const cc_plan* P = plans[p];
            M->n_splits += (int64_t)P->splits.size();
            if (P->splits.empty()) continue;
            std::vector<int> producer(P->tables.size(), -1);
            for (size_t j = 0; j < P->splits.size(); ++j)
                if (P->splits[j].out >= 0) producer[(size_t)P->splits[j].out] = (int)j;
            // a table's global id, computing it (after its inputs, in the plan's own order) unless
            // an equal rooted sub-template was computed before
            std::function<int(int)> need = [&](int t) -> int {
                const std::string& key = P->tables[(size_t)t].key;
                auto it = key_to_g.find(key);
                if (it != key_to_g.end()) return it->second;
                const int j = producer[(size_t)t];
                const cc::Split& sp = P->splits[(size_t)j];
                const int a = sp.act >= 0 ? need(sp.act) : -1;
                const int q = sp.pas >= 0 ? need(sp.pas) : -1;
                const int g = (int)M->table_W.size();
                M->table_W.push_back(P->tables[(size_t)t].W);
                key_to_g[key] = g;
                M->steps.push_back(cc_multi::Step{(int)p, j, a, q, g, {}});
                return g;
            };
            const int jr = (int)P->splits.size() - 1;  // the root split comes last
            const cc::Split& sr = P->splits[(size_t)jr];
            const int a = sr.act >= 0 ? need(sr.act) : -1;
            const int q = sr.pas >= 0 ? need(sr.pas) : -1;
            M->steps.push_back(cc_multi::Step{(int)p, jr, a, q, -2, {}});
        }
        std::vector<int> last(M->table_W.size(), -1);
        for (size_t i = 0; i < M->steps.size(); ++i) {
            if (M->steps[i].act >= 0) last[(size_t)M->steps[i].act] = (int)i;
            if (M->steps[i].pas >= 0) last[(size_t)M->steps[i].pas] = (int)i;
        }
        for (size_t g = 0; g < last.size(); ++g)
            if (last[g] >= 0) M->steps[(size_t)last[g]].release.push_back((int)g);
    } catch (const std::bad_alloc&) {
        delete M;
        return fail(CC_ENOMEM, "host allocation failed");
    }
    *out = M;
    return CC_OK;
}

cc_status cc_multi_info_get(const cc_multi* M, int32_t* n_steps, int64_t* n_splits, int32_t* n_tables) {
    if (!M) return fail(CC_EINVAL, "NULL multi");
    if (n_steps) *n_steps = (int32_t)M->steps.size();
    if (n_splits) *n_splits = M->n_splits;
    if (n_tables) *n_tables = (int32_t)M->table_W.size();
    return CC_OK;
}

cc_status cc_multi_step_get(const cc_multi* M, int32_t i, int32_t* plan, int32_t* split) {
    if (!M || !plan || !split) return fail(CC_EINVAL, "NULL argument");
    if (i < 0 || (size_t)i >= M->steps.size()) return fail(CC_ERANGE, "step index out of range");
    *plan = M->steps[(size_t)i].plan;
    *split = M->steps[(size_t)i].split;
    return CC_OK;
}

void cc_multi_destroy(cc_multi* M) { delete M; }

cc_status cc_count_packed_multi_workspace_bytes(const cc_multi* M, const cc_graph* G, int32_t B, size_t* bytes) {
    if (!M || !G || !bytes) return fail(CC_EINVAL, "NULL argument");
    if (B < 1 || B > CC_MAX_PACKED) return fail(CC_ERANGE, "B must be in [1, CC_MAX_PACKED]");
    *bytes = multi_layout(M, G, B).total;
    return CC_OK;
}

cc_status cc_count_packed_multi(const cc_multi* M, const cc_graph* G, const uint8_t* colours_dev, int32_t B,
                                void* ws_dev, size_t ws_bytes, double* X_dev, void* stream) {
    if (!M || !G) return fail(CC_EINVAL, "NULL multi or graph");
    if (B < 1 || B > CC_MAX_PACKED) return fail(CC_ERANGE, "B must be in [1, CC_MAX_PACKED]");
    if (!X_dev || !ws_dev || (G->n > 0 && !colours_dev)) return fail(CC_EINVAL, "NULL buffer");
    for (const cc_plan* P : M->plans) {
        if (!P->splits.empty() && !P->dev) return fail(CC_EINVAL, "plan not bound to device memory");
        if (!packed_fits(P, B)) return fail(CC_ERANGE, "template too large for the packed layout (use cc_count)");
    }
    PackedLayout L = multi_layout(M, G, B);
    if (ws_bytes < L.total) return fail(CC_ENOSPC, "count workspace too small");
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)ws_dev;
    const int64_t n = G->n;
    const int32_t np = (int32_t)M->plans.size();
    hipError_t e = hipSuccess;
    if (n == 0) {
        e = cc::launch_fill_f64(X_dev, (int64_t)np * B, 0.0, st);
        if (e != hipSuccess) return hip_fail(e, "fill");
        return CC_OK;
    }
    double* arena = (double*)(ws + L.arena_off);
    double* partial = (double*)(ws + L.partial_off);
    double* root_out = (double*)(ws + L.root_off);
    uint8_t* cpk = ws + L.colour_off;
    double* red = (double*)(ws + L.red_off);
    e = cc::launch_transpose_colours(colours_dev, n, B, cpk, st);
    // single-vertex templates: every vertex roots one map
    for (int32_t p = 0; e == hipSuccess && p < np; ++p)
        if (M->plans[(size_t)p]->splits.empty()) {
            e = cc::launch_fill_f64(root_out, n * B, 1.0, st);
            if (e == hipSuccess) e = cc::launch_reduce_packed(root_out, n, B, red, X_dev + (int64_t)p * B, st);
        }
    for (size_t i = 0; e == hipSuccess && i < M->steps.size(); ++i) {
        const cc_multi::Step& S = M->steps[i];
        const cc_plan* P = M->plans[(size_t)S.plan];
        const cc::Split& sp = P->splits[(size_t)S.split];
        const PIds ids{S.act, S.pas, S.out};
        if (cc::packed_kernel_split(sp)) {
            cc::StepParams h = packed_step_params(P, G, sp, ids, cpk, arena, L, partial, root_out, B);
            e = cc::launch_packed_split(h, G->n_cu, st, nullptr);
        } else {
            for (int32_t b = 0; e == hipSuccess && b < B; ++b) {
                cc::StepParams h = packed_one_params(P, G, sp, ids, colours_dev, arena, L, partial, root_out, B, b);
                e = cc::launch_split(h, G->n_cu, st, nullptr);
            }
        }
        if (e == hipSuccess && S.out == -2)
            e = cc::launch_reduce_packed(root_out, n, B, red, X_dev + (int64_t)S.plan * B, st);
    }
    if (e != hipSuccess) return hip_fail(e, "packed multi-template count launch");
    return CC_OK;
}

}  // extern "C"
