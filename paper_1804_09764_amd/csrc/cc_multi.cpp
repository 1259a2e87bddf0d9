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

// dependency level of every step: 0 for splits of single vertices, else one more than the
// deepest step producing one of its inputs (steps are listed producers first)
std::vector<int> step_levels(const cc_multi* M) {
    std::vector<int> producer(M->table_W.size(), -1), lv(M->steps.size(), 0);
    for (size_t i = 0; i < M->steps.size(); ++i) {
        const cc_multi::Step& st = M->steps[i];
        int l = 0;
        if (st.act >= 0) l = std::max(l, lv[(size_t)producer[(size_t)st.act]] + 1);
        if (st.pas >= 0) l = std::max(l, lv[(size_t)producer[(size_t)st.pas]] + 1);
        lv[i] = l;
        if (st.out >= 0) producer[(size_t)st.out] = (int)i;
    }
    return lv;
}

// Workspace of the persistent launch. Tables are placed level by level: the outputs of a level
// are allocated together (first fit) and a table is released only after the level of its last
// reader, since the splits of one level run at the same time. Each split of a level has its own
// chunk-partial slot, each template its own root rows.
struct OneLaunch {
    PackedLayout L;
    std::vector<int> level, slot;
    int n_levels = 0, slots = 1, waves = 4, JP = 1;
    size_t tab_doubles = 0, lds_wave = 0;
    int64_t n_blocks = 0;
    size_t seg_off = 0, block_off = 0, phase_off = 0, bar_off = 0, total = 0;
};

cc::StepParams tile_only_params(const cc_plan* P, const cc::Split& sp, const cc_graph* G, int32_t B, int force_J) {
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
    h.tile_doubles = G->packed_tile;
    h.force_J = force_J;
    cc::packed_tile(&h);
    return h;
}

// tile elements per lane of the persistent launch's p >= 2 variant: the most any split needs
int persistent_JP(const cc_multi* M, const cc_graph* G, int32_t B) {
    int JP = 1;
    for (const auto& st : M->steps) {
        const cc_plan* P = M->plans[(size_t)st.plan];
        const cc::Split& sp = P->splits[(size_t)st.split];
        if (sp.p >= 2) JP = std::max(JP, tile_only_params(P, sp, G, B, 0).pJ);
    }
    return JP;
}

OneLaunch one_launch_layout(const cc_multi* M, const cc_graph* G, int32_t B) {
    OneLaunch O;
    PackedLayout& L = O.L;
    L.n_pad = pad32(G->n);
    O.JP = persistent_JP(M, G, B);
    const size_t nt = M->table_W.size();
    L.col_off.assign(nt, 0);
    L.stride.resize(nt);
    L.bstep.resize(nt);
    for (size_t t = 0; t < nt; ++t) {
        const int64_t W = M->table_W[t];
        L.stride[t] = cc::packed_wide(W) ? cc::packed_stride(W) : cc::packed_stride((int64_t)B * W);
        L.bstep[t] = cc::packed_wide(W) ? L.n_pad * cc::packed_stride(W) : W;
    }
    O.level = step_levels(M);
    for (int l : O.level) O.n_levels = std::max(O.n_levels, l + 1);
    std::vector<int> last_level(nt, -1);
    for (size_t i = 0; i < M->steps.size(); ++i) {
        const cc_multi::Step& st = M->steps[i];
        if (st.act >= 0) last_level[(size_t)st.act] = std::max(last_level[(size_t)st.act], O.level[i]);
        if (st.pas >= 0) last_level[(size_t)st.pas] = std::max(last_level[(size_t)st.pas], O.level[i]);
    }
    std::vector<std::pair<int64_t, int64_t>> used;  // (column offset, columns) of live tables
    int64_t peak = 0, nst = 1;
    O.slot.assign(M->steps.size(), 0);
    std::vector<int> per_level((size_t)O.n_levels, 0);
    for (int lv = 0; lv < O.n_levels; ++lv) {
        for (size_t i = 0; i < M->steps.size(); ++i) {
            if (O.level[i] != lv) continue;
            const cc_multi::Step& st = M->steps[i];
            const cc_plan* P = M->plans[(size_t)st.plan];
            const cc::Split& sp = P->splits[(size_t)st.split];
            nst = std::max(nst, cc::packed_stride((int64_t)B * sp.Cf));
            O.slot[i] = per_level[(size_t)lv]++;
            const cc::StepParams h = tile_only_params(P, sp, G, B, sp.p >= 2 ? O.JP : 0);
            O.tab_doubles = std::max(O.tab_doubles, (size_t)h.tab_doubles);
            O.lds_wave = std::max(O.lds_wave, (size_t)h.lds_wave);
            if (st.out < 0) continue;
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
        for (size_t g = 0; g < nt; ++g)
            if (last_level[g] == lv)
                for (size_t i = 0; i < used.size(); ++i)
                    if (used[i].first == L.col_off[g]) {
                        used.erase(used.begin() + (long)i);
                        break;
                    }
    }
    for (int c : per_level) O.slots = std::max(O.slots, c);
    while (O.waves > 1 && (O.tab_doubles + O.lds_wave * (size_t)O.waves) * sizeof(double) > 64 * 1024) O.waves >>= 1;
    const int64_t tasks = G->n_chunks + G->n_ranges;
    for (size_t i = 0; i < M->steps.size(); ++i) {
        const cc_multi::Step& st = M->steps[i];
        const cc_plan* P = M->plans[(size_t)st.plan];
        const cc::Split& sp = P->splits[(size_t)st.split];
        const cc::StepParams h = tile_only_params(P, sp, G, B, sp.p >= 2 ? O.JP : 0);
        const int64_t tiles = (B + h.bt - 1) / h.bt;
        O.n_blocks += (tasks * tiles + O.waves - 1) / O.waves + (G->n_hubs * tiles + O.waves - 1) / O.waves;
    }
    const int64_t np = (int64_t)M->plans.size();
    L.nstride = nst;
    L.arena_off = 0;
    L.partial_off = align256((size_t)peak * (size_t)L.n_pad * sizeof(double));
    L.root_off = align256(L.partial_off + (size_t)O.slots * (size_t)G->n_chunks * (size_t)nst * sizeof(double));
    L.colour_off = align256(L.root_off + (size_t)np * (size_t)std::max<int64_t>(G->n, 1) * (size_t)B * sizeof(double));
    L.red_off = align256(L.colour_off + (size_t)std::max<int64_t>(G->n, 1) * (size_t)B);
    O.seg_off = align256(L.red_off + (size_t)cc::packed_reduce_blocks(G->n) * (size_t)B * sizeof(double));
    O.block_off = align256(O.seg_off + M->steps.size() * sizeof(cc::PSeg));
    O.phase_off = align256(O.block_off + (size_t)O.n_blocks * sizeof(cc::PItemBlock));
    O.bar_off = align256(O.phase_off + (size_t)(2 * O.n_levels) * sizeof(cc::PPhase));
    // barrier count, generation, error flag, then one item-block counter per phase
    O.total = align256(O.bar_off + (size_t)(3 + 2 * O.n_levels) * sizeof(unsigned));
    L.total = O.total;
    return O;
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

extern "C" {

cc_status cc_count_packed_multi_persistent_workspace_bytes(const cc_multi* M, const cc_graph* G, int32_t B,
                                                           size_t* bytes) {
    if (!M || !G || !bytes) return fail(CC_EINVAL, "NULL argument");
    if (B < 1 || B > CC_MAX_PACKED) return fail(CC_ERANGE, "B must be in [1, CC_MAX_PACKED]");
    *bytes = one_launch_layout(M, G, B).total;
    return CC_OK;
}

cc_status cc_count_packed_multi_persistent(const cc_multi* M, const cc_graph* G, const uint8_t* colours_dev,
                                           int32_t B, void* ws_dev, size_t ws_bytes, double* X_dev, void* stream) {
    if (!M || !G) return fail(CC_EINVAL, "NULL multi or graph");
    if (B < 1 || B > CC_MAX_PACKED) return fail(CC_ERANGE, "B must be in [1, CC_MAX_PACKED]");
    if (!X_dev || !ws_dev || (G->n > 0 && !colours_dev)) return fail(CC_EINVAL, "NULL buffer");
    for (const cc_plan* P : M->plans) {
        if (!P->splits.empty() && !P->dev) return fail(CC_EINVAL, "plan not bound to device memory");
        if (!packed_fits(P, B)) return fail(CC_ERANGE, "template too large for the packed layout (use cc_count)");
        for (const auto& sp : P->splits)
            if (!cc::packed_kernel_split(sp))
                return fail(CC_ERANGE, "a split's rows exceed 64 entries per colouring: use cc_count_packed_multi");
    }
    const OneLaunch O = one_launch_layout(M, G, B);
    if (ws_bytes < O.total) return fail(CC_ENOSPC, "count workspace too small");
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
    const PackedLayout& L = O.L;
    double* arena = (double*)(ws + L.arena_off);
    double* partial = (double*)(ws + L.partial_off);
    double* roots = (double*)(ws + L.root_off);
    uint8_t* cpk = ws + L.colour_off;
    double* red = (double*)(ws + L.red_off);
    cc::PSeg* seg_dev = (cc::PSeg*)(ws + O.seg_off);
    cc::PItemBlock* block_dev = (cc::PItemBlock*)(ws + O.block_off);
    cc::PPhase* phase_dev = (cc::PPhase*)(ws + O.phase_off);
    unsigned* bar = (unsigned*)(ws + O.bar_off);
    const size_t root_rows = (size_t)n * (size_t)B;
    try {
        M->pseg_host.assign(M->steps.size(), cc::PSeg{});
        for (size_t i = 0; i < M->steps.size(); ++i) {
            const cc_multi::Step& S = M->steps[i];
            const cc_plan* P = M->plans[(size_t)S.plan];
            const cc::Split& sp = P->splits[(size_t)S.split];
            double* part = partial + (size_t)O.slot[i] * (size_t)G->n_chunks * (size_t)L.nstride;
            cc::StepParams h = packed_step_params(P, G, sp, PIds{S.act, S.pas, S.out}, cpk, arena, L, part,
                                                  roots + (size_t)S.plan * root_rows, B);
            h.force_J = sp.p >= 2 ? O.JP : 0;
            cc::packed_tile(&h);
            h.lds_wave = (int)O.lds_wave;  // every wavefront's slice has the widest split's size
            M->pseg_host[i].S = h;
            M->pseg_host[i].p1 = sp.p == 1 ? 1 : 0;
        }
        M->pblock_host.clear();
        M->pphase_host.clear();
        const int64_t tasks = G->n_chunks + G->n_ranges;
        for (int lv = 0; lv < O.n_levels; ++lv) {
            for (int phase = 0; phase < 2; ++phase) {
                cc::PPhase ph{(int64_t)M->pblock_host.size(), 0};
                for (size_t i = 0; i < M->steps.size(); ++i) {
                    if (O.level[i] != lv) continue;
                    // items: (task or cut row, colouring tile) pairs
                    const cc::StepParams& h = M->pseg_host[i].S;
                    const int64_t items = (phase == 0 ? tasks : G->n_hubs) * (int64_t)((h.B + h.bt - 1) / h.bt);
                    for (int64_t f = 0; f < items; f += O.waves)
                        M->pblock_host.push_back(
                            cc::PItemBlock{(int32_t)i, (int32_t)std::min<int64_t>(O.waves, items - f), f});
                }
                ph.n_blocks = (int64_t)M->pblock_host.size() - ph.first_block;
                M->pphase_host.push_back(ph);
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(CC_ENOMEM, "host allocation failed");
    }
    if ((int64_t)M->pblock_host.size() > O.n_blocks) return fail(CC_EINTERNAL, "item blocks exceed the layout");
    e = cc::launch_transpose_colours(colours_dev, n, B, cpk, st);
    if (e == hipSuccess && M->k == 1) {
        // single-vertex templates: every vertex roots one map
        for (int32_t p = 0; e == hipSuccess && p < np; ++p) {
            e = cc::launch_fill_f64(roots + (size_t)p * root_rows, n * B, 1.0, st);
            if (e == hipSuccess)
                e = cc::launch_reduce_packed(roots + (size_t)p * root_rows, n, B, red, X_dev + (int64_t)p * B, st);
        }
        if (e != hipSuccess) return hip_fail(e, "packed single-vertex count");
        return CC_OK;
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(seg_dev, M->pseg_host.data(), M->pseg_host.size() * sizeof(cc::PSeg), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(block_dev, M->pblock_host.data(), M->pblock_host.size() * sizeof(cc::PItemBlock),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(phase_dev, M->pphase_host.data(), M->pphase_host.size() * sizeof(cc::PPhase),
                           hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = cc::launch_fill_u32(bar, 3 + (int64_t)M->pphase_host.size(), 0u, st);
    if (e == hipSuccess)
        e = cc::launch_packed_persistent(seg_dev, block_dev, M->pphase_host.data(), phase_dev,
                                         (int)M->pphase_host.size(), O.waves, O.JP, O.tab_doubles, O.lds_wave, bar,
                                         G->n_cu, st);
    for (int32_t p = 0; e == hipSuccess && p < np; ++p)
        e = cc::launch_reduce_packed(roots + (size_t)p * root_rows, n, B, red, X_dev + (int64_t)p * B, st);
    if (e == hipSuccess) e = cc::launch_poison_if(bar + 2, X_dev, (int64_t)np * B, st);
    if (e != hipSuccess) return hip_fail(e, "persistent packed multi-template count");
    return CC_OK;
}

}  // extern "C"
