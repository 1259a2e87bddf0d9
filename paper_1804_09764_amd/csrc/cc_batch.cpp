// Instance batches (cc_batch_*): many (template, graph, colouring) instances in one persistent
// launch, or one launch per dependency level, each bit-identical to its plain count.
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

extern "C" {

cc_status cc_batch_create(int32_t n_inst, const cc_instance* inst, uint32_t flags, cc_batch** out) {
    if (!out) return fail(CC_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_inst < 0 || (n_inst > 0 && !inst)) return fail(CC_EINVAL, "bad instance array");
    cc_batch* B = new (std::nothrow) cc_batch();
    if (!B) return fail(CC_ENOMEM, "batch allocation failed");
    B->flags = flags;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    try {
        B->inst.resize((size_t)n_inst);
        std::vector<std::vector<int>> seg_of;  // per instance: final segment of each split
        std::vector<cc_batch::Seg> segs;
        for (int32_t i = 0; i < n_inst; ++i) {
            const cc_instance& in = inst[i];
            if (!in.plan || !in.graph || !in.X_dev || (in.graph->n > 0 && !in.colours_dev)) {
                delete B;
                return fail(CC_EINVAL, "instance " + std::to_string(i) + ": NULL plan, graph or buffer");
            }
            if (!in.plan->splits.empty() && !in.plan->dev) {
                delete B;
                return fail(CC_EINVAL, "instance " + std::to_string(i) + ": plan not bound to device memory");
            }
            const cc_plan* P = in.plan;
            const cc_graph* G = in.graph;
            if (B->n_cu == 0) B->n_cu = G->n_cu;
            cc_batch::Inst& I = B->inst[(size_t)i];
            I.in = in;
            const int64_t n_pad = pad32(G->n);
            I.arena_off = take((size_t)P->arena_cols * (size_t)n_pad * sizeof(double));
            I.partial_off = take((size_t)G->n_chunks * (size_t)P->max_stride_N * sizeof(double));
            I.root_off = in.vertex_dev ? 0 : take((size_t)std::max<int64_t>(G->n, 1) * sizeof(double));
            I.red_off = take(1024 * sizeof(double));
            B->max_red_blocks = std::max(B->max_red_blocks, cc::reduce_blocks_for(G->n));
            if (G->n == 0) continue;
            // segments of this instance in plan order, each waiting for the previous one: the
            // instance's splits share its table arena (first-fit reuse) and its chunk-partial
            // scratch, so a split may overwrite what an earlier split reads; running them in plan
            // order, as a plain count does, removes every such hazard. Instances run side by side.
            std::vector<int> last(P->splits.size(), -1);
            for (size_t j = 0; j < P->splits.size(); ++j) {
                const cc::Split& sp = P->splits[j];
                cc_batch::Seg a{};
                a.inst = i;
                a.split = (int)j;
                a.phase = 0;
                a.n_items = G->n_chunks + G->n_ranges;
                a.ndep = 0;
                a.level = 0;
                if (j > 0) {
                    const int d = last[j - 1];
                    a.dep[a.ndep++] = d;
                    a.level = segs[(size_t)d].level + 1;
                }
                segs.push_back(a);
                last[j] = (int)segs.size() - 1;
                if (G->n_hubs > 0) {
                    cc_batch::Seg h{};
                    h.inst = i;
                    h.split = (int)j;
                    h.phase = 1;
                    h.n_items = G->n_hubs;
                    h.ndep = 1;
                    h.dep[0] = last[j];
                    h.level = a.level + 1;
                    segs.push_back(h);
                    last[j] = (int)segs.size() - 1;
                }
                if (sp.p >= 2)
                    B->J = std::max(B->J, cc::pick_J(sp.Wp, G->cols_per_lane));
                B->lds_wave = std::max(B->lds_wave, cc::split_lds_wave(sp.Nw, sp.Wa, sp.a));
                // level mode launches each split's tasks with the kernel a plain count uses (all
                // variants give the same bits: the same order of terms, or for the 2-vertex table
                // exact integer sums); cut-row finishes run in variant 0
                const int var = cc::split_variant(sp.p, sp.Wp, G->cols_per_lane);
                const int base = cc::split_lds_wave(sp.Nw, sp.Wa, sp.a);
                for (size_t q = (size_t)(G->n_hubs > 0 ? last[j] - 1 : last[j]); q <= (size_t)last[j]; ++q) {
                    segs[q].variant = segs[q].phase == 0 ? var : 0;
                    segs[q].lds_wave = base + (segs[q].phase == 0 ? cc::variant_stage(var) : 0);
                }
            }
        }
        // instance-major order (as built) for the persistent launch; level order for the
        // level-by-level launches (stable: instance, split, phase within a level)
        B->segs = segs;
        B->ranges.assign((size_t)n_inst, cc::SegRange{0, 0});
        for (size_t q = 0; q < segs.size(); ++q) {
            cc::SegRange& r = B->ranges[(size_t)segs[q].inst];
            if (r.count == 0) r.first = (int32_t)q;
            r.count++;
        }
        B->level_order.resize(segs.size());
        for (size_t q = 0; q < segs.size(); ++q) B->level_order[q] = (int)q;
        std::stable_sort(B->level_order.begin(), B->level_order.end(), [&](int x, int y) {
            const cc_batch::Seg &a = segs[(size_t)x], &b = segs[(size_t)y];
            return a.level != b.level ? a.level < b.level : a.variant < b.variant;
        });
        B->groups.clear();
        int64_t item = 0;
        for (size_t q = 0; q < B->level_order.size(); ++q) {
            const cc_batch::Seg& sg = segs[(size_t)B->level_order[q]];
            if (B->groups.empty() || segs[(size_t)B->level_order[(size_t)B->groups.back().seg_lo]].level != sg.level ||
                B->groups.back().variant != sg.variant)
                B->groups.push_back(cc_batch::Group{(int)q, (int)q, sg.variant, 16, item, item});
            cc_batch::Group& g = B->groups.back();
            g.seg_hi = (int)q + 1;
            g.item_hi = item + sg.n_items;
            g.lds_wave = std::max(g.lds_wave, sg.lds_wave);
            item += sg.n_items;
        }
        if (B->lds_wave == 0) B->lds_wave = 16;
        const size_t nseg = std::max<size_t>(B->segs.size(), 1);
        B->seg_off = take(nseg * sizeof(cc::SegDesc));
        B->seg_level_off = take(nseg * sizeof(cc::SegDesc));
        B->range_off = take(std::max<size_t>((size_t)n_inst, 1) * sizeof(cc::SegRange));
        B->rd_off = take(std::max<size_t>((size_t)n_inst, 1) * sizeof(cc::ReduceDesc));
        B->total = off;
        B->seg_host.resize(B->segs.size());
        B->seg_level_host.resize(B->segs.size());
        B->rd_host.resize((size_t)n_inst);
    } catch (const std::bad_alloc&) {
        delete B;
        return fail(CC_ENOMEM, "host allocation failed while preparing the batch");
    }
    *out = B;
    return CC_OK;
}

cc_status cc_batch_workspace_bytes(const cc_batch* B, size_t* bytes) {
    if (!B || !bytes) return fail(CC_EINVAL, "NULL argument");
    *bytes = B->total;
    return CC_OK;
}

cc_status cc_batch_run(cc_batch* B, void* ws_dev, size_t ws_bytes, void* stream) {
    if (!B || (!ws_dev && B->total > 0)) return fail(CC_EINVAL, "NULL argument");
    if (ws_bytes < B->total) return fail(CC_ENOSPC, "batch workspace too small");
    if (B->inst.empty()) return CC_OK;
    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)ws_dev;
    cc::SegDesc* seg_dev = (cc::SegDesc*)(ws + B->seg_off);
    cc::SegDesc* seg_level_dev = (cc::SegDesc*)(ws + B->seg_level_off);
    cc::SegRange* range_dev = (cc::SegRange*)(ws + B->range_off);
    cc::ReduceDesc* rd_dev = (cc::ReduceDesc*)(ws + B->rd_off);
    for (size_t q = 0; q < B->segs.size(); ++q) {
        const cc_batch::Seg& sg = B->segs[q];
        const cc_batch::Inst& I = B->inst[(size_t)sg.inst];
        const cc_plan* P = I.in.plan;
        const cc_graph* G = I.in.graph;
        double* root_out = I.in.vertex_dev ? I.in.vertex_dev : (double*)(ws + I.root_off);
        cc::SegDesc& D = B->seg_host[q];
        D = cc::SegDesc{};
        D.S = step_params(P, G, P->splits[(size_t)sg.split], I.in.colours_dev, (double*)(ws + I.arena_off),
                          pad32(G->n), (double*)(ws + I.partial_off), root_out);
        D.item_start = 0;
        D.n_items = sg.n_items;
        D.phase = sg.phase;
    }
    int64_t item = 0;
    for (size_t q = 0; q < B->level_order.size(); ++q) {
        cc::SegDesc& D = B->seg_level_host[q];
        D = B->seg_host[(size_t)B->level_order[q]];
        D.item_start = item;
        D.S.stage_off = cc::split_lds_wave(D.S.Nw, D.S.Wa, D.S.a);  // narrow stage after N and A rows
        item += D.n_items;
    }
    for (size_t i = 0; i < B->inst.size(); ++i) {
        const cc_batch::Inst& I = B->inst[i];
        cc::ReduceDesc& R = B->rd_host[i];
        R.x = I.in.vertex_dev ? I.in.vertex_dev : (const double*)(ws + I.root_off);
        R.n = I.in.graph->n;
        R.out = I.in.X_dev;
        R.partial = (double*)(ws + I.red_off);
    }
    const bool levels = (B->flags & CC_BATCH_LEVELS) != 0;
    hipError_t e = hipSuccess;
    if (!B->segs.empty()) {
        if (levels)
            e = hipMemcpyAsync(seg_level_dev, B->seg_level_host.data(), B->seg_level_host.size() * sizeof(cc::SegDesc),
                               hipMemcpyHostToDevice, st);
        else
            e = hipMemcpyAsync(seg_dev, B->seg_host.data(), B->seg_host.size() * sizeof(cc::SegDesc),
                               hipMemcpyHostToDevice, st);
        if (e == hipSuccess && !levels)
            e = hipMemcpyAsync(range_dev, B->ranges.data(), B->ranges.size() * sizeof(cc::SegRange),
                               hipMemcpyHostToDevice, st);
    }
    if (e == hipSuccess)
        e = hipMemcpyAsync(rd_dev, B->rd_host.data(), B->rd_host.size() * sizeof(cc::ReduceDesc), hipMemcpyHostToDevice, st);
    // instances without splits (k = 1): every vertex roots one map
    for (size_t i = 0; e == hipSuccess && i < B->inst.size(); ++i) {
        const cc_batch::Inst& I = B->inst[i];
        if (I.in.graph->n > 0 && I.in.plan->splits.empty())
            e = cc::launch_fill_f64(const_cast<double*>(B->rd_host[i].x), I.in.graph->n, 1.0, st);
    }
    if (e == hipSuccess && !B->segs.empty()) {
        if (levels) {
            for (size_t l = 0; e == hipSuccess && l < B->groups.size(); ++l) {
                const cc_batch::Group& g = B->groups[l];
                e = cc::launch_batch_level(seg_level_dev, g.seg_lo, g.seg_hi, g.item_lo, g.item_hi, g.variant, g.lds_wave,
                                           B->n_cu, st);
            }
        } else {
            e = cc::launch_batch_inst(seg_dev, range_dev, (int)B->inst.size(), B->J, B->lds_wave, B->n_cu,
                                      (int)((B->flags >> 8) & 0xFFu), st);
        }
    }
    for (size_t i = 0; e == hipSuccess && i < B->inst.size(); ++i)
        if (B->inst[i].in.graph->n == 0) e = cc::launch_fill_f64(B->inst[i].in.X_dev, 1, 0.0, st);
    if (e == hipSuccess) e = cc::launch_reduce_batch(rd_dev, (int)B->inst.size(), B->max_red_blocks, st);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return CC_OK;
}

cc_status cc_batch_check(cc_batch* B, void* stream) {
    if (!B) return fail(CC_EINVAL, "NULL batch");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "batch check");
    return CC_OK;
}

void cc_batch_destroy(cc_batch* B) { delete B; }

}  // extern "C"
