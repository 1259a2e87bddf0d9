// Host helpers shared by the C ABI's source files (cc_api.cpp, cc_multi.cpp, cc_batch.cpp).
#pragma once

#include <hip/hip_runtime_api.h>

#include <string>
#include <vector>

#include "cc_internal.h"

namespace cc {
namespace host {

extern thread_local std::string g_err;  // cc_last_error()

cc_status fail(cc_status st, const std::string& msg);
cc_status hip_fail(hipError_t e, const char* what);

inline size_t align256(size_t x) { return (x + 255) / 256 * 256; }
inline int64_t pad32(int64_t n) { return (n + 31) / 32 * 32; }

// workspace of a packed count with B colourings per row
struct PackedLayout {
    size_t arena_off, partial_off, root_off, colour_off, red_off, total;
    int64_t n_pad, nstride;
    std::vector<int64_t> col_off;  // per table, in columns of n_pad doubles
    std::vector<int64_t> stride;   // per table: doubles between consecutive vertices
    std::vector<int64_t> bstep;    // per table: doubles between consecutive colourings
};

PackedLayout packed_layout(const cc_plan* P, const cc_graph* G, int32_t B);

// the tables of one split in a packed layout: ids into PackedLayout (-1: a single vertex; out -2:
// the template's root counts)
struct PIds {
    int act, pas, out;
};

inline PIds own_ids(const cc::Split& sp) { return PIds{sp.act, sp.pas, sp.out}; }

// a split's arguments without its table pointers; with the plain plan's tables; with packed tables
cc::StepParams base_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, const uint8_t* colour,
                           double* partial, double* root_out);
cc::StepParams step_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, const uint8_t* colour,
                           double* arena, int64_t n_pad, double* partial, double* root_out);
cc::StepParams packed_step_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, PIds t,
                                  const uint8_t* colour, double* arena, const PackedLayout& L, double* partial,
                                  double* root_out, int32_t B);
cc::StepParams packed_one_params(const cc_plan* P, const cc_graph* G, const cc::Split& sp, PIds t,
                                 const uint8_t* colours_bn, double* arena, const PackedLayout& L, double* partial,
                                 double* root_out, int32_t B, int32_t b);
bool packed_fits(const cc_plan* P, int32_t B);

}  // namespace host
}  // namespace cc
