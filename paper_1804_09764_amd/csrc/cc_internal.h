// Internal declarations shared by the planner, the host API and the kernels of libcc.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/cc.h"

namespace cc {

constexpr int kMaxK = CC_MAX_K;
constexpr int kWave = 64;             // CDNA wavefront width
constexpr uint16_t kNoSlot = 0xFFFF;  // fold map: this passive entry does not reach v

int64_t binom(int n, int r);

// One cut of a sub-template T_i (size s) into the active part T_i' (size a, keeps the root) and
// the passive part T_i'' (size p, rooted at the cut child). Table widths are per vertex, in the
// colour-anchored layout: a table for a sub-template of size t stores, for vertex v, the counts of
// the colour sets S with col(v) in S, one entry per S \ {col(v)} over the k-1 other colours
// (re-numbered 0..k-2), in the storage order entry_order gives for sets of t-1 colours (colex
// order for rows of up to 16 entries). Its width is W(t) = C(k-1, t-1).
struct Split {
    int s, a, p;
    int act;        // table id of T_i' (-1: a single vertex, count 1 for its own colour)
    int pas;        // table id of T_i'' (-1: a single vertex)
    int out;        // table id of T_i (-2: the full template, one value per vertex)
    int Wa, Wp, Ws; // anchored widths of T_i', T_i'', T_i
    int Nw;         // width of the neighbour sum N(v, Q), |Q| = p, Q over the k-1 other colours
    int npairs;     // C(s-1, p): splits of one output set
    int64_t split_off;  // byte offset of the pair list in the device constants (a = 1: N entry of
                        // each output position)
    int64_t fold_off;   // byte offset of the fold map in the device constants (-1 if p == 1)
    int64_t mask_off;   // byte offset of the passive entries' colour-set masks (-1 if p == 1)
    // packed layout (several colourings per row): neighbour sums are kept over all k colours,
    // C(k, p) entries per colouring
    int Cf;             // C(k, p)
    int64_t full_off;   // byte offset of FM[cu][j]: full-space rank of passive entry j (-1 if p == 1)
    int64_t emap_off;   // byte offset of E[cv][q]: full-space rank of N entry q written without cv
    // projected passive rows (wide passive rows, p >= 2 and Wp > 64): for a centre colour cv the
    // entries of a neighbour's row whose set avoids cv, C(k-2, p-1) = Wn of them, in colex order
    // of the set, copied into a contiguous row of Wn_pad doubles
    int Wn;               // C(k-2, p-1), 0 if the split has no projected form
    int Wn_pad;           // Wn rounded up to 16 doubles (whole 128-byte lines)
    double lines_need;    // expected 128-byte lines of a stored passive row that hold a needed entry
    int64_t proj_src_off;   // byte offset of S[cu][cv][j]: storage position in u's row of projected entry j
    int64_t proj_fold_off;  // byte offset of F[cu][cv][j]: N entry of projected entry j
    int64_t proj_mask_off;  // byte offset of Wn zero masks (every projected entry is needed)
};

struct Table {
    int size;        // sub-template size t
    int W;           // C(k-1, t-1)
    std::string key; // canonical form of the rooted sub-template (equal keys: equal tables)
    int stride;      // row stride in doubles
    int64_t col_off; // offset in columns (1 column = n_pad doubles) inside the table arena
};

}  // namespace cc

struct cc_plan {
    int k = 0;
    int root = 0;
    std::vector<int32_t> edges;
    std::vector<cc::Split> splits;
    std::vector<cc::Table> tables;
    int64_t arena_cols = 0;   // peak columns of the table arena
    int max_Nw = 0;           // widest neighbour-sum row over splits
    int max_stride_N = 0;     // its padded stride
    std::vector<uint8_t> consts;  // device constants, host copy
    void* dev = nullptr;
    size_t dev_bytes = 0;
    double aut = 1.0;
    int64_t units_per_edge = 0;
    int64_t t3_memory = 0, t3_compute = 0;
    int64_t gather_per_edge = 0, combine_per_vertex = 0;
    int64_t peak_live_cols = 0;
    // measurement (cc_profile_*): event triples per (colouring, split); opaque hipEvent_t handles
    bool profiling = false;
    mutable std::vector<std::vector<void*>> prof_events;  // per split: start, mid, end, start, ...
    mutable std::vector<int64_t> prof_launches;
    ~cc_plan();
};

namespace cc {

// work items of a prepared graph
struct ChunkItem {
    int64_t beg;     // first CSR entry of the chunk
    int32_t v;       // row
    int32_t len;     // number of entries (<= chunk)
};

struct HubItem {
    int32_t v;
    int32_t n_chunks;
    int64_t first_chunk;
};

// storage order of a table row of m-sets over K colours: order[pos] = colex rank of the set at pos
std::vector<int> entry_order(int K, int m);

cc_status plan_build(int k, const int32_t* edges, int root, uint32_t flags, cc_plan* P,
                     std::string* err);

int pad_stride(int W);

// Tables of a packed count (B colourings). A narrow table (W <= 64 entries per colouring) is
// interleaved: row v holds the B entry blocks of v side by side, [v][b][W], row stride rounded up
// to 16 doubles. A wide table is colouring-major, [b][v][W rounded up to 16], i.e. B one-colouring
// tables one after another, which the one-colouring kernels read exactly as they read a plain
// table.
inline bool packed_wide(int64_t W) { return W > 64; }
inline int64_t packed_stride(int64_t W) { return (W + 15) / 16 * 16; }
inline int64_t packed_cols(int64_t W, int B) { return packed_wide(W) ? B * packed_stride(W) : packed_stride(B * W); }
// The plan's allocation sequence replayed with these table widths (in columns of n_pad doubles).
// Returns the arena width; col_off[t] per table.
int64_t packed_arena(const cc_plan* P, int B, std::vector<int64_t>* col_off);
// Splits of a packed count whose per-colouring rows are all narrow (<= 64 entries) run the packed
// kernels; wider ones run the one-colouring kernels once per colouring over the packed rows (a
// wide row already fills the wavefront). The choice depends on the split only, never on B.
inline bool packed_kernel_split(const Split& sp) {
    return (sp.p < 2 || sp.Wp <= 64) && sp.Wa <= 64 && sp.Ws <= 64;
}

// Arguments of one split over one graph and one colouring (shared by host and device code).
struct StepParams {
    const int64_t* row_ptr;
    const int32_t* col;
    const uint8_t* colour;       // colour of vertex u at colour[u * cstride]
    const uint8_t* ecol;         // NULL, or the colour of each CSR entry's vertex: ecol[e] = colour[col[e]]
    const int32_t* light;        // light rows, heaviest first
    const int32_t* light_start;  // light range r = light[light_start[r] .. light_start[r+1])
    const ChunkItem* chunks;
    const HubItem* hubs;
    int64_t n_light, n_ranges, n_chunks, n_hubs;
    const double* P;             // passive table (p >= 2)
    const double* A;             // active table (a >= 2)
    double* O;                   // output table, or the per-vertex root counts
    double* partial;             // chunk partial rows
    const uint16_t* fold;
    const uint32_t* split;
    const uint16_t* mask;        // colour set of each passive entry (over the neighbour's other colours)
    int64_t pstride, astride, ostride, nstride, cstride;
    int k, s, a, p, Wa, Wp, Ws, Nw, npairs;
    int lds_wave;       // doubles of LDS per wavefront
    int a_off;          // offset of the staged active row inside the wavefront's LDS slice
    int stage_a;        // 1: the combine stages the active row in LDS; 0: reads it from HBM
    int stage_off;      // offset of the narrow-row stage inside the wavefront's LDS slice
    int waves_per_block;
    int cols_per_lane;  // 0 = choose from Wp
    // packed layout: B colourings per row, row v = [b][entry] (entry block of colouring b at
    // b * W); colour points to the colours as [v][b]. B == 0 selects the one-colouring layout.
    int B;
    int bt;             // colourings per tile of a row (<= 64)
    int tile_doubles;   // doubles of a tile row per neighbour (0: 256 when p >= 2, 512 when p = 1)
    int force_J;        // tile elements per lane per pass (0: the smallest that covers a tile row)
    int Cf;             // C(k, p): neighbour-sum entries per colouring, over all k colours
    int tab_u16;        // entries of the block-shared maps at the start of LDS: FM (k * Wp) then E (k * Nw)
    int tab_doubles;    // their size in doubles (rounded up)
    int pJ;             // tile elements per lane per pass (1, 2, 4, 8)
    int tg_off;         // offset of the per-lane target table (pJ * k * 64 int16) in a wavefront's slice
    int cs_off;         // offset of the colour stage of a CSR block (64 * bt bytes)
    const uint16_t* fullmap;  // FM[cu][j] (p >= 2)
    const uint16_t* emap;     // E[cv][q]
    // centre colours this launch processes: bit c for colour c < k, bit kAnyInvalid for the rows
    // whose colour is not below k (they only write zeros); all bits set outside projected passes
    uint32_t cls_mask;
    // projected passes: the passive row of a neighbour for a centre of colour cv starts at
    // P + slot(cv) * class_stride, slot(cv) = number of colours below cv in cls_mask; 0 otherwise
    int64_t class_stride;
};

constexpr uint32_t kAnyInvalid = 1u << 16;
constexpr uint32_t kAllClasses = 0x1FFFFu;

// LDS layout of one split: N row (padded), then the active row when a >= 2 and both rows fit in
// 16 KB per wavefront; wider active rows are read from HBM by the combine, which keeps the
// wavefronts' LDS slices small enough for several to share a CU
inline bool split_stage_a(int Nw, int Wa, int a) { return a >= 2 && pad_stride(Nw) + pad_stride(Wa) <= 2048; }
inline int split_a_off(int Nw) { return pad_stride(Nw); }
inline int split_lds_wave(int Nw, int Wa, int a) { return pad_stride(Nw) + (split_stage_a(Nw, Wa, a) ? pad_stride(Wa) : 0); }

// One segment of a batched launch: all work items of one phase of one split of one instance.
// phase 0 = the split's tasks (chunks + light ranges), phase 1 = its cut-row finishes.
struct SegDesc {
    StepParams S;
    int64_t item_start;  // first global item of the segment
    int64_t n_items;
    int32_t phase;
    int32_t ndep;
    int32_t dep[2];      // segments that must be complete first
    uint32_t need[2];    // their item counts
};

// the segments of one instance in a batch: segs[first .. first + count)
struct SegRange {
    int32_t first;
    int32_t count;
};

// One persistent launch of a multi-template packed count: the splits that run, grouped by
// dependency level (a split's inputs come from earlier levels only). Each level has a task phase
// (chunks of cut rows and light rows of every split of the level) and a cut-row finish phase;
// a device-wide barrier separates consecutive phases. Work is dealt in item blocks: up to one
// workgroup's worth of consecutive items of one split.
struct PSeg {
    StepParams S;        // packed arguments of the split (tile, maps, tables, scratch)
    int32_t p1;          // 1 when the passive part is a single vertex (colour counts)
    int32_t pad;
};

struct PItemBlock {
    int32_t seg;         // index into the PSeg array
    int32_t count;       // items in the block (<= waves per workgroup)
    int64_t first;       // first item: a task (phase 0) or a cut row (phase 1) of the split
};

struct PPhase {
    int64_t first_block; // item blocks [first_block, first_block + n_blocks) of the phase
    int64_t n_blocks;
};

// per-instance root reduction of a batch
struct ReduceDesc {
    const double* x;
    int64_t n;
    double* out;
    double* partial;  // reduce_blocks_for(n) slots
};

}  // namespace cc

#include <hip/hip_runtime_api.h>
namespace cc {
hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t st);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st);
// ecol[e] = colour[col[e]] for the nnz CSR entries (one colouring, colour stride 1)
hipError_t launch_edge_colours(const int32_t* col, const uint8_t* colour, int64_t nnz, uint8_t* ecol, hipStream_t st);
hipError_t launch_colour(uint64_t seed, uint64_t first_iter, int64_t n, int k, int B, uint8_t* out,
                         hipStream_t st);
// root sums: blocks of kReducePerBlock values (at most 1024 blocks), then one final block; the
// batched root sums use the same layout so that their totals equal a plain count's bit for bit
constexpr int64_t kReducePerBlock = 8192;
int reduce_blocks_for(int64_t n);
hipError_t launch_reduce(const double* x, int64_t n, double* partial, double* out, hipStream_t st);
hipError_t launch_validate(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz,
                           unsigned* flags, hipStream_t st);
// mid (optional) is recorded between the gather kernel and the cut-row finish kernel
hipError_t launch_split(StepParams S, int n_cu, hipStream_t st, hipEvent_t mid);
// the two halves of launch_split: the task kernel (chunks of cut rows and light rows whose centre
// colour is in S.cls_mask) and the cut-row finish (every cut row)
hipError_t launch_split_tasks(StepParams S, int n_cu, hipStream_t st);
hipError_t launch_hub_finish(StepParams S, int n_cu, hipStream_t st);
// projected passive rows for the centre colours in cls_mask (bit c: colour c; at most one
// projected row per (vertex, colour)): out + slot(c) * class_stride + u * qstride holds the Wn
// entries src[(col(u) * k + c) * Wn + j] of P's row u (W entries), for every u whose colour is
// below k and other than c
hipError_t launch_project(const double* P, int64_t pstride, int W, const uint8_t* colour, int64_t n, int k,
                          const uint16_t* src, int Wn, int64_t qstride, int64_t class_stride, uint32_t cls_mask,
                          double* out, hipStream_t st);
// kernel variant of a split (general path with 1/2/4/8 doubles per lane = 0..3, or narrow rows
// with 16/32 lanes per row = 4/5) and the LDS stage per wavefront a narrow variant adds
int split_variant(int p, int Wp, int cols_per_lane);
int variant_stage(int variant);
// batched launches: one persistent launch with instances owned by workgroups (segments of an
// instance contiguous, in plan order; inst_dev[i] = {first segment, count}), or one launch per
// (dependency level, variant) group: level-ordered segments [seg_lo, seg_hi), items [item_lo, item_hi)
hipError_t launch_batch_inst(const SegDesc* segs_dev, const SegRange* inst_dev, int n_inst, int J, int lds_wave, int n_cu,
                             int share, hipStream_t st);
hipError_t launch_batch_level(const SegDesc* segs_dev, int seg_lo, int seg_hi, int64_t item_lo, int64_t item_hi,
                              int variant, int lds_wave, int n_cu, hipStream_t st);
hipError_t launch_reduce_batch(const ReduceDesc* rd_dev, int n_inst, int max_blocks, hipStream_t st);
int pick_J(int Wp, int want);
// packed layout: tile choice and LDS size of one split (host), the split launch, the [B][n] ->
// [n][B] colour transpose and the per-colouring root sums of a [n][B] table
void packed_tile(StepParams* S);
size_t packed_lds_bytes(const StepParams& S, int waves);
hipError_t launch_packed_split(StepParams S, int n_cu, hipStream_t st, hipEvent_t mid);
hipError_t launch_transpose_colours(const uint8_t* in, int64_t n, int B, uint8_t* out, hipStream_t st);
int packed_reduce_blocks(int64_t n);
hipError_t launch_reduce_packed(const double* x, int64_t n, int B, double* partial, double* out, hipStream_t st);
// the persistent multi-template launch: phases[0 .. n_phases) in order over the item blocks, all of
// whose splits run the packed kernels; bar = 3 + n_phases zeroed unsigned (barrier count,
// generation, error flag, one item-block counter per phase), lds = dynamic LDS bytes for `waves` wavefronts per workgroup (the widest split's maps and
// slices). Returns hipErrorCooperativeLaunchTooLarge when the grid cannot be co-resident.
// Every split with p >= 2 takes JP tile elements per lane per pass (StepParams.force_J), so that
// the kernel holds one gather variant; a split with p = 1 keeps its own (StepParams.pJ), the colour
// count variants being small.
hipError_t launch_packed_persistent(const PSeg* segs, const PItemBlock* blocks, const PPhase* phases_host,
                                    const PPhase* phases_dev, int n_phases, int waves, int JP, size_t tab_doubles,
                                    size_t lds_wave, unsigned* bar, int n_cu, hipStream_t st);
// X[0 .. n) = NaN when *flag != 0 (queued after the root sums of a persistent launch)
hipError_t launch_poison_if(const unsigned* flag, double* X, int64_t n, hipStream_t st);
}  // namespace cc

struct cc_graph {
    int64_t n = 0, nnz = 0, max_degree = 0;
    const int64_t* row_ptr = nullptr;
    const int32_t* col = nullptr;
    int32_t* light = nullptr;        // device: light rows, heaviest first
    int32_t* light_start = nullptr;  // device: n_ranges + 1 starts of light ranges
    cc::ChunkItem* chunks = nullptr; // device
    cc::HubItem* hubs = nullptr;     // device
    int64_t n_light = 0, n_ranges = 0, n_chunks = 0, n_hubs = 0;
    int32_t hub_threshold = 0, chunk = 0;
    int32_t cols_per_lane = 0;
    int32_t proj_classes = 0;  // cc_tuning.proj_classes
    int32_t packed_tile = 0;   // cc_tuning.packed_tile
    int device = 0;
    int n_cu = 0;
};

// Several templates of one size counted together with packed rows; tables of equal rooted
// sub-templates (equal canonical keys) are computed once and shared.
struct cc_multi {
    int k = 0;
    std::vector<const cc_plan*> plans;
    struct Step {
        int plan, split;       // the split that runs (plan index, split index in that plan)
        int act, pas, out;     // global table ids (-1: a single vertex; out -2: the plan's root counts)
        std::vector<int> release;  // global tables whose last use is this step
    };
    std::vector<Step> steps;
    std::vector<int> table_W;  // per global table: entries per colouring
    int64_t n_splits = 0;      // splits of all plans together (before sharing)
    // host copies of the persistent launch's descriptors (kept alive while the asynchronous
    // uploads of the last call are in flight)
    mutable std::vector<cc::PSeg> pseg_host;
    mutable std::vector<cc::PItemBlock> pblock_host;
    mutable std::vector<cc::PPhase> pphase_host;
};

struct cc_batch {
    struct Inst {
        cc_instance in;
        size_t arena_off, partial_off, root_off, red_off;
    };
    struct Seg {
        int inst, split, phase, level, variant, lds_wave;
        int64_t n_items;
        int dep[2];
        int ndep;
    };
    std::vector<Inst> inst;
    std::vector<Seg> segs;             // instance-major, plan order within an instance
    std::vector<cc::SegRange> ranges;  // per instance: its segments in `segs`
    std::vector<int> level_order;      // segment ids ordered by (dependency level, kernel variant)
    struct Group {                     // one level-mode launch
        int seg_lo, seg_hi, variant, lds_wave;
        int64_t item_lo, item_hi;
    };
    std::vector<Group> groups;
    std::vector<cc::SegDesc> seg_host;        // instance-major
    std::vector<cc::SegDesc> seg_level_host;  // level-major, item_start counted in that order
    std::vector<cc::ReduceDesc> rd_host;
    size_t seg_off = 0, seg_level_off = 0, range_off = 0, rd_off = 0, total = 0;
    int J = 1, lds_wave = 0, max_red_blocks = 1, n_cu = 0;
    uint32_t flags = 0;
};
