/*
 * cc.h — C ABI of the MI355X colour-coding tree counter (libcc.so).
 *
 * The library counts colourful embeddings of a tree template T (k vertices) in an undirected
 * graph G on one AMD MI355X (gfx950) GPU, following the colour-coding method of Section 2.1 of
 * Chen et al., "High-Performance Massive Subgraph Counting using Pipelined Adaptive-Group
 * Communication" (2018): colour G at random with k colours (Algorithm 1, the colouring loop),
 * partition T recursively into active/passive sub-templates (Section 2.1, Figure 1(a); Algorithm 1,
 * "Partition T into subtrees"), evaluate the dynamic program of Eq. 1 bottom-up, sum the per-vertex
 * counts at the full template (Algorithm 1, Eq. 3), and scale to an estimate of #emb(T, G)
 * (Section 2, "Subgraph-counting problem"; the colourful probability k!/k^k of Section 2.1).
 *
 * Conventions for every entry point:
 *   - Plain C types only. "dev" pointers are device (HBM) addresses on the current HIP device;
 *     "host" pointers are ordinary host memory. `stream` is a hipStream_t passed as void*
 *     (NULL = the null stream).
 *   - The caller owns every device buffer it passes (graph arrays, colours, workspaces, outputs)
 *     and keeps it alive until work queued on `stream` that uses it has finished. The library
 *     never frees caller memory.
 *   - Opaque handles (cc_plan, cc_graph) are owned by the library and freed by their destroy
 *     call; they must outlive the stream work that uses them.
 *   - Every call returns a cc_status. On failure nothing has been launched, and cc_last_error()
 *     returns a message (thread-local, valid until the next call on the same thread).
 *     Argument and shape errors are detected on the host before any launch. Faults raised
 *     asynchronously by kernels surface as CC_EDEVICE from a later call, or at the caller's sync.
 *   - No exception, abort or exit crosses this interface.
 *   - Graph format: CSR with int64 row offsets (n+1 entries) and int32 columns (nnz entries),
 *     rows sorted, no self-loops, no duplicates, symmetric (Section 2: G is undirected; an edge
 *     is stored in both directions).
 *   - Count values are IEEE double. They are exact integers when below 2^53. Results are
 *     deterministic: the reduction order of every entry is fixed by the plan and the graph's
 *     work split, never by the batch it runs in.
 */
#ifndef CC_H
#define CC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CC_OK = 0,
    CC_EINVAL = -1,    /* malformed argument: not a tree, bad CSR, null pointer, size mismatch */
    CC_ERANGE = -2,    /* k outside [1, CC_MAX_K], or a size the kernels do not support */
    CC_ENOMEM = -3,    /* host allocation failed */
    CC_ENOSPC = -4,    /* the caller's workspace is smaller than the size the library asked for */
    CC_EDEVICE = -5,   /* a HIP runtime call failed (launch, copy, or an earlier kernel fault) */
    CC_EINTERNAL = -6
} cc_status;

#define CC_MAX_K 16

/* ------------------------------------------------------------------------------------------ */
/* Errors                                                                                      */
/* ------------------------------------------------------------------------------------------ */

/* Message for the last failing call on this thread ("" if none). */
const char* cc_last_error(void);

/* ------------------------------------------------------------------------------------------ */
/* Load tree template (Section 2.1: the template T, its root rho(T) and the recursive split    */
/* into active T' and passive T'' sub-templates; Algorithm 1, "Partition T into subtrees")    */
/* ------------------------------------------------------------------------------------------ */

typedef struct cc_plan cc_plan;

/* flags for cc_plan_create */
#define CC_PLAN_CENTRE_SMALLEST 1u  /* root = centre, attach children smallest subtree first
                                       (the fixed reference partition used for bookkeeping) */
#define CC_PLAN_NO_SHARING 2u       /* run every split of the partition. By default a split whose
                                       rooted sub-template equals one computed earlier in the same
                                       template (equal canonical forms: the same table, Eq. 1) is
                                       not run, and its consumers read the earlier table; the
                                       reference partition never shares */

/*
 * k in [1, CC_MAX_K]; edges (host) = 2*(k-1) int32 vertex ids in [0, k) forming a tree.
 * root in [0, k) fixes the template vertex that the per-vertex counts refer to; root = -1 lets
 * the planner choose the cheapest root (the total X does not depend on the root or the
 * partition). Returns CC_ERANGE for k out of range, CC_EINVAL if the edges are not a tree.
 * The plan is host-only until cc_plan_bind_device.
 */
cc_status cc_plan_create(int32_t k, const int32_t* edges_host, int32_t root, uint32_t flags,
                         cc_plan** out);

typedef struct {
    int32_t k;
    int32_t root;
    int32_t n_splits;                 /* splits that run: k-1, fewer when equal sub-templates are
                                         shared (CC_PLAN_NO_SHARING keeps all k-1) */
    double aut;                       /* |Aut(T)|, the automorphism count of T */
    int64_t units_per_edge;           /* colour-set-edge units per directed CSR entry, counted on
                                         the reference partition: sum over splits of C(k,p), p the
                                         passive size (1 for p = 1) */
    int64_t table3_memory;            /* sum of C(k,|T_i|) and of C(k,|T_i|) C(|T_i|,|T_i'|) over */
    int64_t table3_compute;           /*   this plan's split sub-templates other than T itself
                                           (the bookkeeping of the paper's Table 3) */
    int64_t gather_doubles_per_edge;  /* doubles read per CSR entry over all splits (this plan) */
    int64_t combine_fma_per_vertex;   /* multiply-adds per vertex over all splits (this plan) */
    int64_t peak_live_columns;        /* widest sum of live per-vertex table columns (doubles) */
    size_t device_bytes;              /* size of the plan's device constants (cc_plan_bind_device) */
} cc_plan_info;

cc_status cc_plan_info_get(const cc_plan* plan, cc_plan_info* out);

/* Sub-template sizes of split i in execution order: *s = |T_i|, *a = |T_i'|, *p = |T_i''|. */
cc_status cc_plan_split_get(const cc_plan* plan, int32_t i, int32_t* s, int32_t* a, int32_t* p);

/* The maps one split reads (Section 2.1, Eq. 1: the neighbour sum over T_i'' and the combine over
 * the splits of each colour set), as byte offsets into the plan's device constants (-1: absent):
 *   split_off: a >= 2: u32 [C(s-1, p)][W(s)], for each output entry (storage order) its pairs
 *              (storage position of S1 in the active row) | (colex rank of S \ S1 in N) << 16;
 *              a = 1: u32 [W(s)], the colex rank in N of each output entry;
 *   fold_off:  p >= 2: u16 [k][k][W(p)], fold[col(u)][col(v)][j] = colex rank in N of passive entry j,
 *              or 0xFFFF when its set holds col(v);
 *   mask_off:  p >= 2: u16 [W(p)], the colour set of passive entry j over the k-1 colours other
 *              than the neighbour's;
 *   full_off, emap_off: the packed layout's maps (colour sets over all k colours);
 *   proj_src_off, proj_fold_off: splits whose passive rows exceed 64 entries (Wn > 0): u16
 *              [k][k][Wn], Wn = C(k-2, p-1): for a neighbour of colour cu and a centre of colour
 *              cv, the storage positions of the passive entries whose set avoids cv, in increasing
 *              order of their colex rank in N, and those ranks (the projected rows, cc_tuning).
 * act, pas: table ids read (-1: a single vertex); out: table id written (-2: the full template).
 * For inspection and host-side checks of the planner; no count call needs it. CC_ERANGE for i out
 * of range, CC_EINVAL for NULL arguments. */
typedef struct {
    int32_t act, pas, out;
    int64_t split_off, fold_off, mask_off, full_off, emap_off;
    int64_t proj_src_off, proj_fold_off;
    int32_t Wn;
} cc_split_maps;

cc_status cc_plan_split_maps(const cc_plan* plan, int32_t i, cc_split_maps* out);

/* Copy the plan's device constants (info.device_bytes bytes) into host memory `host` of `bytes`
 * bytes (CC_ENOSPC if smaller). Host-only; the same bytes cc_plan_bind_device uploads. */
cc_status cc_plan_constants_get(const cc_plan* plan, void* host, size_t bytes);

/*
 * Copy the plan's constant tables (colour-set split lists and neighbour fold maps) into the
 * caller's device buffer `dev` of at least info.device_bytes bytes, on `stream`, and remember it.
 * Must be called once before the plan is used by cc_count*; calling it again rebinds.
 */
cc_status cc_plan_bind_device(cc_plan* plan, void* dev, size_t bytes, void* stream);

void cc_plan_destroy(cc_plan* plan);

/*
 * Storage order of the entries of a colour-anchored table row (Section 2.1, Eq. 1: the counts
 * C(v, T_i, S) of one vertex, S over the k colours): for templates on k vertices and sets holding
 * m colours besides col(v), order[pos] receives the colex rank, over the k-1 other colours, of the
 * set stored at position pos. Rows of more than 16 entries are stored so that 128-byte lines hold
 * sets sharing a common subset; shorter rows keep colex order. `order` is host memory of n
 * entries, n = C(k-1, m). CC_ERANGE for k outside [1, CC_MAX_K] or m outside [0, k-1], CC_EINVAL
 * for a NULL pointer or another n.
 */
cc_status cc_entry_order(int32_t k, int32_t m, int32_t* order, int64_t n);

/* ------------------------------------------------------------------------------------------ */
/* Load CSR graph                                                                               */
/* ------------------------------------------------------------------------------------------ */

typedef struct cc_graph cc_graph;

/* work-split tuning (the degree split of Section 3.3, Algorithm 4, mapped to wavefronts) */
typedef struct {
    int32_t hub_threshold;  /* rows with more neighbours than this are cut into chunks (0 = auto) */
    int32_t chunk;          /* neighbours per chunk of a cut row (0 = auto; multiple of 64) */
    int32_t cols_per_lane;  /* passive-row doubles each lane holds per pass: 1, 2, 4, 8 or 16 (0 = auto) */
    /* projected passive rows for splits whose passive rows exceed 64 entries: a centre of colour c
     * adds up only the neighbour entries whose colour set avoids c (Eq. 1: the active and passive
     * colour sets are disjoint), so the count can copy those entries of every row into one
     * contiguous row per colour and run the split's centres colour class by colour class, a few
     * classes per pass, reading whole 128-byte lines that hold only needed entries.
     * 0 = auto (a byte model per split and graph decides; the copies take at most as much
     * workspace as the table arena), -1 = never, 1..16 = always, this many colour classes per
     * pass. Results are exact below 2^53 either way, and bit-identical when a passive row fits in
     * one pass of the gather (the same terms reach each sum in the same order). */
    int32_t proj_classes;
    /* packed counts: doubles of one neighbour's row tile (the colourings of a tile side by side)
     * that a wavefront reads per pass, 128, 256 or 512 (0 = auto: 256 when p >= 2, 512 when
     * p = 1); more colourings per tile read each CSR entry fewer times but hold more registers */
    int32_t packed_tile;
} cc_tuning;

/* flags for cc_graph_prepare */
#define CC_GRAPH_TRUST 1u   /* skip the device-side CSR validation */

/* Upper bound of the graph workspace (device bytes) for a graph of n vertices and nnz entries. */
cc_status cc_graph_workspace_bytes(int64_t n, int64_t nnz, const cc_tuning* tuning, size_t* bytes);

/*
 * Prepare a graph whose CSR lives in caller device memory (row_ptr_dev: n+1 int64,
 * col_dev: nnz int32). Unless CC_GRAPH_TRUST is set, a validation kernel checks that the rows are
 * sorted, in range, free of self-loops and duplicates, and symmetric (CC_EINVAL otherwise).
 * Builds the per-graph work lists (light rows, cut rows and their chunks) into `ws_dev`.
 * Synchronises `stream` once (the row offsets are read back to the host to cut rows).
 * The CSR and the workspace must stay alive and unchanged while the graph handle is used.
 */
cc_status cc_graph_prepare(int64_t n, int64_t nnz, const int64_t* row_ptr_dev, const int32_t* col_dev,
                           void* ws_dev, size_t ws_bytes, const cc_tuning* tuning, uint32_t flags,
                           void* stream, cc_graph** out);

typedef struct {
    int64_t n, nnz;
    int64_t max_degree;
    int64_t n_light, n_hubs, n_chunks;
    int32_t hub_threshold, chunk, cols_per_lane, proj_classes, packed_tile;
} cc_graph_info;

cc_status cc_graph_info_get(const cc_graph* g, cc_graph_info* out);

void cc_graph_release(cc_graph* g);

/* ------------------------------------------------------------------------------------------ */
/* Colour (Algorithm 1: every vertex picks a colour in {1..k} uniformly at random)             */
/* ------------------------------------------------------------------------------------------ */

/*
 * colours_dev[b*n + v] = colour of v in colouring (first_iter + b), for b in [0, B):
 *   h = mix64(mix64(seed + 0x9E3779B97F4A7C15*(iter+1)) + 0xD1B54A32D192ED03*(v+1)),
 *   colour = floor(k * h / 2^64)
 * where mix64 is the SplitMix64 finaliser. colours_dev holds B*n bytes (caller-owned).
 */
cc_status cc_color(const cc_graph* g, int32_t k, uint64_t seed, uint64_t first_iter, int32_t B,
                   uint8_t* colours_dev, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Count (Algorithm 1: the dynamic program of Eq. 1 over the partition, then Eq. 3's sum)      */
/* ------------------------------------------------------------------------------------------ */

/* Device workspace needed by cc_count for this plan on this graph (independent of B): the live
 * count tables, the cut rows' chunk partials, the root row, the reduction scratch, the
 * per-CSR-entry neighbour colours of one colouring (nnz bytes) and, when a split runs on projected
 * passive rows (cc_tuning.proj_classes), the projected rows of one pass. */
cc_status cc_count_workspace_bytes(const cc_plan* plan, const cc_graph* g, size_t* bytes);

/* How cc_count runs each split of this plan on this graph: classes[i] = colour classes per pass
 * of split i on projected passive rows (cc_tuning.proj_classes), 0 when split i reads the passive
 * table itself. `classes` is host memory of n >= info.n_splits entries. Host-only. CC_EINVAL for
 * NULL arguments or a short array. */
cc_status cc_count_projection(const cc_plan* plan, const cc_graph* g, int32_t* classes, int32_t n);

/*
 * For b in [0, B): X_dev[b] = number of colourful labelled embeddings of T in G under colouring
 * colours_dev + b*n (values in [0, k)), i.e. the number of injective maps phi : V_T -> V_G that
 * keep every template edge and give the k template vertices k different colours.
 * vertex_dev (optional, may be NULL): B*n doubles; vertex_dev[b*n + v] = the number of those maps
 * with phi(root) = v, root as reported by cc_plan_info.
 * The colourings are processed one after another on `stream`, reusing the workspace.
 */
cc_status cc_count(const cc_plan* plan, const cc_graph* g, const uint8_t* colours_dev, int32_t B,
                   void* ws_dev, size_t ws_bytes, double* X_dev, double* vertex_dev, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): cc_count with the workspace taken from a fixed array of
 * CC_NOALLOC_SCRATCH_BYTES that the library holds in device memory, one per GPU, until the process
 * ends. Same arguments and results as cc_count (bit for bit: the same kernels in the same order);
 * no workspace argument. Allocates nothing (no hipMalloc, hipFree or allocating library call);
 * the plan's profiling must be off. CC_ENOSPC with a message when cc_count_workspace_bytes for this
 * plan and graph exceeds CC_NOALLOC_SCRATCH_BYTES, CC_EINVAL when the graph's device is not the
 * current one. All calls on one GPU share the array: calls that overlap on one GPU (other streams,
 * other threads) race and must be serialised by the caller.
 */
#define CC_NOALLOC_SCRATCH_BYTES (128u << 20)  /* 128 MiB per GPU */
cc_status cc_count_noalloc(const cc_plan* plan, const cc_graph* g, const uint8_t* colours_dev, int32_t B,
                           double* X_dev, double* vertex_dev, void* stream);

/*
 * Count within a device-memory budget (the paper's concern with the peak memory of intermediate
 * count tables, Section 3.2, Eq. (peakm), and Section 4.4). The live tables of Eq. 1 peak where a
 * large table waits between two uses while others are computed (for example the active table of
 * the root split, written early and read last). cc_count_budget parks such tables in host memory:
 * a parked table goes to the caller's host buffer after its last use before the idle stretch and
 * comes back into the device arena just before its next reader; the arena is laid out again
 * without it in between (tables placed largest first, each at the lowest columns free over its
 * lifetime). Tables are chosen greedily until the arena fits the budget: the largest table idle at
 * the split where the resident columns peak. The kernels and their
 * order are those of cc_count, so the counts are bit-identical to cc_count's; only where the
 * tables live changes (copies are queued on `stream` and ordered with the kernels). When no table
 * is idle at the peak, the scratch of projected passive rows (cc_tuning.proj_classes) shrinks to
 * fewer colour classes per pass, then to none (more passes: exact below 2^53 and 1e-12 above
 * against cc_count, bit-identical when every passive row fits one gather pass).
 *
 * cc_count_budget_plan reports, for this plan, graph and budget (bytes of device workspace),
 * the workspace and host bytes cc_count_budget needs, how many tables it parks, and the table
 * arena with and without parking (in per-vertex doubles); CC_ENOSPC when even parking every
 * table idle at the peak does not meet the budget. host_buf: host memory of host_bytes, page-
 * locked for asynchronous copies (hipHostMalloc, or torch's pin_memory), owned by the caller and
 * left untouched when no table is parked. Other arguments and errors as cc_count.
 */
typedef struct {
    size_t workspace_bytes;    /* device workspace cc_count_budget needs (<= the budget when it fits) */
    size_t host_bytes;         /* host bytes of the parked tables */
    int32_t parked_tables;     /* tables parked over an idle stretch (between two uses) */
    int32_t proj_classes;      /* most colour classes per pass of projected rows (0: none projected) */
    int64_t arena_columns;     /* device table arena, per-vertex doubles */
    int64_t unbounded_columns; /* the arena of cc_count */
} cc_budget_info;

cc_status cc_count_budget_plan(const cc_plan* plan, const cc_graph* g, size_t device_budget, cc_budget_info* out);

cc_status cc_count_budget(const cc_plan* plan, const cc_graph* g, const uint8_t* colours_dev, int32_t B,
                          size_t device_budget, void* ws_dev, size_t ws_bytes, void* host_buf, size_t host_bytes,
                          double* X_dev, double* vertex_dev, void* stream);

/*
 * Inspection of one step of the dynamic program (Section 2.1, Eq. 1: the table C(., T_i, .) of a
 * split is computed from the tables of its active part T_i' and passive part T_i'' alone), so that
 * a caller can check any single split at sizes where the whole count cannot be recomputed on the
 * host. Runs the splits 0..last (execution order) of one colouring (colours_dev: n bytes) in the
 * count workspace of cc_count (ws_bytes >= cc_count_workspace_bytes) and stops, without the root
 * reduction. Afterwards the tables that split `last` reads (its act and pas ids from
 * cc_plan_split_maps) and the table it writes (its out id) hold their values in the workspace
 * (cc_plan_table_get says where); when split `last` is the root split (out = -2) its per-vertex
 * counts go to vertex_dev (n doubles, required then, ignored otherwise). Queued on `stream`.
 * CC_ERANGE for `last` out of range, CC_EINVAL for NULL pointers or an unbound plan, CC_ENOSPC
 * for a small workspace.
 */
cc_status cc_count_inspect(const cc_plan* plan, const cc_graph* g, const uint8_t* colours_dev, int32_t last,
                           void* ws_dev, size_t ws_bytes, double* vertex_dev, void* stream);

/* Where table `table` (an id of cc_plan_split_maps) lives in a cc_count workspace for this plan on
 * this graph: row v of the table starts at byte offset + 8 * v * stride of the workspace and holds
 * width = C(k-1, size-1) doubles, the counts C(v, T_i, S) of the colour sets S of `size` colours
 * that contain col(v); entry j is the set made of col(v) and the (size-1)-set over the other k-1
 * colours (renumbered 0..k-2 in increasing order) whose colex rank is order[j] of
 * cc_entry_order(k, size-1). Host-only. CC_ERANGE for a table id out of range. */
typedef struct {
    int32_t size;    /* sub-template size |T_i| */
    int32_t width;   /* doubles per row that hold counts */
    int64_t stride;  /* doubles between the rows of consecutive vertices */
    int64_t offset;  /* byte offset of vertex 0's row in the workspace */
} cc_table_desc;

cc_status cc_plan_table_get(const cc_plan* plan, const cc_graph* g, int32_t table, cc_table_desc* out);

/* ------------------------------------------------------------------------------------------ */
/* Packed count: B colourings of one template in one pass over the graph                        */
/* ------------------------------------------------------------------------------------------ */

#define CC_MAX_PACKED 4096  /* largest B of a packed count */

/* Device workspace needed by cc_count_packed for this plan, graph and B. */
cc_status cc_count_packed_workspace_bytes(const cc_plan* plan, const cc_graph* g, int32_t B, size_t* bytes);

/*
 * The outer loop of Algorithm 1 (Section 2.1) over B colourings, evaluated together: every table
 * row holds the counts of all B colourings side by side (row v = [colouring][colour set]), so each
 * split reads a neighbour's row and CSR entry once for all colourings. Computes, for b in [0, B),
 * the same X_dev[b] as cc_count (Eq. 1 applied per colouring): exact below 2^53, and above it
 * within the rounding of a different but fixed summation order (every neighbour sum adds its
 * terms in CSR order), so a colouring's result does not depend on B or on the other colourings.
 * colours_dev: B*n bytes, colouring b at colours_dev + b*n (the layout cc_color writes).
 * vertex_dev (optional, may be NULL): n*B doubles, vertex_dev[v*B + b] = the maps of colouring b
 * with phi(root) = v. CC_ERANGE when B is outside [1, CC_MAX_PACKED] or when a split of the plan
 * is too wide for the packed kernels (templates of up to 12 vertices always fit).
 */
cc_status cc_count_packed(const cc_plan* plan, const cc_graph* g, const uint8_t* colours_dev, int32_t B,
                          void* ws_dev, size_t ws_bytes, double* X_dev, double* vertex_dev, void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Packed count of several templates of one size, sharing equal sub-template tables            */
/* ------------------------------------------------------------------------------------------ */

typedef struct cc_multi cc_multi;

/*
 * Prepare a count of n_plans templates with the same k over the same colourings (host only; the
 * plans must outlive the object). Eq. 1 gives every rooted sub-template T_i of a partition the
 * same table C(., T_i, .) whichever template and partition it comes from (Section 2.1), so the
 * table of each distinct rooted sub-template (equal canonical forms) is computed once, in the
 * first template that needs it, and kept until its last use; a template's splits whose output is
 * already there are not run, nor the splits that only feed them. CC_EINVAL for NULL plans or
 * different k.
 */
cc_status cc_multi_create(int32_t n_plans, const cc_plan* const* plans, cc_multi** out);

/* Splits that run (n_steps), splits of all plans before sharing (n_splits), shared tables. */
cc_status cc_multi_info_get(const cc_multi* multi, int32_t* n_steps, int64_t* n_splits, int32_t* n_tables);

/* Step i (0 <= i < n_steps, execution order): the plan index and that plan's split index it runs
 * (cc_plan_split_get gives the split's sizes). CC_ERANGE for i out of range. */
cc_status cc_multi_step_get(const cc_multi* multi, int32_t i, int32_t* plan, int32_t* split);

void cc_multi_destroy(cc_multi* multi);

/* Device workspace needed by cc_count_packed_multi for this multi-template count, graph and B. */
cc_status cc_count_packed_multi_workspace_bytes(const cc_multi* multi, const cc_graph* g, int32_t B, size_t* bytes);

/*
 * X_dev[p*B + b] = the colourful count of template p under colouring b (colours_dev as for
 * cc_count_packed: B*n bytes, colouring b at colours_dev + b*n), every template's tables in the
 * packed layout. Exact below 2^53; above, within the rounding of a fixed summation order (a shared
 * table may come from another partition than the template's own, so values above 2^53 can differ
 * in the last bits from cc_count_packed of that template alone). Errors as cc_count_packed.
 */
cc_status cc_count_packed_multi(const cc_multi* multi, const cc_graph* g, const uint8_t* colours_dev, int32_t B,
                                void* ws_dev, size_t ws_bytes, double* X_dev, void* stream);

/* Device workspace of cc_count_packed_multi_persistent for this multi-template count, graph and B. */
cc_status cc_count_packed_multi_persistent_workspace_bytes(const cc_multi* multi, const cc_graph* g, int32_t B,
                                                           size_t* bytes);

/*
 * The same counts as cc_count_packed_multi (bit for bit: every item runs the same device code on
 * the same tiles), in one persistent launch over (split, task or cut row, colouring tile) items:
 * the outer loop of Algorithm 1 over B colourings and every template's splits of Eq. 1
 * (Section 2.1), the neighbour lists cut into tasks as in Section 3.3, Algorithm 4. The splits are
 * grouped by dependency level; the resident workgroups take each level's tasks, then its cut-row
 * finishes, one item block at a time from a per-phase counter in the workspace, with a device-wide
 * barrier between phases (a cooperative launch, so every workgroup is resident and the barrier
 * cannot wait on one that never runs). Tables are placed so
 * that the splits of one level never share memory. Then the per-template root sums.
 * Every split must run the packed kernels (rows of at most 64 entries per colouring: templates of
 * up to 7 vertices, or wider templates whose splits stay narrow); CC_ERANGE otherwise. A barrier
 * that does not open within about 10 s (which a resident grid cannot cause) makes every count NaN.
 * The multi object holds the launch's host descriptors until the next call: concurrent calls with
 * one multi object must be serialised by the caller.
 */
cc_status cc_count_packed_multi_persistent(const cc_multi* multi, const cc_graph* g, const uint8_t* colours_dev,
                                           int32_t B, void* ws_dev, size_t ws_bytes, double* X_dev, void* stream);

/* Synchronise `stream` and report any device error of the work queued on it (CC_EDEVICE). */
cc_status cc_stream_check(void* stream);

/* ------------------------------------------------------------------------------------------ */
/* Batched count: many colourings and templates, on one or more graphs, in one launch          */
/* (the independent outer iterations of Algorithm 1 run together)                              */
/* ------------------------------------------------------------------------------------------ */

typedef struct {
    const cc_plan* plan;         /* bound to device memory (cc_plan_bind_device) */
    const cc_graph* graph;
    const uint8_t* colours_dev;  /* n bytes: one colouring of the graph, values in [0, plan k) */
    double* X_dev;               /* 1 double: receives X for this colouring */
    double* vertex_dev;          /* optional n doubles of per-vertex counts (NULL = not kept) */
} cc_instance;

typedef struct cc_batch cc_batch;

#define CC_BATCH_LEVELS 1u  /* one launch per split level instead of one persistent launch */
/* The persistent launch sizes its grid to the device's resident capacity; a batch meant to run
 * next to d-1 other batches on other streams can take 1/d of it, set as CC_BATCH_SHARE(d)
 * (1 <= d <= 255), leaving room for their workgroups. */
#define CC_BATCH_SHARE(d) (((uint32_t)(d) & 0xFFu) << 8)

/*
 * Prepare a batch of n_inst instances (host only; the instance array is copied). Every instance
 * computes exactly what cc_count computes for its plan, graph and colouring, bit for bit: the
 * kernels and the per-entry summation order are the same. By default the whole batch runs in one
 * persistent launch in which each workgroup owns whole instances and runs their splits in plan
 * order (a workgroup barrier between splits; no device-wide synchronisation); CC_BATCH_LEVELS
 * runs one launch per split level across all instances instead.
 */
cc_status cc_batch_create(int32_t n_inst, const cc_instance* inst, uint32_t flags, cc_batch** out);

/* Device workspace needed by cc_batch_run (tables of every instance are resident together). */
cc_status cc_batch_workspace_bytes(const cc_batch* batch, size_t* bytes);

/*
 * Queue the batch on `stream`. The batch object, its plans and graphs and all buffers must stay
 * alive until the work has finished; a batch may be run again only after its previous run has
 * finished.
 */
cc_status cc_batch_run(cc_batch* batch, void* ws_dev, size_t ws_bytes, void* stream);

/* Synchronise `stream` and report any device error of the work queued on it (CC_EDEVICE). */
cc_status cc_batch_check(cc_batch* batch, void* stream);

void cc_batch_destroy(cc_batch* batch);

/* ------------------------------------------------------------------------------------------ */
/* Measurement                                                                                  */
/* ------------------------------------------------------------------------------------------ */

/*
 * Per-split kernel timing. While enabled on a plan, every cc_count and cc_count_packed with that
 * plan records HIP events on its stream around (1) the neighbour-gather + combine kernel and (2)
 * the cut-row finish kernel of each split, for every launch: one per colouring for cc_count and
 * for the splits a packed count runs colouring by colouring, one per packed count for the splits
 * it runs on packed rows. Not thread-safe: one counting stream per plan while enabled. Enabling
 * again clears what was recorded.
 */
cc_status cc_profile_enable(cc_plan* plan, int32_t enable);

/*
 * Synchronise on the recorded events and return, for each of the first n splits (execution
 * order), the summed milliseconds of its gather kernel and of its finish kernel and the number of
 * launches recorded. Any array may be NULL. Recording stays enabled and is cleared.
 */
cc_status cc_profile_read(cc_plan* plan, int32_t n, double* gather_ms_host, double* finish_ms_host,
                          int64_t* launches_host);

/* ------------------------------------------------------------------------------------------ */
/* Estimate (Algorithm 1, Eq. 3 and the final averaging; Section 2.1 colourful probability)    */
/* ------------------------------------------------------------------------------------------ */

/*
 * Host-side: *estimate = mean_b(X_host[b]) * k^k / k! / |Aut(T)|, evaluated in long double and
 * rounded once; *std_err = the standard error of that mean (0 for B = 1).
 */
cc_status cc_estimate(const cc_plan* plan, const double* X_host, int32_t B, double* estimate,
                      double* std_err);

/*
 * Host-side (epsilon, delta) estimate of Algorithm 1's last step: split the B values into
 * `groups` groups of equal size (B must be a multiple of groups), average each, and return the
 * median of the group means, scaled as in cc_estimate.
 */
cc_status cc_estimate_median_of_means(const cc_plan* plan, const double* X_host, int32_t B,
                                      int32_t groups, double* estimate);

/*
 * Host-side sample sizes for an (epsilon, delta)-approximation (Algorithm 1: the number of
 * colourings, of order e^k log(1/delta) / epsilon^2, split into t groups of order log(1/delta)
 * whose means are combined by a median). The paper gives only the orders; the constants are this
 * library's reading: each group mean is within epsilon of the truth with probability >= 3/4 by
 * Chebyshev when the group holds ceil(4 e^k / epsilon^2) colourings (the relative variance of one
 * scaled colourful count taken as at most e^k), and the median of t = ceil(8 ln(1/delta)) such
 * means fails only if half of them fail, which Hoeffding bounds by exp(-t/8) <= delta.
 * *per_group = ceil(4 e^k / epsilon^2), *groups = max(1, ceil(8 ln(1/delta))); the total is their
 * product. CC_ERANGE unless 1 <= k <= 16, 0 < epsilon < 1, 0 < delta < 1, or if per_group would
 * exceed 2^62.
 */
cc_status cc_iterations(int32_t k, double epsilon, double delta, int64_t* per_group, int32_t* groups);

#ifdef __cplusplus
}
#endif

#endif /* CC_H */
