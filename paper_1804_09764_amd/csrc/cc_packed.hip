// HIP kernels and launchers of the packed layout (B colourings per table row); the device
// functions they run are in cc_packed.h.
#include <hip/hip_runtime.h>

#include "cc_device.h"
#include "cc_internal.h"
#include "cc_packed.h"

namespace cc {

// ---------------------------------------------------------------------------------------------
// packed layout: one split for B colourings at once
// ---------------------------------------------------------------------------------------------

template <int J, bool P1>
__global__ __launch_bounds__(256) void k_psplit(StepParams S) {
    extern __shared__ double lds[];
    const PMaps M = stage_maps(S, lds);
    __syncthreads();
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    double* N = lds + S.tab_doubles + (int64_t)wib * S.lds_wave;
    double* Ash = N + S.a_off;
    // the wavefronts form groups of `tiles`, one per colouring tile; the groups take the tasks
    // round-robin (the launch has at least `tiles` wavefronts)
    const int tiles = ptiles(S);
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * S.waves_per_block + wib);
    const int groups = (int)(gridDim.x * S.waves_per_block) / tiles;
    const int g = w / tiles;
    const int b0 = (w - g * tiles) * S.bt;
    if (g >= groups) return;
    const int64_t n_tasks = S.n_chunks + S.n_ranges;
    for (int64_t t = g; t < n_tasks; t += groups) do_ptask<J, P1>(S, t, b0, N, Ash, M, lane);
}

__global__ __launch_bounds__(256) void k_phub(StepParams S) {
    extern __shared__ double lds[];
    const PMaps M = stage_maps(S, lds);
    __syncthreads();
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    double* N = lds + S.tab_doubles + (int64_t)wib * S.lds_wave;
    double* Ash = N + S.a_off;
    const int tiles = ptiles(S);
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * S.waves_per_block + wib);
    const int groups = (int)(gridDim.x * S.waves_per_block) / tiles;
    const int g = w / tiles;
    const int b0 = (w - g * tiles) * S.bt;
    if (g >= groups) return;
    for (int64_t t = g; t < S.n_hubs; t += groups) do_phub(S, t, b0, N, Ash, M, lane);
}

// [B][n] -> [n][B] bytes through 64 x 64 LDS tiles
__global__ __launch_bounds__(256) void k_transpose_colours(const uint8_t* __restrict__ in, int64_t n, int B,
                                                           uint8_t* __restrict__ out) {
    __shared__ uint8_t tile[64][65];
    const int64_t v0 = (int64_t)blockIdx.x * 64;
    const int b0 = blockIdx.y * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int r = ty; r < 64; r += 4) {
        const int b = b0 + r;
        const int64_t v = v0 + tx;
        tile[r][tx] = (b < B && v < n) ? in[(int64_t)b * n + v] : 0;
    }
    __syncthreads();
    for (int r = ty; r < 64; r += 4) {
        const int64_t v = v0 + r;
        const int b = b0 + tx;
        if (b < B && v < n) out[v * B + b] = tile[tx][r];
    }
}

// per-colouring sums of x[v][b]: block (range, 64 colourings); each thread adds its vertices in the
// blocked order, the four threads of a colouring are added in order, then the block sums in the
// blocked order
__global__ __launch_bounds__(256) void k_reduce_packed_blocks(const double* __restrict__ x, int64_t n, int B,
                                                              int64_t per_block, double* __restrict__ partial) {
    __shared__ double sh[256];
    const int tb = threadIdx.x & 63, tv = threadIdx.x >> 6;
    const int b = blockIdx.y * 64 + tb;
    const int64_t lo = blockIdx.x * per_block;
    const int64_t hi = lo + per_block < n ? lo + per_block : n;
    double s = 0.0;
    if (b < B && lo + tv < hi) {
        const int m = (int)((hi - lo - tv + 3) / 4);  // this thread's vertices lo + tv, lo + tv + 4, ...
        s = blocked_sum(m, [&](int i) { return x[(lo + tv + 4 * (int64_t)i) * B + b]; });
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    if (tv == 0 && b < B) partial[(int64_t)blockIdx.x * B + b] = ((sh[tb] + sh[64 + tb]) + sh[128 + tb]) + sh[192 + tb];
}

__global__ __launch_bounds__(256) void k_reduce_packed_final(const double* __restrict__ partial, int blocks, int B,
                                                             double* __restrict__ out) {
    const int b = blockIdx.x * 256 + threadIdx.x;
    if (b >= B) return;
    out[b] = blocked_sum(blocks, [&](int i) { return partial[(int64_t)i * B + b]; });
}

// ---------------------------------------------------------------------------------------------
// packed layout launchers
// ---------------------------------------------------------------------------------------------

void packed_tile(StepParams* S) {
    const int per = S->Cf + (S->a >= 2 ? S->Wa : 0);
    const int width = S->p >= 2 ? S->Wp : S->k;
    int cap = S->B < kWave ? S->B : kWave;
    // tile elements per lane: up to 4 (p >= 2: a tile row of about 2 KB) or 8 (p = 1: counts in
    // registers), unless the graph's tuning sets the tile row
    const int elems = S->tile_doubles > 0 ? S->tile_doubles : (S->p >= 2 ? 256 : 512);
    const int by_width = elems / width > 1 ? elems / width : 1;
    const int by_lds = 1024 / per > 1 ? 1024 / per : 1;      // about 8 KB of LDS per wavefront
    if (cap > by_width) cap = by_width;
    if (cap > by_lds) cap = by_lds;
    if (cap < 1) cap = 1;
    // equal tiles, a multiple of 4 colourings when that stays within the caps
    const int tiles = (S->B + cap - 1) / cap;
    int bt = (S->B + tiles - 1) / tiles;
    if (((bt + 3) & ~3) <= cap) bt = (bt + 3) & ~3;
    S->bt = bt;
    int J = 1;
    while (J < 8 && kWave * J < bt * width) J <<= 1;
    if (S->force_J > 0) J = S->force_J;
    S->pJ = J;
    // every offset is even (16-byte aligned) so that the colour stage takes 16-byte LDS stores
    auto even = [](int x) { return (x + 1) & ~1; };
    S->a_off = even(bt * S->Cf);
    S->tg_off = even(S->a_off + (S->a >= 2 ? bt * S->Wa : 0));
    S->cs_off = even(S->tg_off + (S->p >= 2 ? J * S->k * kWave / 4 : 0));
    S->lds_wave = even(S->cs_off + (kWave * bt + 7) / 8);
    S->tab_u16 = (S->a >= 2 ? 2 * S->npairs * S->Ws : 0) + (S->p >= 2 ? S->k * S->Wp : 0) + S->k * S->Nw;
    S->tab_doubles = even((S->tab_u16 + 3) / 4);
}

size_t packed_lds_bytes(const StepParams& S, int waves) {
    return ((size_t)S.tab_doubles + (size_t)S.lds_wave * waves) * sizeof(double);
}

hipError_t launch_packed_split(StepParams S, int n_cu, hipStream_t st, hipEvent_t mid) {
    packed_tile(&S);
    if (packed_lds_bytes(S, 1) > 64 * 1024) return hipErrorInvalidConfiguration;
    int w = 4;
    while (w > 1 && packed_lds_bytes(S, w) > 64 * 1024) w >>= 1;
    S.waves_per_block = w;
    const int threads = w * kWave;
    const size_t lds = packed_lds_bytes(S, w);
    const int J = S.pJ;
    const void* fn;
    if (S.p == 1)
        fn = J == 1 ? (const void*)k_psplit<1, true>
           : J == 2 ? (const void*)k_psplit<2, true>
           : J == 4 ? (const void*)k_psplit<4, true>
                    : (const void*)k_psplit<8, true>;
    else
        fn = J == 1 ? (const void*)k_psplit<1, false>
           : J == 2 ? (const void*)k_psplit<2, false>
           : J == 4 ? (const void*)k_psplit<4, false>
                    : (const void*)k_psplit<8, false>;
    int per_cu = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
    if (err != hipSuccess) return err;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int64_t tiles = (S.B + S.bt - 1) / S.bt;
    const int64_t total = (S.n_chunks + S.n_ranges) * tiles;
    int64_t blocks = (int64_t)per_cu * n_cu;
    const int64_t need = (total + w - 1) / w;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    if (total > 0) {
        void* args[] = {&S};
        err = hipLaunchKernel(fn, dim3((unsigned)blocks), dim3(threads), args, lds, st);
        if (err != hipSuccess) return err;
        err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    if (mid) {
        err = hipEventRecord(mid, st);
        if (err != hipSuccess) return err;
    }
    if (S.n_hubs > 0) {
        int per_cu2 = 0;
        err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, (const void*)k_phub, threads, lds);
        if (err != hipSuccess) return err;
        if (per_cu2 < 1) return hipErrorInvalidConfiguration;
        int64_t b2 = (int64_t)per_cu2 * n_cu;
        const int64_t need2 = (S.n_hubs * tiles + w - 1) / w;
        if (b2 > need2) b2 = need2;
        hipLaunchKernelGGL(k_phub, dim3((unsigned)b2), dim3(threads), lds, st, S);
        err = hipGetLastError();
    }
    return err;
}

// ---------------------------------------------------------------------------------------------
// multi-template packed count in one persistent launch
// ---------------------------------------------------------------------------------------------

// Device-wide barrier of a cooperative launch (every workgroup is resident). bar[0] counts the
// workgroups that arrived, bar[1] is the generation: the last to arrive resets the count and opens
// the next generation. Stores before the barrier are released at device scope and loads after it
// acquire at device scope, so tables written by one XCD are seen by the others. The wait is
// bounded by the 100 MHz real-time counter: after about 10 s a workgroup stops waiting and sets
// bar[2], so a barrier that never opens ends the kernel (with the error flag raised) instead of
// hanging it.
constexpr uint64_t kBarrierTicks = 1000000000ull;

__device__ void grid_barrier(unsigned* bar, unsigned nblocks) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(bar + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        const unsigned arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(bar + 1, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(8);
                if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTicks) {
                    __hip_atomic_store(bar + 2, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// The phases in order (even: the tasks of a dependency level, odd: its cut-row finishes; an item
// is one colouring tile of a task or cut row). Item blocks are taken from a per-phase counter
// (bar[3 + ph], zero at launch): a workgroup that ends its block early takes the next one, so the
// phase ends about one block after the first workgroup runs out of work, whatever the spread of
// item costs (light-row ranges of many small rows cost several times a range of one large row).
// The workgroup stages the block's split maps in LDS when the split changes, and each of its
// wavefronts runs one item of the block. Which workgroup runs an item changes nothing in its
// arithmetic.
template <int JP>
__global__ __launch_bounds__(256, 3) void k_pmulti(const PSeg* __restrict__ segs, const PItemBlock* __restrict__ blocks,
                                                const PPhase* __restrict__ phases, int n_phases, int tab_doubles,
                                                int lds_wave, unsigned* bar) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    double* N = lds + tab_doubles + (int64_t)wib * lds_wave;
    int staged = -1;
    PMaps M{};
    // the current split's arguments, staged in LDS with its maps (read from HBM they measured
    // 25 % slower: fields are read inside the neighbour loops)
    __shared__ StepParams Ssh;
    __shared__ unsigned next;
    for (int ph = 0; ph < n_phases; ++ph) {
        const PPhase P = phases[ph];
        const bool finish = (ph & 1) != 0;
        for (;;) {
            if (threadIdx.x == 0)
                next = __hip_atomic_fetch_add(bar + 3 + ph, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            const int64_t b = next;
            __syncthreads();  // every wavefront has read `next` before it is written again
            if (b >= P.n_blocks) break;
            const PItemBlock ib = blocks[P.first_block + b];
            const int seg = __builtin_amdgcn_readfirstlane(ib.seg);
            if (seg != staged) {
                M = stage_maps(segs[seg].S, lds);  // the workgroup is past the previous block
                if (threadIdx.x == 0) Ssh = segs[seg].S;
                __syncthreads();
                staged = seg;
            }
            const StepParams& S = Ssh;
            if (wib < ib.count) {
                double* Ash = N + S.a_off;
                const int tiles = ptiles(S);
                const int64_t item = ib.first + __builtin_amdgcn_readfirstlane(wib);
                const int64_t t = item / tiles;
                const int b0 = (int)(item - t * tiles) * S.bt;
                if (finish) do_phub(S, t, b0, N, Ash, M, lane);
                else if (segs[seg].p1) {
                    if (__builtin_amdgcn_readfirstlane(S.pJ) <= 4) do_ptask<4, true>(S, t, b0, N, Ash, M, lane);
                    else do_ptask<8, true>(S, t, b0, N, Ash, M, lane);
                } else do_ptask<JP, false>(S, t, b0, N, Ash, M, lane);
            }
        }
        if (ph + 1 < n_phases) grid_barrier(bar, gridDim.x);
    }
}

hipError_t launch_packed_persistent(const PSeg* segs, const PItemBlock* blocks, const PPhase* phases_host,
                                    const PPhase* phases_dev, int n_phases, int waves, int JP, size_t tab_doubles,
                                    size_t lds_wave, unsigned* bar, int n_cu, hipStream_t st) {
    if (n_phases <= 0) return hipSuccess;
    const size_t lds = (tab_doubles + lds_wave * (size_t)waves) * sizeof(double);
    if (lds > 64 * 1024) return hipErrorInvalidConfiguration;
    const void* fn = JP == 1 ? (const void*)k_pmulti<1>
                   : JP == 2 ? (const void*)k_pmulti<2>
                   : JP == 4 ? (const void*)k_pmulti<4>
                             : (const void*)k_pmulti<8>;
    const int threads = waves * kWave;
    int per_cu = 0;
    hipError_t err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
    if (err != hipSuccess) return err;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int64_t most = 1;
    for (int i = 0; i < n_phases; ++i) most = phases_host[i].n_blocks > most ? phases_host[i].n_blocks : most;
    int64_t grid = (int64_t)per_cu * n_cu;
    if (grid > most) grid = most;
    int nph = n_phases;
    int tabd = (int)tab_doubles;
    int lw = (int)lds_wave;
    void* args[] = {(void*)&segs, (void*)&blocks, (void*)&phases_dev, &nph, &tabd, &lw, (void*)&bar};
    err = hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(threads), args, (unsigned)lds, st);
    if (err != hipSuccess) return err;
    return hipGetLastError();
}

// X[i] = NaN for i < n when flag[0] != 0 (a persistent launch whose barrier timed out)
__global__ void k_poison_if(const unsigned* flag, double* X, int64_t n) {
    if (*flag == 0u) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        X[i] = __builtin_nan("");
}

hipError_t launch_poison_if(const unsigned* flag, double* X, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_poison_if, dim3(1), dim3(256), 0, st, flag, X, n);
    return hipGetLastError();
}

hipError_t launch_transpose_colours(const uint8_t* in, int64_t n, int B, uint8_t* out, hipStream_t st) {
    if (n <= 0 || B <= 0) return hipSuccess;
    const int64_t gx = (n + 63) / 64;
    const int gy = (B + 63) / 64;
    if (gx > 0x7FFFFFFF || gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_transpose_colours, dim3((unsigned)gx, (unsigned)gy), dim3(256), 0, st, in, n, B, out);
    return hipGetLastError();
}

// one block per 1024 vertices (every block reads 1024 x B values), at most 1024 blocks
int packed_reduce_blocks(int64_t n) {
    int64_t b = (n + 1023) / 1024;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

hipError_t launch_reduce_packed(const double* x, int64_t n, int B, double* partial, double* out, hipStream_t st) {
    if (B <= 0) return hipSuccess;
    const int blocks = packed_reduce_blocks(n);
    const int64_t per = (n + blocks - 1) / blocks;
    const int gy = (B + 63) / 64;
    if (gy > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reduce_packed_blocks, dim3(blocks, gy), dim3(256), 0, st, x, n, B, per, partial);
    hipLaunchKernelGGL(k_reduce_packed_final, dim3((B + 255) / 256), dim3(256), 0, st, (const double*)partial, blocks,
                       B, out);
    return hipGetLastError();
}

}  // namespace cc
