// GPU twin of inputs/gen.c: the same seeded R-MAT edge draws, built into the same sorted,
// symmetric, de-duplicated CSR directly in device memory (input side only; no colour-coding
// arithmetic). Used for graphs too large to build quickly on the host.
//
// Steps: count endpoint degrees of the draws (atomics), exclusive scan (host-provided offsets),
// scatter both directions, sort + de-duplicate every row (bitonic sort in LDS for rows of at most
// 4096 entries, a bitmap over the vertex range for longer rows), then compact into the final CSR.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

struct Params {
    int scale;
    int shift;
    uint64_t mask, p1, q1, p2, q2, seed;
    uint32_t ta, tb, tc;
};

__device__ __forceinline__ uint64_t perm(const Params& P, uint64_t x) {
    x = (x * P.p1 + P.q1) & P.mask;
    x ^= x >> P.shift;
    x = (x * P.p2 + P.q2) & P.mask;
    x ^= x >> P.shift;
    return x;
}

__device__ __forceinline__ bool draw(const Params& P, uint64_t e, uint32_t* src, uint32_t* dst) {
    const uint64_t base = mix64(P.seed + 0x9E3779B97F4A7C15ULL * (e + 1));
    uint64_t s = 0, d = 0;
    for (int l = 0; l < P.scale; ++l) {
        const uint32_t r = (uint32_t)(mix64(base + 0xD1B54A32D192ED03ULL * (uint64_t)(l + 1)) >> 32);
        const uint64_t bs = r >= P.tb ? 1 : 0;
        const uint64_t bd = ((r >= P.ta && r < P.tb) || r >= P.tc) ? 1 : 0;
        s = (s << 1) | bs;
        d = (d << 1) | bd;
    }
    s = perm(P, s);
    d = perm(P, d);
    *src = (uint32_t)s;
    *dst = (uint32_t)d;
    return s != d;
}

__global__ void k_count(Params P, uint64_t E, unsigned* deg) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t s, d;
        if (draw(P, e, &s, &d)) {
            atomicAdd(deg + s, 1u);
            atomicAdd(deg + d, 1u);
        }
    }
}

__global__ void k_scatter(Params P, uint64_t E, unsigned long long* cursor, uint32_t* raw) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < E; e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t s, d;
        if (draw(P, e, &s, &d)) {
            raw[atomicAdd(cursor + s, 1ull)] = d;
            raw[atomicAdd(cursor + d, 1ull)] = s;
        }
    }
}

// rows of at most 4096 entries: bitonic sort in LDS, then keep the first of each run
constexpr int kSmall = 4096;

__global__ __launch_bounds__(256) void k_sort_small(const int64_t* off, const int32_t* rows, int64_t n_rows,
                                                    uint32_t* raw, unsigned* uniq) {
    __shared__ uint32_t sh[kSmall];
    __shared__ unsigned cnt_sh;
    for (int64_t q = blockIdx.x; q < n_rows; q += gridDim.x) {
        const int v = rows[q];
        const int64_t b = off[v];
        const int len = (int)(off[v + 1] - b);
        int N = 1;
        while (N < len) N <<= 1;
        for (int i = threadIdx.x; i < N; i += blockDim.x) sh[i] = i < len ? raw[b + i] : 0xFFFFFFFFu;
        __syncthreads();
        for (int k = 2; k <= N; k <<= 1) {
            for (int j = k >> 1; j > 0; j >>= 1) {
                for (int i = threadIdx.x; i < N; i += blockDim.x) {
                    const int ixj = i ^ j;
                    if (ixj > i) {
                        const uint32_t a = sh[i], c = sh[ixj];
                        const bool up = (i & k) == 0;
                        if ((a > c) == up) {
                            sh[i] = c;
                            sh[ixj] = a;
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (threadIdx.x == 0) {
            unsigned u = 0;
            for (int i = 0; i < len; ++i)
                if (i == 0 || sh[i] != sh[i - 1]) raw[b + u++] = sh[i];
            cnt_sh = u;
        }
        __syncthreads();
        if (threadIdx.x == 0) uniq[v] = cnt_sh;
        __syncthreads();
    }
}

// long rows: one bitmap of n bits per row of the current group
__global__ void k_bitmap_set(const int64_t* off, const int32_t* rows, int n_rows, const uint32_t* raw,
                             uint32_t* bitmaps, int64_t words) {
    const int q = blockIdx.y;
    if (q >= n_rows) return;
    const int v = rows[q];
    const int64_t b = off[v], e = off[v + 1];
    uint32_t* bm = bitmaps + (int64_t)q * words;
    for (int64_t i = b + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < e; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = raw[i];
        atomicOr(bm + (x >> 5), 1u << (x & 31));
    }
}

// write the set bits of each row's bitmap back to the row in increasing order
__global__ __launch_bounds__(256) void k_bitmap_compact(const int64_t* off, const int32_t* rows, int n_rows,
                                                         uint32_t* raw, const uint32_t* bitmaps, int64_t words,
                                                         unsigned* uniq) {
    __shared__ unsigned part[256];
    const int q = blockIdx.x;
    if (q >= n_rows) return;
    const int v = rows[q];
    const int64_t b = off[v];
    const uint32_t* bm = bitmaps + (int64_t)q * words;
    const int64_t per = (words + 255) / 256;
    const int64_t w0 = threadIdx.x * per;
    const int64_t w1 = w0 + per < words ? w0 + per : words;
    unsigned c = 0;
    for (int64_t w = w0; w < w1; ++w) c += __popc(bm[w]);
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned acc = 0;
        for (int i = 0; i < 256; ++i) {
            const unsigned x = part[i];
            part[i] = acc;
            acc += x;
        }
        uniq[v] = acc;
    }
    __syncthreads();
    int64_t pos = b + part[threadIdx.x];
    for (int64_t w = w0; w < w1; ++w) {
        uint32_t bits = bm[w];
        while (bits) {
            const int t = __ffs(bits) - 1;
            bits &= bits - 1;
            raw[pos++] = (uint32_t)(w * 32 + t);
        }
    }
}

__global__ void k_compact(const int64_t* off, const int64_t* row_ptr, const uint32_t* raw, int64_t n, int32_t* col) {
    // one wavefront per row
    const int lane = threadIdx.x & 63;
    for (int64_t v = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; v < n;
         v += ((int64_t)gridDim.x * blockDim.x) >> 6) {
        const int64_t src = off[v], dst = row_ptr[v], len = row_ptr[v + 1] - row_ptr[v];
        for (int64_t i = lane; i < len; i += 64) col[dst + i] = (int32_t)raw[src + i];
    }
}

}  // namespace

extern "C" {

// host helpers (each returns hipError_t as int); all pointers are device pointers
int gen_gpu_count(int scale, uint64_t E, const uint64_t* k8, uint64_t seed, unsigned* deg, void* stream) {
    Params P;
    P.scale = scale;
    P.shift = (int)k8[7];
    P.mask = (1ULL << scale) - 1;
    P.ta = (uint32_t)k8[0]; P.tb = (uint32_t)k8[1]; P.tc = (uint32_t)k8[2];
    P.p1 = k8[3]; P.q1 = k8[4]; P.p2 = k8[5]; P.q2 = k8[6];
    P.seed = seed;
    hipLaunchKernelGGL(k_count, dim3(8192), dim3(256), 0, (hipStream_t)stream, P, E, deg);
    return (int)hipGetLastError();
}

int gen_gpu_scatter(int scale, uint64_t E, const uint64_t* k8, uint64_t seed, unsigned long long* cursor,
                    uint32_t* raw, void* stream) {
    Params P;
    P.scale = scale;
    P.shift = (int)k8[7];
    P.mask = (1ULL << scale) - 1;
    P.ta = (uint32_t)k8[0]; P.tb = (uint32_t)k8[1]; P.tc = (uint32_t)k8[2];
    P.p1 = k8[3]; P.q1 = k8[4]; P.p2 = k8[5]; P.q2 = k8[6];
    P.seed = seed;
    hipLaunchKernelGGL(k_scatter, dim3(8192), dim3(256), 0, (hipStream_t)stream, P, E, cursor, raw);
    return (int)hipGetLastError();
}

int gen_gpu_sort_small(const int64_t* off, const int32_t* rows, int64_t n_rows, uint32_t* raw, unsigned* uniq,
                       void* stream) {
    if (n_rows <= 0) return 0;
    const int64_t g = n_rows < 65536 * 4 ? n_rows : 65536 * 4;
    hipLaunchKernelGGL(k_sort_small, dim3((unsigned)g), dim3(256), 0, (hipStream_t)stream, off, rows, n_rows, raw, uniq);
    return (int)hipGetLastError();
}

int gen_gpu_sort_large(const int64_t* off, const int32_t* rows, int n_rows, uint32_t* raw, uint32_t* bitmaps,
                       int64_t words, unsigned* uniq, void* stream) {
    if (n_rows <= 0) return 0;
    hipLaunchKernelGGL(k_bitmap_set, dim3(64, (unsigned)n_rows), dim3(256), 0, (hipStream_t)stream, off, rows, n_rows,
                       raw, bitmaps, words);
    hipLaunchKernelGGL(k_bitmap_compact, dim3((unsigned)n_rows), dim3(256), 0, (hipStream_t)stream, off, rows, n_rows,
                       raw, bitmaps, words, uniq);
    return (int)hipGetLastError();
}

int gen_gpu_compact(const int64_t* off, const int64_t* row_ptr, const uint32_t* raw, int64_t n, int32_t* col,
                    void* stream) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_compact, dim3(16384), dim3(256), 0, (hipStream_t)stream, off, row_ptr, raw, n, col);
    return (int)hipGetLastError();
}

}  // extern "C"
