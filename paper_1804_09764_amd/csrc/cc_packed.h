// Device code of the packed layout: B colourings per table row.
//
// The B colourings of one batch are independent evaluations of the same split of Eq. 1
// (Section 2.1) on the same graph; Algorithm 1 runs them one after another. Storing them side by
// side, row v = [colouring b][entry], turns the narrow rows of small sub-templates into one wide,
// contiguous row per neighbour, reads each CSR entry once for all B colourings, and keeps the
// arithmetic of every colouring separate.
//
// A row tile holds the colourings [b0, b0 + nb). Its neighbour sum is kept over all k colours,
// C(k, p) entries per colouring, so that the passive entry j of a neighbour u goes to the
// full-space rank FM[col_b(u)][j], a map that does not depend on col_b(v). The combine reads
// N(v, Q) for the sets Q that avoid col_b(v) through E[col_b(v)][q], q being the rank of Q over the
// other k-1 colours, which is the index the split lists use. Entries whose set contains col_b(v)
// are neither loaded nor added (no term of the combine reads them).
//
// Summation order: every N entry receives its neighbours' terms in CSR order (one term per
// neighbour), so a colouring's counts do not depend on B, on the tile or on the other colourings
// of the batch. Cut rows use the same chunk partials and fixed-order chunk sums as the one-colouring
// layout.
#pragma once

#include "cc_device.h"
#include "cc_internal.h"

namespace cc {

// block-shared copies of the split's maps in LDS
struct PMaps {
    const uint32_t* sp;  // split list [pair][output] (a >= 2)
    const uint16_t* fm;  // FM[cu][j] (p >= 2)
    const uint16_t* em;  // E[cv][q]
};

// Colours of the 64 entries of a CSR block for the tile's colourings, staged in LDS:
// cs[i * bt + bl] = col_{b0 + bl}(u_i). Lane i copies the colours of its own entry, so a block's
// colours arrive in one round trip instead of one per entry. Every load of a lane is issued before
// its first store (loads past the tile's colourings re-read its last word and are not stored), and
// the words are held in plain registers: an array here would be placed in scratch memory.
typedef unsigned cc_u32x4 __attribute__((ext_vector_type(4)));

__device__ inline void stage_colours(const StepParams& S, int uvec, int cnt, int b0, int nb, uint8_t* cs, int lane) {
    wave_sync_lds();  // earlier reads of the stage are done
    if (lane < cnt) {
        const uint8_t* src = S.colour + (int64_t)uvec * S.B + b0;
        uint8_t* dst = cs + lane * S.bt;
        if (((S.B | b0 | nb | S.bt) & 15) == 0) {  // 16 colourings per load (nb <= 64)
            const int last = (nb >> 4) - 1;
            const cc_u32x4* s4 = reinterpret_cast<const cc_u32x4*>(src);
            cc_u32x4* d4 = reinterpret_cast<cc_u32x4*>(dst);
            const cc_u32x4 w0 = s4[0];
            const cc_u32x4 w1 = s4[last < 1 ? last : 1];
            const cc_u32x4 w2 = s4[last < 2 ? last : 2];
            const cc_u32x4 w3 = s4[last < 3 ? last : 3];
            d4[0] = w0;
            if (last >= 1) d4[1] = w1;
            if (last >= 2) d4[2] = w2;
            if (last >= 3) d4[3] = w3;
        } else if (((S.B | b0 | nb | S.bt) & 3) == 0) {  // four colourings per load
            const int last = (nb >> 2) - 1;
            const uint32_t* s1 = reinterpret_cast<const uint32_t*>(src);
            uint32_t* d1 = reinterpret_cast<uint32_t*>(dst);
            for (int q0 = 0; q0 <= last; q0 += 4) {
                const uint32_t w0 = s1[q0];
                const uint32_t w1 = s1[q0 + 1 <= last ? q0 + 1 : last];
                const uint32_t w2 = s1[q0 + 2 <= last ? q0 + 2 : last];
                const uint32_t w3 = s1[q0 + 3 <= last ? q0 + 3 : last];
                d1[q0] = w0;
                if (q0 + 1 <= last) d1[q0 + 1] = w1;
                if (q0 + 2 <= last) d1[q0 + 2] = w2;
                if (q0 + 3 <= last) d1[q0 + 3] = w3;
            }
        } else {
            for (int q = 0; q < nb; ++q) dst[q] = src[q];
        }
    }
    wave_sync_lds();
}

// active rows of v for the tile's colourings into LDS (a >= 2), eight loads in flight per lane;
// issued before the neighbour sum, whose closing barrier orders them before the combine
__device__ inline void pstage_a(const StepParams& S, int v, int b0, int nb, double* Ash, int lane) {
    if (S.a < 2) return;
    const double* arow = S.A + (int64_t)v * S.astride + (int64_t)b0 * S.Wa;
    const int na = nb * S.Wa;
    for (int i0 = 0; i0 < na; i0 += 8 * kWave) {
        double a8[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = i0 + q * kWave + lane;
            a8[q] = i < na ? arow[i] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int i = i0 + q * kWave + lane;
            if (i < na) Ash[i] = a8[q];
        }
    }
}

// rows of entries [g D, g D + D) of a block in flight: values and N targets (-1: nothing to add)
template <int J, int D>
__device__ __forceinline__ void pload(const StepParams& S, int g, int cnt, int uvec, const uint8_t* cs, const int (&bl)[J],
                                      const int16_t* tg, const double* Pt, double (&X)[D][J], int (&F)[D][J], int lane) {
    const int k = S.k;
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const int i = g * D + q;
        const bool live = i < cnt;
        const int u = bcast(uvec, live ? i : 0);
#pragma unroll
        for (int t = 0; t < J; ++t) {
            const int cu = live ? (int)cs[i * S.bt + bl[t]] : 255;
            F[q][t] = cu < k ? (int)tg[(t * k + cu) * kWave + lane] : -1;
            X[q][t] = F[q][t] >= 0 ? Pt[(int64_t)u * S.pstride + kWave * t] : 0.0;
        }
    }
}

// N[F] += X for the group, in (entry, element) order. An LDS add without return (ds_add_f64) keeps
// the wavefront from waiting on a read of N; a wavefront's LDS operations complete in issue order
// and the targets of one instruction are distinct, so every entry still receives its terms in
// CSR order.
template <int J, int D>
__device__ __forceinline__ void padd(double* N, const double (&X)[D][J], const int (&F)[D][J]) {
#pragma unroll
    for (int q = 0; q < D; ++q)
#pragma unroll
        for (int t = 0; t < J; ++t)
            if (F[q][t] >= 0) __hip_atomic_fetch_add(N + F[q][t], X[q][t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// neighbour sum of CSR entries [beg, end) for the tile's colourings, p >= 2; cvrow = col_b(v) for
// the tile's colourings, fml = FM in LDS, tg = this wavefront's target table (J * k * 64 entries),
// cs = its colour stage (64 * bt bytes)
template <int J>
__device__ void pgather(const StepParams& S, int64_t beg, int64_t end, const uint8_t* cvrow, int b0, int nb,
                        double* N, const uint16_t* fml, int16_t* tg, uint8_t* cs, int lane) {
    constexpr int D = 8 / J;  // entries per group; two groups (16 loads per lane) are in flight
    const int k = S.k, Wp = S.Wp, Cf = S.Cf;
    const int E = nb * Wp;
    for (int c0 = 0; c0 < E; c0 += kWave * J) {
        // element f = c0 + lane + 64 t of the tile is (colouring b0 + bl, passive entry jj). Its
        // N target for a neighbour of colour c depends only on c: tabulate it per lane,
        // tg[(t k + c) 64 + lane] = bl Cf + FM[c][jj], or -1 when the entry is of no use to v
        // (c = col_b(v), or the entry's set holds col_b(v), or v has no valid colour)
        int bl[J];
#pragma unroll
        for (int t = 0; t < J; ++t) {
            const int f = c0 + lane + kWave * t;
            const bool ok = f < E;
            bl[t] = ok ? f / Wp : 0;
            const int jj = ok ? f - bl[t] * Wp : 0;
            const int cv = ok ? (int)cvrow[bl[t]] : 255;
            const int msk = ok ? (int)S.mask[jj] : 0xFFFF;
            for (int c = 0; c < k; ++c) {
                const bool valid = cv < k && c != cv;
                const int xpos = valid ? cv - (cv > c ? 1 : 0) : 0;
                const bool need = valid && ((msk >> xpos) & 1) == 0;
                tg[(t * k + c) * kWave + lane] = need ? (int16_t)(bl[t] * Cf + (int)fml[c * Wp + jj]) : (int16_t)-1;
            }
        }
        const double* Pt = S.P + (int64_t)b0 * Wp + c0 + lane;
        for (int64_t e0 = beg; e0 < end; e0 += kWave) {
            const int64_t e = e0 + lane;
            const int uvec = e < end ? S.col[e] : 0;
            const int cnt = (end - e0 < kWave) ? (int)(end - e0) : kWave;
            stage_colours(S, uvec, cnt, b0, nb, cs, lane);
            const int ng = (cnt + D - 1) / D;
            double XA[D][J], XB[D][J];
            int FA[D][J], FB[D][J];
            pload<J, D>(S, 0, cnt, uvec, cs, bl, tg, Pt, XA, FA, lane);
            for (int g = 0; g < ng; g += 2) {
                if (g + 1 < ng) pload<J, D>(S, g + 1, cnt, uvec, cs, bl, tg, Pt, XB, FB, lane);
                padd<J, D>(N, XA, FA);
                if (g + 1 >= ng) break;
                if (g + 2 < ng) pload<J, D>(S, g + 2, cnt, uvec, cs, bl, tg, Pt, XA, FA, lane);
                padd<J, D>(N, XB, FB);
            }
        }
    }
}

// p = 1: N[bl * k + c] += number of entries in [beg, end) whose colour under colouring b0 + bl is c
template <int J>
__device__ void pcount(const StepParams& S, int64_t beg, int64_t end, int b0, int nb, double* N, uint8_t* cs,
                       int lane) {
    const int k = S.k, Cf = S.Cf;
    const int E = nb * k;
    for (int c0 = 0; c0 < E; c0 += kWave * J) {
        int bl[J], ct[J];
        unsigned cnt_t[J];
#pragma unroll
        for (int t = 0; t < J; ++t) {
            const int f = c0 + lane + kWave * t;
            const bool ok = f < E;
            bl[t] = ok ? f / k : 0;
            ct[t] = ok ? f - bl[t] * k : 255;
            cnt_t[t] = 0;
        }
        for (int64_t e0 = beg; e0 < end; e0 += kWave) {
            const int64_t e = e0 + lane;
            const int uvec = e < end ? S.col[e] : 0;
            const int cnt = (end - e0 < kWave) ? (int)(end - e0) : kWave;
            stage_colours(S, uvec, cnt, b0, nb, cs, lane);
            for (int i = 0; i < cnt; ++i)
#pragma unroll
                for (int t = 0; t < J; ++t) cnt_t[t] += ((int)cs[i * S.bt + bl[t]] == ct[t]) ? 1u : 0u;
        }
#pragma unroll
        for (int t = 0; t < J; ++t)
            if (c0 + lane + kWave * t < E) N[bl[t] * Cf + ct[t]] += (double)cnt_t[t];
    }
}

// output rows of v for the tile's colourings from N and v's active rows (both in LDS)
__device__ inline void pcombine(const StepParams& S, int v, const uint8_t* cvrow, int b0, int nb, const double* N,
                                double* Ash, const PMaps& M, int lane) {
    const uint16_t* eml = M.em;
    const int k = S.k, Ws = S.Ws, Cf = S.Cf, Nw = S.Nw;
    double* orow = S.O + (int64_t)v * S.ostride + (int64_t)b0 * Ws;
    const int E = nb * Ws;
    if (S.a == 1) {
        // T' is the single vertex v: C(v, T, .) = N(v, .) (here Ws = Nw)
        for (int f = lane; f < E; f += kWave) {
            const int bl = f / Ws, r = f - bl * Ws;
            const int cv = cvrow[bl];
            orow[f] = cv < k ? N[bl * Cf + eml[cv * Nw + r]] : 0.0;
        }
        return;
    }
    // the active rows are already in Ash (pstage_a)
    for (int f = lane; f < E; f += kWave) {
        const int bl = f / Ws, r = f - bl * Ws;
        const int cv = cvrow[bl];
        double sum = 0.0;
        if (cv < k) {
            const double* Ab = Ash + bl * S.Wa;
            const double* Nb = N + bl * Cf;
            const uint16_t* eb = eml + cv * Nw;
            const uint32_t* sp = M.sp + r;
            sum = blocked_sum(S.npairs, [&](int j) {
                const uint32_t pr = sp[(int64_t)j * Ws];
                return Ab[pr & 0xFFFFu] * Nb[eb[pr >> 16]];
            });
        }
        orow[f] = sum;
    }
}

// P1: the split's passive part is a single vertex (p = 1)
template <int J, bool P1>
__device__ __forceinline__ void pneighbours(const StepParams& S, int64_t beg, int64_t end, const uint8_t* cvrow, int b0,
                                            int nb, double* N, const PMaps& M, int lane) {
    const uint16_t* fml = M.fm;
    uint8_t* cs = reinterpret_cast<uint8_t*>(N + S.cs_off);
    if constexpr (P1) pcount<J>(S, beg, end, b0, nb, N, cs, lane);
    else pgather<J>(S, beg, end, cvrow, b0, nb, N, fml, reinterpret_cast<int16_t*>(N + S.tg_off), cs, lane);
}

// colouring tiles of a row: the work items of a packed split are (task, tile) and (cut row, tile)
// pairs, so that the tiles of one task run on different wavefronts
__device__ __forceinline__ int ptiles(const StepParams& S) { return (S.B + S.bt - 1) / S.bt; }

// light row v, colourings [b0, b0 + nb): neighbour sum, then the combine
template <int J, bool P1>
__device__ void plight_row(const StepParams& S, int v, int b0, int nb, double* N, double* Ash, const PMaps& M,
                           int lane) {
    const int64_t beg = S.row_ptr[v];
    const int64_t end = S.row_ptr[v + 1];
    const uint8_t* cvrow = S.colour + (int64_t)v * S.B + b0;
    pstage_a(S, v, b0, nb, Ash, lane);
    for (int i = lane; i < nb * S.Cf; i += kWave) N[i] = 0.0;
    wave_sync_lds();
    if (beg < end) pneighbours<J, P1>(S, beg, end, cvrow, b0, nb, N, M, lane);
    wave_sync_lds();
    pcombine(S, v, cvrow, b0, nb, N, Ash, M, lane);
    wave_sync_lds();
}

// colourings [b0, b0 + bt) of task t: a chunk of a cut row (partial rows to scratch) or a range
// of light rows
template <int J, bool P1>
__device__ void do_ptask(const StepParams& S, int64_t t, int b0, double* N, double* Ash, const PMaps& M, int lane) {
    const int nb = (S.B - b0 < S.bt) ? S.B - b0 : S.bt;
    if (t < S.n_chunks) {
        const ChunkItem ch = S.chunks[t];
        const int v = __builtin_amdgcn_readfirstlane(ch.v);
        double* prow = S.partial + t * S.nstride + (int64_t)b0 * S.Cf;
        for (int i = lane; i < nb * S.Cf; i += kWave) N[i] = 0.0;
        wave_sync_lds();
        pneighbours<J, P1>(S, ch.beg, ch.beg + ch.len, S.colour + (int64_t)v * S.B + b0, b0, nb, N, M, lane);
        wave_sync_lds();
        for (int i = lane; i < nb * S.Cf; i += kWave) prow[i] = N[i];
        wave_sync_lds();
    } else {
        const int64_t r = t - S.n_chunks;
        const int i0 = S.light_start[r], i1 = S.light_start[r + 1];
        for (int i = i0; i < i1; ++i) plight_row<J, P1>(S, S.light[i], b0, nb, N, Ash, M, lane);
    }
}

// colourings [b0, b0 + bt) of cut row t: the row's chunk partials added in the fixed blocked order,
// then the combine
__device__ inline void do_phub(const StepParams& S, int64_t t, int b0, double* N, double* Ash, const PMaps& M,
                               int lane) {
    const HubItem h = S.hubs[t];
    const int nb = (S.B - b0 < S.bt) ? S.B - b0 : S.bt;
    pstage_a(S, h.v, b0, nb, Ash, lane);
    for (int i = lane; i < nb * S.Cf; i += kWave) {
        const double* pp = S.partial + h.first_chunk * S.nstride + (int64_t)b0 * S.Cf + i;
        N[i] = blocked_sum(h.n_chunks, [&](int c) { return pp[(int64_t)c * S.nstride]; });
    }
    wave_sync_lds();
    pcombine(S, h.v, S.colour + (int64_t)h.v * S.B + b0, b0, nb, N, Ash, M, lane);
    wave_sync_lds();
}

// block-shared maps, copied from the plan constants: the split list (a >= 2, u32), then FM
// (p >= 2) and E (u16)
__device__ inline PMaps stage_maps(const StepParams& S, void* lds) {
    uint32_t* sp = reinterpret_cast<uint32_t*>(lds);
    const int nsp = S.a >= 2 ? S.npairs * S.Ws : 0;
    uint16_t* fm = reinterpret_cast<uint16_t*>(sp + nsp);
    const int nfm = S.p >= 2 ? S.k * S.Wp : 0;
    uint16_t* em = fm + nfm;
    for (int i = threadIdx.x; i < nsp; i += blockDim.x) sp[i] = S.split[i];
    for (int i = threadIdx.x; i < nfm; i += blockDim.x) fm[i] = S.fullmap[i];
    for (int i = threadIdx.x; i < S.k * S.Nw; i += blockDim.x) em[i] = S.emap[i];
    return PMaps{sp, fm, em};
}

}  // namespace cc
