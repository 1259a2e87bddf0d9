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

// neighbour sum of CSR entries [beg, end) for the tile's colourings, p >= 2; cvrow = col_b(v) for
// the tile's colourings, fml = FM in LDS
template <int J>
__device__ void pgather(const StepParams& S, int64_t beg, int64_t end, const uint8_t* cvrow, int b0, int nb,
                        double* N, const uint16_t* fml, int lane) {
    constexpr int D = (J >= 8) ? 2 : 4;  // neighbours in flight per wavefront
    const int k = S.k, Wp = S.Wp, B = S.B, Cf = S.Cf;
    const int E = nb * Wp;
    const uint8_t* cp = S.colour + b0;
    for (int c0 = 0; c0 < E; c0 += kWave * J) {
        // element f = c0 + lane + 64 t of the tile: colouring b0 + bl, passive entry jj
        int bl[J], jj[J], cvt[J], msk[J];
#pragma unroll
        for (int t = 0; t < J; ++t) {
            const int f = c0 + lane + kWave * t;
            const bool ok = f < E;
            bl[t] = ok ? f / Wp : 0;
            jj[t] = ok ? f - bl[t] * Wp : 0;
            const int c = ok ? (int)cvrow[bl[t]] : 255;
            cvt[t] = c < k ? c : 255;  // 255: no valid colour, the element never contributes
            msk[t] = ok ? (int)S.mask[jj[t]] : 0xFFFF;
        }
        const double* Pt = S.P + (int64_t)b0 * Wp + c0 + lane;
        for (int64_t e0 = beg; e0 < end; e0 += kWave) {
            const int64_t e = e0 + lane;
            const int uvec = e < end ? S.col[e] : 0;
            const int cnt = (end - e0 < kWave) ? (int)(end - e0) : kWave;
            for (int i = 0; i < cnt; i += D) {
                int cb[D], uq[D];
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const bool live = i + q < cnt;
                    uq[q] = bcast(uvec, live ? i + q : 0);
                    cb[q] = (live && lane < nb) ? (int)cp[(int64_t)uq[q] * B + lane] : 255;
                }
                double x[D][J];
                int dst[D][J];
#pragma unroll
                for (int q = 0; q < D; ++q)
#pragma unroll
                    for (int t = 0; t < J; ++t) {
                        const int cu = __shfl(cb[q], bl[t]);
                        const bool valid = cu < k && cvt[t] < k && cu != cvt[t];
                        const int xpos = valid ? cvt[t] - (cvt[t] > cu ? 1 : 0) : 0;
                        const bool need = valid && ((msk[t] >> xpos) & 1) == 0;
                        dst[q][t] = need ? bl[t] * Cf + (int)fml[cu * Wp + jj[t]] : -1;
                        x[q][t] = need ? Pt[(int64_t)uq[q] * S.pstride + kWave * t] : 0.0;
                    }
#pragma unroll
                for (int q = 0; q < D; ++q)
#pragma unroll
                    for (int t = 0; t < J; ++t)
                        if (dst[q][t] >= 0) N[dst[q][t]] += x[q][t];
            }
        }
    }
}

// p = 1: N[bl * k + c] += number of entries in [beg, end) whose colour under colouring b0 + bl is c
template <int J>
__device__ void pcount(const StepParams& S, int64_t beg, int64_t end, int b0, int nb, double* N, int lane) {
    constexpr int D = 4;
    const int k = S.k, B = S.B, Cf = S.Cf;
    const int E = nb * k;
    const uint8_t* cp = S.colour + b0;
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
            for (int i = 0; i < cnt; i += D) {
                int cb[D];
#pragma unroll
                for (int q = 0; q < D; ++q) {
                    const bool live = i + q < cnt;
                    const int u = bcast(uvec, live ? i + q : 0);
                    cb[q] = (live && lane < nb) ? (int)cp[(int64_t)u * B + lane] : 255;
                }
#pragma unroll
                for (int q = 0; q < D; ++q)
#pragma unroll
                    for (int t = 0; t < J; ++t) cnt_t[t] += (__shfl(cb[q], bl[t]) == ct[t]) ? 1u : 0u;
            }
        }
#pragma unroll
        for (int t = 0; t < J; ++t)
            if (c0 + lane + kWave * t < E) N[bl[t] * Cf + ct[t]] += (double)cnt_t[t];
    }
}

// output rows of v for the tile's colourings from N (LDS) and v's active rows
__device__ inline void pcombine(const StepParams& S, int v, const uint8_t* cvrow, int b0, int nb, const double* N,
                                double* Ash, const uint16_t* eml, int lane) {
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
    const double* arow = S.A + (int64_t)v * S.astride + (int64_t)b0 * S.Wa;
    for (int i = lane; i < nb * S.Wa; i += kWave) Ash[i] = arow[i];
    wave_sync_lds();
    for (int f = lane; f < E; f += kWave) {
        const int bl = f / Ws, r = f - bl * Ws;
        const int cv = cvrow[bl];
        double sum = 0.0;
        if (cv < k) {
            const double* Ab = Ash + bl * S.Wa;
            const double* Nb = N + bl * Cf;
            const uint16_t* eb = eml + cv * Nw;
            const uint32_t* sp = S.split + r;
            for (int j = 0; j < S.npairs; ++j) {
                const uint32_t pr = sp[(int64_t)j * Ws];
                sum += Ab[pr & 0xFFFFu] * Nb[eb[pr >> 16]];
            }
        }
        orow[f] = sum;
    }
}

template <int J>
__device__ __forceinline__ void pneighbours(const StepParams& S, int64_t beg, int64_t end, const uint8_t* cvrow, int b0,
                                            int nb, double* N, const uint16_t* fml, int lane) {
    if (S.p == 1) pcount<J>(S, beg, end, b0, nb, N, lane);
    else pgather<J>(S, beg, end, cvrow, b0, nb, N, fml, lane);
}

template <int J>
__device__ void plight_row(const StepParams& S, int v, double* N, double* Ash, const uint16_t* fml,
                           const uint16_t* eml, int lane) {
    const int64_t beg = S.row_ptr[v];
    const int64_t end = S.row_ptr[v + 1];
    const uint8_t* cvall = S.colour + (int64_t)v * S.B;
    for (int b0 = 0; b0 < S.B; b0 += S.bt) {
        const int nb = (S.B - b0 < S.bt) ? S.B - b0 : S.bt;
        for (int i = lane; i < nb * S.Cf; i += kWave) N[i] = 0.0;
        wave_sync_lds();
        if (beg < end) pneighbours<J>(S, beg, end, cvall + b0, b0, nb, N, fml, lane);
        wave_sync_lds();
        pcombine(S, v, cvall + b0, b0, nb, N, Ash, eml, lane);
        wave_sync_lds();
    }
}

// task t: a chunk of a cut row (partial rows of all colourings to scratch) or a range of light rows
template <int J>
__device__ void do_ptask(const StepParams& S, int64_t t, double* N, double* Ash, const uint16_t* fml,
                         const uint16_t* eml, int lane) {
    if (t < S.n_chunks) {
        const ChunkItem ch = S.chunks[t];
        const int v = __builtin_amdgcn_readfirstlane(ch.v);
        const uint8_t* cvall = S.colour + (int64_t)v * S.B;
        double* prow = S.partial + t * S.nstride;
        for (int b0 = 0; b0 < S.B; b0 += S.bt) {
            const int nb = (S.B - b0 < S.bt) ? S.B - b0 : S.bt;
            for (int i = lane; i < nb * S.Cf; i += kWave) N[i] = 0.0;
            wave_sync_lds();
            pneighbours<J>(S, ch.beg, ch.beg + ch.len, cvall + b0, b0, nb, N, fml, lane);
            wave_sync_lds();
            for (int i = lane; i < nb * S.Cf; i += kWave) prow[(int64_t)b0 * S.Cf + i] = N[i];
            wave_sync_lds();
        }
    } else {
        const int64_t r = t - S.n_chunks;
        const int i0 = S.light_start[r], i1 = S.light_start[r + 1];
        for (int i = i0; i < i1; ++i) plight_row<J>(S, S.light[i], N, Ash, fml, eml, lane);
    }
}

// cut row t: chunk partials added in chunk order, then the combine
__device__ inline void do_phub(const StepParams& S, int64_t t, double* N, double* Ash, const uint16_t* eml, int lane) {
    const HubItem h = S.hubs[t];
    const uint8_t* cvall = S.colour + (int64_t)h.v * S.B;
    for (int b0 = 0; b0 < S.B; b0 += S.bt) {
        const int nb = (S.B - b0 < S.bt) ? S.B - b0 : S.bt;
        for (int i = lane; i < nb * S.Cf; i += kWave) {
            double sum = 0.0;
            const double* pp = S.partial + h.first_chunk * S.nstride + (int64_t)b0 * S.Cf + i;
            for (int c = 0; c < h.n_chunks; ++c) sum += pp[(int64_t)c * S.nstride];
            N[i] = sum;
        }
        wave_sync_lds();
        pcombine(S, h.v, cvall + b0, b0, nb, N, Ash, eml, lane);
        wave_sync_lds();
    }
}

// block-shared maps: FM (p >= 2) then E, copied from the plan constants
__device__ inline void stage_maps(const StepParams& S, uint16_t* tab) {
    const int nfm = S.p >= 2 ? S.k * S.Wp : 0;
    for (int i = threadIdx.x; i < nfm; i += blockDim.x) tab[i] = S.fullmap[i];
    for (int i = threadIdx.x; i < S.k * S.Nw; i += blockDim.x) tab[nfm + i] = S.emap[i];
}

}  // namespace cc
