// HIP kernels of the colour-coding hot path (gfx950, wave64).
//
// One split of the dynamic program (Section 2.1, Eq. 1) is evaluated in its distributive form:
//
//   N(v, Q)  = sum_{u in N(v)} C(u, T'', Q)                         neighbour sum, |Q| = p
//   C(v,T,S) = sum_{S1 subset S, |S1| = a} C(v, T', S1) * N(v, S \ S1)   combine
//
// which regroups the double sum of Eq. 1 (the neighbour loop moves inside, next to the passive
// factor, because C(v, T', S1) does not depend on u).
//
// Tables use the colour-anchored layout: a sub-template's count C(v, T_i, S) is zero unless
// col(v) is in S (the root of T_i sits on v), so row v stores only the sets containing col(v),
// one entry per set S \ {col(v)} over the k-1 other colours renumbered 0..k-2. Rows of up to 16
// entries keep colex order; longer rows are stored with 128-byte lines of sets that share a
// common subset (the planner's storage order), and the plan's maps are written for that order.
// The neighbour sum N is indexed by colex rank. A neighbour u's passive row is written over the
// colours other than col(u); the fold map M[col(u)][col(v)][j] moves its entry j to the index of
// the same set over the colours other than col(v) (or drops it when the set contains col(v),
// which no term of the combine can use). Neighbours with col(u) = col(v) contribute nothing and
// are skipped.
//
// Work split (the neighbour-list partitioning of Section 3.3, Algorithm 4, on wavefronts): every
// row of at most `hub_threshold` entries is one work item processed by one wavefront; longer rows
// are cut into chunks of `chunk` entries whose partial neighbour sums go to scratch and are added
// in a fixed blocked order by a second kernel, so every entry has one fixed summation order (no atomics on
// counts). Light rows are grouped into ranges of about `chunk` entries (at most 64 rows); chunks and
// ranges are dealt round-robin to persistent wavefronts.
#include <hip/hip_runtime.h>

#include "cc_internal.h"
#include "cc_device.h"

namespace cc {

// Neighbour sum of one CSR segment into N[0..Nw) (LDS), p >= 2.
//
// The segment is read in blocks of 64 entries. The usable neighbours of a block (colour valid and
// different from col(v)) are sorted by (colour, position) with a lane permutation, then streamed
// through two register batches of D rows each: the rows of batch b+1 are in flight while batch b
// is added. Consecutive members of one colour are summed in registers (in member order) and folded
// into N through the fold map once per colour and block; the fold-map entries of a colour are
// loaded together with the row of its first member. Fold-map entries and colour-set masks are
// 16-bit; up to eight columns per lane each register holds those of two columns (t and t + 1):
// fewer registers per wavefront, more wavefronts per SIMD, more rows in flight. At sixteen columns
// the packed form was measured slower (two wavefronts per SIMD either way), so it keeps one per
// register.
template <int J>
struct Idx16 {
    static constexpr bool kPack = J <= 8;
    static constexpr int kWords = kPack ? (J + 1) / 2 : J;
    uint32_t w[kWords];
    __device__ __forceinline__ int get(int t) const {
        if constexpr (kPack) return (int)((w[t >> 1] >> (16 * (t & 1))) & 0xFFFFu);
        else return (int)w[t];
    }
    // columns are put in increasing t; in the packed form an even t starts its register
    __device__ __forceinline__ void put(int t, uint32_t v) {
        if constexpr (kPack) w[t >> 1] = (t & 1) ? (w[t >> 1] | (v << 16)) : v;
        else w[t] = v;
    }
    __device__ __forceinline__ void fill(uint32_t v) {
#pragma unroll
        for (int t = 0; t < J; ++t) put(t, v);
    }
};

// Slot of centre colour cv among the colours of a projected pass (0 outside projected passes,
// where class_stride is 0).
__device__ __forceinline__ int class_slot(const StepParams& S, int cv) {
    return __popc(S.cls_mask & ((1u << cv) - 1u));
}

// Whether this launch processes a row whose centre has colour cv (rows of colours >= k only write
// zeros and belong to the launch that holds kAnyInvalid).
__device__ __forceinline__ bool class_in(const StepParams& S, int cv) {
    return cv < S.k ? ((S.cls_mask >> cv) & 1u) != 0 : (S.cls_mask & kAnyInvalid) != 0;
}

template <int J, int D>
__device__ __forceinline__ void load_batch(const StepParams& S, const double* Pb, int b, int cnt, int su, int sc,
                                           int c0, int cv, int lane, const Idx16<J>& msk, double (&X)[D][J],
                                           Idx16<J> (&F)[D]) {
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const int i = b * D + q;
        if (i < cnt) {
            const int ui = bcast(su, i);
            const int ci = bcast(sc, i);
            // position of col(v) among the colours other than col(u): entries whose set holds it
            // are dropped by the fold, so they are not loaded (whole cache lines are skipped)
            const int x = cv - (cv > ci ? 1 : 0);
            const double* row = Pb + (int64_t)ui * S.pstride + c0;
#pragma unroll
            for (int t = 0; t < J; ++t) {
                const bool need = ((msk.get(t) >> x) & 1) == 0;
                X[q][t] = need ? row[lane + kWave * t] : 0.0;
            }
            const bool first = (i == 0) || (ci != bcast(sc, i > 0 ? i - 1 : 0));
            if (first) {
                const uint16_t* fm = S.fold + ((int64_t)ci * S.k + cv) * S.Wp + c0;
#pragma unroll
                for (int t = 0; t < J; ++t) {
                    const int j = c0 + lane + kWave * t;
                    F[q].put(t, (j < S.Wp) ? (uint32_t)fm[lane + kWave * t] : (uint32_t)kNoSlot);
                }
            }
        }
    }
}

template <int J>
__device__ __forceinline__ void fold_acc(double* N, const double (&acc)[J], const Idx16<J>& f) {
    // wide rows: one LDS add per entry (ds_add_f64, no read back; a wavefront's LDS operations
    // complete in issue order and one colour's targets are distinct, so each entry's order is
    // unchanged); narrow rows: read, add, write (measured faster there)
#pragma unroll
    for (int t = 0; t < J; ++t) {
        const int ft = f.get(t);
        if (ft != (int)kNoSlot) {
            if constexpr (J >= 4) __hip_atomic_fetch_add(N + ft, acc[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
            else N[ft] += acc[t];
        }
    }
}

template <int J, int D>
__device__ __forceinline__ void consume_batch(int b, int cnt, int sc, int& cur, double* N, double (&acc)[J],
                                              Idx16<J>& fcur, const double (&X)[D][J], const Idx16<J> (&F)[D]) {
#pragma unroll
    for (int q = 0; q < D; ++q) {
        const int i = b * D + q;
        if (i < cnt) {
            const int ci = bcast(sc, i);
            if (ci != cur) {
                if (cur >= 0) fold_acc<J>(N, acc, fcur);
                cur = ci;
                fcur = F[q];
#pragma unroll
                for (int t = 0; t < J; ++t) acc[t] = X[q][t];
            } else {
#pragma unroll
                for (int t = 0; t < J; ++t) acc[t] += X[q][t];
            }
        }
    }
}

template <int J>
__device__ void gather_fold(const StepParams& S, int64_t beg, int64_t end, int cv, double* N, int lane) {
    // rows per batch (two batches in flight): from 4 doubles per lane one row, which keeps the
    // 4-double variant at five wavefronts per SIMD (two rows: four, and 8 % slower)
    constexpr int D = (J >= 4) ? 1 : 4;
    const int k = S.k;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // the passive rows: the table itself, or in a projected pass the copy for this centre colour
    const double* Pb = S.P + (int64_t)class_slot(S, cv) * S.class_stride;
    for (int c0 = 0; c0 < S.Wp; c0 += kWave * J) {
        // colour-set masks of this lane's columns; columns past the row get an all-ones mask,
        // which marks them as never needed
        Idx16<J> msk;
#pragma unroll
        for (int t = 0; t < J; ++t) {
            const int j = c0 + lane + kWave * t;
            msk.put(t, (j < S.Wp) ? (uint32_t)S.mask[j] : 0xFFFFu);
        }
        for (int64_t e0 = beg; e0 < end; e0 += kWave) {
            const int64_t e = e0 + lane;
            const bool valid = e < end;
            const int u = valid ? S.col[e] : 0;
            const int cu = valid ? (int)(S.ecol ? S.ecol[e] : S.colour[(int64_t)u * S.cstride]) : 255;
            const bool use = valid && cu < k && cu != cv;
            const uint64_t used = __ballot(use);
            const int cnt = __popcll((unsigned long long)used);
            if (cnt == 0) continue;
            // position of this lane in (colour, lane) order; unused lanes go after the used ones
            int rank = use ? 0 : cnt + __popcll((unsigned long long)(~used & below));
            for (int c = 0; c < k; ++c) {
                const uint64_t bc = __ballot(use && cu == c);
                if (use && cu > c) rank += __popcll((unsigned long long)bc);
                if (use && cu == c) rank += __popcll((unsigned long long)(bc & below));
            }
            const int su = __builtin_amdgcn_ds_permute(rank << 2, u);
            const int sc = __builtin_amdgcn_ds_permute(rank << 2, cu);
            double acc[J];
            Idx16<J> fcur;
            double XA[D][J], XB[D][J];
            Idx16<J> FA[D], FB[D];
#pragma unroll
            for (int t = 0; t < J; ++t) acc[t] = 0.0;
            fcur.fill(kNoSlot);
#pragma unroll
            for (int q = 0; q < D; ++q) {
                FA[q].fill(kNoSlot);
                FB[q].fill(kNoSlot);
            }
            int cur = -1;
            const int nb = (cnt + D - 1) / D;
            load_batch<J, D>(S, Pb, 0, cnt, su, sc, c0, cv, lane, msk, XA, FA);
            for (int b = 0; b < nb; b += 2) {
                if (b + 1 < nb) load_batch<J, D>(S, Pb, b + 1, cnt, su, sc, c0, cv, lane, msk, XB, FB);
                consume_batch<J, D>(b, cnt, sc, cur, N, acc, fcur, XA, FA);
                if (b + 1 >= nb) break;
                if (b + 2 < nb) load_batch<J, D>(S, Pb, b + 2, cnt, su, sc, c0, cv, lane, msk, XA, FA);
                consume_batch<J, D>(b + 1, cnt, sc, cur, N, acc, fcur, XB, FB);
            }
            fold_acc<J>(N, acc, fcur);
        }
    }
}

// Neighbour sum for narrow passive rows (Wp <= G <= 32): G lanes per row, so 64/G rows per load
// instruction. The usable neighbours of a 64-entry block are sorted by colour as in gather_fold and
// all of their rows are loaded at once and staged in LDS; each colour run is then summed column by
// column in member order and folded into N in colour order, which is exactly gather_fold's
// arithmetic (same order, same fold), so results do not depend on which of the two paths ran. Each lane keeps the
// fold-map entries of its column for the colours of its slot (slot, slot + 64/G, ...).
template <int G>
__device__ void gather_fold_narrow(const StepParams& S, int64_t beg, int64_t end, int cv, double* N, double* stage,
                                   int lane) {
    constexpr int R = kWave / G;         // rows per load instruction
    constexpr int Q = G;                 // load instructions per block of 64 members
    constexpr int NC = (kMaxK + R - 1) / R;
    const int k = S.k;
    const int g = lane / G;
    const int j = lane % G;
    const bool colok = j < S.Wp;
    const int mskj = colok ? (int)S.mask[j] : 0xFFFF;
    int fidx[NC];
#pragma unroll
    for (int m = 0; m < NC; ++m) {
        const int c = g + m * R;
        fidx[m] = (colok && c < k && c != cv) ? (int)S.fold[((int64_t)c * k + cv) * S.Wp + j] : (int)kNoSlot;
    }
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const double* Pb = S.P + (int64_t)class_slot(S, cv) * S.class_stride;
    for (int64_t e0 = beg; e0 < end; e0 += kWave) {
        const int64_t e = e0 + lane;
        const bool valid = e < end;
        const int u = valid ? S.col[e] : 0;
        const int cu = valid ? (int)(S.ecol ? S.ecol[e] : S.colour[(int64_t)u * S.cstride]) : 255;
        const bool use = valid && cu < k && cu != cv;
        const uint64_t used = __ballot(use);
        const int cnt = __popcll((unsigned long long)used);
        if (cnt == 0) continue;
        int rank = use ? 0 : cnt + __popcll((unsigned long long)(~used & below));
        for (int c = 0; c < k; ++c) {
            const uint64_t bc = __ballot(use && cu == c);
            if (use && cu > c) rank += __popcll((unsigned long long)bc);
            if (use && cu == c) rank += __popcll((unsigned long long)(bc & below));
        }
        const int su = __builtin_amdgcn_ds_permute(rank << 2, u);
        const int sc = __builtin_amdgcn_ds_permute(rank << 2, cu);
        double x[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int i = q * R + g;
            const int uq = __shfl(su, i);
            const int cq = __shfl(sc, i);
            const int xpos = cv - (cv > cq ? 1 : 0);
            const bool need = i < cnt && ((mskj >> xpos) & 1) == 0;
            x[q] = need ? Pb[(int64_t)uq * S.pstride + j] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < Q; ++q) stage[(q * R + g) * G + j] = x[q];
        wave_sync_lds();
        // colour runs are taken R at a time, one per group of G lanes: each group sums its run in
        // member order (four staged rows in flight), then the groups fold into N one after the
        // other in run order, so every entry of N receives its terms in the order above
        int r0 = 0;
        while (r0 < cnt) {
            int my_s = 0, my_e = 0, idx = (int)kNoSlot;
#pragma unroll
            for (int h = 0; h < R; ++h) {
                const int c = r0 < cnt ? bcast(sc, r0) : -1;
                const int r1 = c >= 0 ? r0 + __popcll((unsigned long long)__ballot(lane < cnt && sc == c)) : r0;
                int f = (int)kNoSlot;
#pragma unroll
                for (int m = 0; m < NC; ++m)
                    if (c >= 0 && m == c / R) f = fidx[m];
                const int fh = __shfl(f, ((c >= 0 ? c : 0) % R) * G + j);
                if (g == h) {
                    my_s = r0;
                    my_e = r1;
                    idx = c >= 0 ? fh : (int)kNoSlot;
                }
                r0 = r1;
            }
            const bool act = idx != (int)kNoSlot && my_s < my_e;
            double acc = 0.0;
            if (act) {
                acc = stage[my_s * G + j];
                int i = my_s + 1;
                for (; i + 4 <= my_e; i += 4) {
                    const double a0 = stage[i * G + j], a1 = stage[(i + 1) * G + j];
                    const double a2 = stage[(i + 2) * G + j], a3 = stage[(i + 3) * G + j];
                    acc += a0;
                    acc += a1;
                    acc += a2;
                    acc += a3;
                }
                for (; i < my_e; ++i) acc += stage[i * G + j];
            }
#pragma unroll
            for (int h = 0; h < R; ++h) {
                if (g == h && act) N[idx] += acc;
                wave_sync_lds();  // runs of different colours may reach the same entry
            }
        }
        wave_sync_lds();
    }
}

// Neighbour sum of the 2-vertex passive table (p = 2). Entry j of a neighbour u's row is the number
// of u's neighbours of the j-th colour other than col(u) (Eq. 1 for an edge), so every term, and
// every partial sum of N, is an integer below the number of CSR entries: exact in any order. The
// terms therefore go to N by LDS atomic adds in whatever order they arrive, and each 64-entry block
// issues all of its row loads (16 lanes per row, four rows per load instruction) before its first
// add; the sums are bit for bit those of the ordered paths. ft (LDS, k x 16 entries) receives the
// N position of every (neighbour colour, entry) for this centre colour, or kNoSlot.
__device__ void gather_p2(const StepParams& S, int64_t beg, int64_t end, int cv, double* N, uint16_t* ft,
                          int lane) {
    const int k = S.k;
    const int Wp = S.Wp;
    const int g = lane >> 4, j = lane & 15;
    for (int t = lane; t < k * 16; t += kWave) {
        const int c = t >> 4, jj = t & 15;
        uint16_t f = kNoSlot;
        if (jj < Wp && c != cv) {
            const int xpos = cv - (cv > c ? 1 : 0);
            if (((S.mask[jj] >> xpos) & 1) == 0) f = S.fold[((int64_t)c * k + cv) * Wp + jj];
        }
        ft[t] = f;
    }
    wave_sync_lds();
    const double* Pb = S.P + (int64_t)class_slot(S, cv) * S.class_stride;
    for (int64_t e0 = beg; e0 < end; e0 += kWave) {
        const int64_t e = e0 + lane;
        const bool valid = e < end;
        const int u = valid ? S.col[e] : 0;
        const int cu = valid ? (int)(S.ecol ? S.ecol[e] : S.colour[(int64_t)u * S.cstride]) : 255;
        const int cnt = (end - e0 < kWave) ? (int)(end - e0) : kWave;
        double x[16];
        int tq[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int i = q * 4 + g;
            const int ui = __shfl(u, i < cnt ? i : 0);
            const int ci = __shfl(cu, i < cnt ? i : 0);
            const bool row = i < cnt && ci < k && ci != cv && j < Wp;
            x[q] = row ? Pb[(int64_t)ui * S.pstride + j] : 0.0;
            tq[q] = row ? (int)ft[ci * 16 + j] : (int)kNoSlot;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q)
            if (tq[q] != (int)kNoSlot)
                __hip_atomic_fetch_add(N + tq[q], x[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
}

// neighbour sum of a segment for p >= 2 (NARROW = G lanes per row, 2 for the 2-vertex table, or 0
// for the general path)
template <int J, int NARROW>
__device__ __forceinline__ void gather_rows(const StepParams& S, int64_t beg, int64_t end, int cv, double* N,
                                            int lane) {
    if constexpr (NARROW == 2) gather_p2(S, beg, end, cv, N, reinterpret_cast<uint16_t*>(N + S.stage_off), lane);
    else if constexpr (NARROW > 0) gather_fold_narrow<NARROW>(S, beg, end, cv, N, N + S.stage_off, lane);
    else gather_fold<J>(S, beg, end, cv, N, lane);
}

// N[lane'] += number of neighbours in [beg, end) with colour c, lane' = c renumbered without cv
__device__ void count_colours(const StepParams& S, int64_t beg, int64_t end, int cv, double* N, int lane) {
    const int k = S.k;
    unsigned cnt = 0;
    const int my_c = lane + (lane >= cv ? 1 : 0);
    for (int64_t e0 = beg; e0 < end; e0 += kWave) {
        const int64_t e = e0 + lane;
        const bool valid = e < end;
        const int cu = valid ? (int)(S.ecol ? S.ecol[e] : S.colour[(int64_t)S.col[e] * S.cstride]) : 255;
        for (int c = 0; c < k; ++c) {
            const uint64_t b = __ballot(cu == c);
            if (c == my_c) cnt += (unsigned)__popcll((unsigned long long)b);
        }
    }
    if (lane < k - 1) N[lane] += (double)cnt;
}

// output sets of v from N (LDS) and the active row A (staged in LDS, or in HBM when wide)
__device__ __forceinline__ void combine_sets(const StepParams& S, double* orow, const double* A, const double* N,
                                             int lane) {
    if (S.Ws >= kWave / 2) {
        for (int r = lane; r < S.Ws; r += kWave) {
            const uint32_t* sp = S.split + r;
            // pairs in runs of 16 (four pairs' loads in flight, their products added in pair
            // order), the runs of a group of 16 added in order, then the groups: the blocked
            // order of blocked_sum, written out to keep the loads in flight
            double total = 0.0;
            for (int g = 0; g < S.npairs; g += kSumRun * kSumRun) {
                const int ge = (S.npairs - g < kSumRun * kSumRun) ? S.npairs : g + kSumRun * kSumRun;
                double gs = 0.0;
                for (int b = g; b < ge; b += kSumRun) {
                    const int be = (ge - b < kSumRun) ? ge : b + kSumRun;
                    double bs = 0.0;
                    int j = b;
                    for (; j + 4 <= be; j += 4) {
                        uint32_t pr[4];
                        double av[4], nv[4];
#pragma unroll
                        for (int q = 0; q < 4; ++q) pr[q] = sp[(int64_t)(j + q) * S.Ws];
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            av[q] = A[pr[q] & 0xFFFFu];
                            nv[q] = N[pr[q] >> 16];
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) bs += av[q] * nv[q];
                    }
                    for (; j < be; ++j) {
                        const uint32_t pr = sp[(int64_t)j * S.Ws];
                        bs += A[pr & 0xFFFFu] * N[pr >> 16];
                    }
                    gs += bs;
                }
                total += gs;
            }
            orow[r] = total;
        }
    } else {
        // few outputs: G lanes per output set, pairs strided over 64/G parts, fixed-order reduce
        int G = 1;
        while (G < S.Ws) G <<= 1;
        const int parts = kWave / G;
        const int r = lane & (G - 1);
        const int part = lane / G;
        double sum = 0.0;
        if (r < S.Ws) {
            // this lane's pairs part, part + parts, ... in blocked order
            const uint32_t* sp = S.split + r;
            const int mine = (S.npairs - part + parts - 1) / parts;
            sum = blocked_sum(mine, [&](int i) {
                const uint32_t pr = sp[(int64_t)(part + i * parts) * S.Ws];
                return A[pr & 0xFFFFu] * N[pr >> 16];
            });
        }
        for (int off = G; off < kWave; off <<= 1) sum += __shfl_xor(sum, off);
        if (part == 0 && r < S.Ws) orow[r] = sum;
    }
}

// out row of v from N (LDS) and the active row of v
__device__ void combine_store(const StepParams& S, int v, double* N, double* Ash, int lane) {
    double* orow = S.O + (int64_t)v * S.ostride;
    if (S.a == 1) {
        // T' is the single vertex v: C(v, T', {col(v)}) = 1, so C(v, T, .) = N(v, .), written in
        // the output row's storage order
        // (with a = 1 the split list holds, for each output position, its entry of N)
        for (int r = lane; r < S.Ws; r += kWave) orow[r] = N[S.split[r]];
        return;
    }
    const double* arow = S.A + (int64_t)v * S.astride;
    if (S.stage_a) {
        for (int r = lane; r < S.Wa; r += kWave) Ash[r] = arow[r];
        wave_sync_lds();
    }
    // one copy of the loop for both cases (a second inlined copy costs registers in every variant)
    combine_sets(S, orow, S.stage_a ? (const double*)Ash : arow, N, lane);
}

// one light row: neighbour sum into LDS, then combine and store
template <int J, int NARROW>
__device__ __forceinline__ void light_row(const StepParams& S, int v, double* N, double* Ash, int lane) {
    const int64_t beg = S.row_ptr[v];
    const int64_t end = S.row_ptr[v + 1];
    // a vertex without a valid colour (>= k) roots no colourful embedding
    const int cv = __builtin_amdgcn_readfirstlane((int)S.colour[(int64_t)v * S.cstride]);
    if (!class_in(S, cv)) return;  // another pass of a projected split owns this row
    if (beg == end || cv >= S.k) {
        double* orow = S.O + (int64_t)v * S.ostride;
        for (int r = lane; r < S.Ws; r += kWave) orow[r] = 0.0;
        return;
    }
    for (int r = lane; r < S.Nw; r += kWave) N[r] = 0.0;
    wave_sync_lds();
    if (S.p == 1) count_colours(S, beg, end, cv, N, lane);
    else gather_rows<J, NARROW>(S, beg, end, cv, N, lane);
    wave_sync_lds();
    combine_store(S, v, N, Ash, lane);
    wave_sync_lds();
}

// task t of a split: a chunk of a cut row (partial N row to scratch) or a range of light rows
template <int J, int NARROW>
__device__ __forceinline__ void do_task(const StepParams& S, int64_t t, double* N, double* Ash, int lane) {
    if (t < S.n_chunks) {
        const ChunkItem ch = S.chunks[t];
        const int v = __builtin_amdgcn_readfirstlane(ch.v);
        const int cv = __builtin_amdgcn_readfirstlane((int)S.colour[(int64_t)v * S.cstride]);
        if (!class_in(S, cv)) return;  // another pass of a projected split owns this chunk
        for (int r = lane; r < S.Nw; r += kWave) N[r] = 0.0;
        wave_sync_lds();
        if (cv < S.k) {
            if (S.p == 1) count_colours(S, ch.beg, ch.beg + ch.len, cv, N, lane);
            else gather_rows<J, NARROW>(S, ch.beg, ch.beg + ch.len, cv, N, lane);
        }
        wave_sync_lds();
        double* prow = S.partial + t * S.nstride;
        for (int r = lane; r < S.Nw; r += kWave) prow[r] = N[r];
        wave_sync_lds();
    } else {
        const int64_t r = t - S.n_chunks;
        const int i0 = S.light_start[r], i1 = S.light_start[r + 1];
        for (int i = i0; i < i1; ++i) light_row<J, NARROW>(S, S.light[i], N, Ash, lane);
    }
}

// cut row t of a split: add its chunk partials in the fixed blocked order, then combine
__device__ __forceinline__ void do_hub(const StepParams& S, int64_t t, double* N, double* Ash, int lane) {
    const HubItem h = S.hubs[t];
    for (int r = lane; r < S.Nw; r += kWave) {
        const double* pp = S.partial + h.first_chunk * S.nstride + r;
        N[r] = blocked_sum(h.n_chunks, [&](int c) { return pp[(int64_t)c * S.nstride]; });
    }
    wave_sync_lds();
    combine_store(S, h.v, N, Ash, lane);
    wave_sync_lds();
}

// Tasks (chunks of cut rows first, then ranges of light rows, all of about `chunk` entries) are
// dealt to the persistent wavefronts round-robin: no shared counter, one fixed owner per task.
// The second bound is the minimum wavefronts per SIMD the register allocation must allow: the
// 16-lane narrow variant and the 8-double gather would otherwise sit just above the 128-register
// step to four (the 8-double gather: 129 registers and three wavefronts; bounded, 6 % faster).
template <int J, int NARROW>
__global__ __launch_bounds__(256, ((NARROW == 16 || J == 8) ? 4 : 1)) void k_split(StepParams S) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    double* N = lds + (int64_t)wib * S.lds_wave;
    double* Ash = N + S.a_off;
    const int64_t n_tasks = S.n_chunks + S.n_ranges;
    const int64_t n_waves = (int64_t)gridDim.x * S.waves_per_block;
    for (int64_t t = (int64_t)blockIdx.x * S.waves_per_block + __builtin_amdgcn_readfirstlane(wib); t < n_tasks; t += n_waves)
        do_task<J, NARROW>(S, t, N, Ash, lane);
}

__global__ __launch_bounds__(256) void k_hub_finish(StepParams S) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    double* N = lds + (int64_t)wib * S.lds_wave;
    double* Ash = N + S.a_off;
    const int64_t n_waves = (int64_t)gridDim.x * S.waves_per_block;
    for (int64_t t = (int64_t)blockIdx.x * S.waves_per_block + __builtin_amdgcn_readfirstlane(wib); t < S.n_hubs; t += n_waves)
        do_hub(S, t, N, Ash, lane);
}

// Projected passive rows for one pass of a split: for each vertex u that has a colour cu below k,
// and each centre colour c of the pass other than cu, the entries of u's row whose colour set
// avoids c (the only ones a centre of colour c adds up), in colex order of the set, as one
// contiguous row. One wavefront per vertex: the row is read once from HBM (staged in LDS when it
// holds at most kProjStage entries), then each copy gathers its entries with all index loads and
// value loads of a lane issued before its stores.
constexpr int kProjStage = 1024;

template <bool STAGE>
__global__ __launch_bounds__(256) void k_project(const double* __restrict__ P, int64_t pstride, int W,
                                                 const uint8_t* __restrict__ colour, int64_t n, int k,
                                                 const uint16_t* __restrict__ src, int Wn, int64_t qstride,
                                                 int64_t class_stride, uint32_t cls_mask, double* __restrict__ out) {
    __shared__ double stage[STAGE ? 4 * kProjStage : 1];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    double* row_sh = stage + (STAGE ? wib * kProjStage : 0);
    const int64_t wave = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
    const int64_t n_waves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t u = wave; u < n; u += n_waves) {
        const int cu = __builtin_amdgcn_readfirstlane((int)colour[u]);
        if (cu >= k) continue;
        const double* prow = P + u * pstride;
        if constexpr (STAGE) {
            // every load of the row in flight before the first store to the stage
            double t[kProjStage / kWave];
#pragma unroll
            for (int q = 0; q < kProjStage / kWave; ++q) {
                const int j = q * kWave + lane;
                t[q] = j < W ? prow[j] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < kProjStage / kWave; ++q) {
                const int j = q * kWave + lane;
                if (j < W) row_sh[j] = t[q];
            }
            wave_sync_lds();
        }
        for (int c = 0; c < k; ++c) {
            if (c == cu || !((cls_mask >> c) & 1u)) continue;
            const int slot = __popc(cls_mask & ((1u << c) - 1u));
            const uint16_t* sm = src + ((int64_t)cu * k + c) * Wn;
            double* orow = out + (int64_t)slot * class_stride + u * qstride;
            for (int j0 = 0; j0 < Wn; j0 += 4 * kWave) {
                int idx[4];
                double val[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = j0 + q * kWave + lane;
                    idx[q] = j < Wn ? (int)sm[j] : -1;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (STAGE) val[q] = idx[q] >= 0 ? row_sh[idx[q]] : 0.0;
                    else val[q] = idx[q] >= 0 ? prow[idx[q]] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (idx[q] >= 0) orow[j0 + q * kWave + lane] = val[q];
            }
        }
        if constexpr (STAGE) wave_sync_lds();  // the next row overwrites the stage
    }
}

// ---------------------------------------------------------------------------------------------
// batched launches: many (instance, split) segments
// ---------------------------------------------------------------------------------------------

// One persistent launch: each workgroup owns whole instances (round-robin over the batch) and
// runs an instance's segments in plan order, its wavefronts sharing each segment's items; a
// workgroup barrier separates consecutive segments. An instance's tables are written and read
// by one workgroup only, so no device-wide synchronisation is needed.
template <int J>
__global__ __launch_bounds__(512) void k_batch_inst(const SegDesc* __restrict__ segs, const SegRange* __restrict__ inst,
                                                    int n_inst, int lds_wave) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    const int wpb = blockDim.x / kWave;
    double* N = lds + (int64_t)wib * lds_wave;
    for (int i = blockIdx.x; i < n_inst; i += gridDim.x) {
        const SegRange range = inst[i];
        for (int q = range.first; q < range.first + range.count; ++q) {
            const SegDesc& D = segs[q];
            double* Ash = N + D.S.a_off;
            for (int64_t t = __builtin_amdgcn_readfirstlane(wib); t < D.n_items; t += wpb) {
                if (D.phase == 0) do_task<J, 0>(D.S, t, N, Ash, lane);
                else do_hub(D.S, t, N, Ash, lane);
            }
            __syncthreads();
        }
    }
}

// One launch per (dependency level, kernel variant) group: items [item_lo, item_hi) of the
// level-ordered segment list, which lie in segments [seg_lo, seg_hi), are dealt round-robin to
// persistent wavefronts; every item of a level is independent.
template <int J, int NARROW>
__global__ __launch_bounds__(256, (NARROW == 16 ? 4 : 1)) void k_batch_level(const SegDesc* __restrict__ segs, int seg_lo, int seg_hi,
                                                     int64_t item_lo, int64_t item_hi, int lds_wave, int wpb) {
    extern __shared__ double lds[];
    const int lane = lane_id();
    const int wib = threadIdx.x / kWave;
    double* N = lds + (int64_t)wib * lds_wave;
    const int64_t n_waves = (int64_t)gridDim.x * wpb;
    int seg = seg_lo;
    int64_t s_begin = segs[seg].item_start, s_end = s_begin + segs[seg].n_items;
    // item and segment indices are wave-uniform: kept in scalar registers
    for (int64_t t = item_lo + (int64_t)blockIdx.x * wpb + __builtin_amdgcn_readfirstlane(wib); t < item_hi;
         t += n_waves) {
        while (t >= s_end && seg + 1 < seg_hi) {  // items only increase: walk forward
            ++seg;
            s_begin = segs[seg].item_start;
            s_end = s_begin + segs[seg].n_items;
        }
        seg = __builtin_amdgcn_readfirstlane(seg);
        const SegDesc& D = segs[seg];
        double* Ash = N + D.S.a_off;
        if (D.phase == 0) do_task<J, NARROW>(D.S, t - s_begin, N, Ash, lane);
        else do_hub(D.S, t - s_begin, N, Ash, lane);
    }
}

// per-instance root sums, blocks laid out exactly as launch_reduce does for one instance
__global__ __launch_bounds__(256) void k_reduce_batch_blocks(const ReduceDesc* rd) {
    __shared__ double sh[256];
    const ReduceDesc R = rd[blockIdx.y];
    int64_t blocks = (R.n + kReducePerBlock - 1) / kReducePerBlock;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    if ((int64_t)blockIdx.x >= blocks) return;
    const int64_t per = (R.n + blocks - 1) / blocks;
    const int64_t lo = blockIdx.x * per;
    const int64_t hi = lo + per < R.n ? lo + per : R.n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += 256) s += R.x[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) R.partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_reduce_batch_final(const ReduceDesc* rd) {
    __shared__ double sh[256];
    const ReduceDesc R = rd[blockIdx.x];
    int64_t blocks = (R.n + kReducePerBlock - 1) / kReducePerBlock;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    double s = 0.0;
    for (int i = threadIdx.x; i < blocks; i += 256) s += R.partial[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) R.out[0] = sh[0];
}

// ---------------------------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------------------------

__global__ void k_fill_u32(unsigned* p, int64_t n, unsigned v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// ecol[e] = colour[col[e]]: four CSR entries per thread when col is 16-byte aligned (ecol is)
__global__ __launch_bounds__(256) void k_edge_colours(const int32_t* __restrict__ col, const uint8_t* __restrict__ colour,
                                                      int64_t nnz, uint8_t* __restrict__ ecol, int vec) {
    const int64_t quads = vec ? nnz / 4 : 0;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = t0; i < quads; i += step) {
        const int4 c = reinterpret_cast<const int4*>(col)[i];
        const uint32_t w = (uint32_t)colour[c.x] | ((uint32_t)colour[c.y] << 8) | ((uint32_t)colour[c.z] << 16) |
                           ((uint32_t)colour[c.w] << 24);
        reinterpret_cast<uint32_t*>(ecol)[i] = w;
    }
    for (int64_t e = quads * 4 + t0; e < nnz; e += step) ecol[e] = colour[col[e]];
}

// colours[b*n + v] = floor(k * h / 2^64), h = mix64(mix64(seed + G*(iter+1)) + H*(v+1))
__global__ void k_colour(uint64_t seed, uint64_t first_iter, int64_t n, int k, int B, uint8_t* out) {
    const int64_t total = (int64_t)B * n;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = i / n, v = i - b * n;
        const uint64_t base = mix64(seed + 0x9E3779B97F4A7C15ULL * (first_iter + (uint64_t)b + 1));
        const uint64_t h = mix64(base + 0xD1B54A32D192ED03ULL * (uint64_t)(v + 1));
        out[i] = (uint8_t)__umul64hi(h, (uint64_t)k);
    }
}

// fixed-order two-level sum of x[0..n) into out[0]; partial has `blocks` slots
constexpr int kRedThreads = 256;

__global__ __launch_bounds__(kRedThreads) void k_reduce_blocks(const double* x, int64_t n, int64_t per_block,
                                                                double* partial) {
    __shared__ double sh[kRedThreads];
    const int64_t lo = blockIdx.x * per_block;
    const int64_t hi = lo + per_block < n ? lo + per_block : n;
    double s = 0.0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += kRedThreads) s += x[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_final(const double* partial, int blocks, double* out) {
    __shared__ double sh[kRedThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < blocks; i += kRedThreads) s += partial[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kRedThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// CSR validation (row offsets already checked on the host): flags bit0 column out of range,
// bit1 self-loop, bit2 unsorted or duplicate, bit3 asymmetric
__global__ void k_validate(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, unsigned* flags) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        // row of e: last v with row_ptr[v] <= e
        int64_t lo = 0, hi = n;  // invariant row_ptr[lo] <= e < row_ptr[hi]
        while (hi - lo > 1) {
            const int64_t mid = (lo + hi) / 2;
            if (row_ptr[mid] <= e) lo = mid; else hi = mid;
        }
        const int64_t v = lo;
        const int32_t u = col[e];
        unsigned f = 0;
        if (u < 0 || u >= n) f |= 1u;
        else {
            if (u == v) f |= 2u;
            if (e > row_ptr[v] && col[e - 1] >= u) f |= 4u;
            // v in row u?
            int64_t a = row_ptr[u], b = row_ptr[u + 1];
            bool found = false;
            while (a < b) {
                const int64_t m = (a + b) / 2;
                const int32_t w = col[m];
                if (w == v) { found = true; break; }
                if (w < v) a = m + 1; else b = m;
            }
            if (!found) f |= 8u;
        }
        if (f) atomicOr(flags, f);
    }
}

// ---------------------------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------------------------

static inline int grid_for(int64_t n, int threads, int cap) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n, 256, 8192)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_edge_colours(const int32_t* col, const uint8_t* colour, int64_t nnz, uint8_t* ecol, hipStream_t st) {
    if (nnz <= 0) return hipSuccess;
    const int vec = ((uintptr_t)col % 16 == 0) ? 1 : 0;
    hipLaunchKernelGGL(k_edge_colours, dim3(grid_for(nnz / 4 + 1, 256, 65536)), dim3(256), 0, st, col, colour, nnz, ecol,
                       vec);
    return hipGetLastError();
}

hipError_t launch_colour(uint64_t seed, uint64_t first_iter, int64_t n, int k, int B, uint8_t* out, hipStream_t st) {
    const int64_t total = (int64_t)B * n;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colour, dim3(grid_for(total, 256, 16384)), dim3(256), 0, st, seed, first_iter, n, k, B, out);
    return hipGetLastError();
}

int reduce_blocks_for(int64_t n) {
    int64_t b = (n + kReducePerBlock - 1) / kReducePerBlock;
    if (b < 1) b = 1;
    if (b > 1024) b = 1024;
    return (int)b;
}

hipError_t launch_reduce(const double* x, int64_t n, double* partial, double* out, hipStream_t st) {
    const int blocks = reduce_blocks_for(n);
    const int64_t per = (n + blocks - 1) / blocks;
    hipLaunchKernelGGL(k_reduce_blocks, dim3(blocks), dim3(kRedThreads), 0, st, x, n, per, partial);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(kRedThreads), 0, st, (const double*)partial, blocks, out);
    return hipGetLastError();
}

hipError_t launch_validate(const int64_t* row_ptr, const int32_t* col, int64_t n, int64_t nnz, unsigned* flags,
                           hipStream_t st) {
    if (nnz > 0)
        hipLaunchKernelGGL(k_validate, dim3(grid_for(nnz, 256, 65536)), dim3(256), 0, st, row_ptr, col, n, nnz, flags);
    return hipGetLastError();
}

// passive-row doubles per lane per pass: the narrowest pass that covers the row, up to 8 (wider
// rows take several passes; eight doubles per lane measured faster than four from 330 up)
int pick_J(int Wp, int want) {
    if (want == 1 || want == 2 || want == 4 || want == 8) return want;
    if (Wp <= 64) return 1;
    if (Wp <= 128) return 2;
    if (Wp <= 256) return 4;
    return 8;
}

// the one-colouring launch may also take 6 doubles per lane (rows of 257..384 entries in one pass
// with fewer idle lanes) or 16 (rows beyond 512 entries)
static int launch_J(int Wp, int want) {
    if (want == 16) return 16;
    const int J = pick_J(Wp, want);
    if (want == 0 && J == 8 && Wp <= 384) return 6;
    if (want == 0 && J == 8 && Wp > 512) return 16;
    return J;
}

// wavefronts per workgroup (4, 2 or 1; a workgroup stays within 64 KB of LDS): a smaller
// workgroup only when it keeps over 10 % more wavefronts resident in a CU's 160 KB of LDS
static int waves_for_lds(int lds_wave) {
    const size_t per = (size_t)lds_wave * sizeof(double);
    int best = 1;
    size_t best_res = 0;
    for (int w = 4; w >= 1; w >>= 1) {
        if (per * w > 64 * 1024) continue;
        const size_t res = (size_t)w * ((160 * 1024) / (per * w > 0 ? per * w : 1));
        if (res * 10 > best_res * 11) {
            best_res = res;
            best = w;
        }
    }
    return best;
}

hipError_t launch_project(const double* P, int64_t pstride, int W, const uint8_t* colour, int64_t n, int k,
                          const uint16_t* src, int Wn, int64_t qstride, int64_t class_stride, uint32_t cls_mask,
                          double* out, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (W <= kProjStage)
        hipLaunchKernelGGL(k_project<true>, dim3(grid_for(n, 4, 65536)), dim3(256), 0, st, P, pstride, W, colour, n, k,
                           src, Wn, qstride, class_stride, cls_mask, out);
    else
        hipLaunchKernelGGL(k_project<false>, dim3(grid_for(n, 4, 65536)), dim3(256), 0, st, P, pstride, W, colour, n, k,
                           src, Wn, qstride, class_stride, cls_mask, out);
    return hipGetLastError();
}

// launch geometry of a split (both kernels use the same workgroup shape and LDS slice)
struct SplitLaunch {
    const void* fn;
    int threads;
    size_t lds;
};

static hipError_t split_geometry(StepParams* Sp, SplitLaunch* L) {
    StepParams& S = *Sp;
    // the 2-vertex table has its own path (a table of k x 16 fold positions in LDS); other narrow
    // passive rows take G lanes per row (a stage of 64 rows in LDS) unless a width is forced
    const bool p2 = S.p == 2 && S.cols_per_lane == 0 && S.Wp <= 16;
    const int narrow = (!p2 && S.p >= 2 && S.cols_per_lane == 0 && S.Wp <= 32) ? (S.Wp <= 16 ? 16 : 32) : 0;
    S.a_off = split_a_off(S.Nw);
    S.stage_a = split_stage_a(S.Nw, S.Wa, S.a) ? 1 : 0;
    S.lds_wave = split_lds_wave(S.Nw, S.Wa, S.a);
    S.stage_off = S.lds_wave;
    S.lds_wave += p2 ? kMaxK * 16 * (int)sizeof(uint16_t) / (int)sizeof(double) : narrow * kWave;
    if ((size_t)S.lds_wave * sizeof(double) > 160 * 1024) return hipErrorInvalidConfiguration;
    const int waves_per_block = waves_for_lds(S.lds_wave);
    const int threads = waves_per_block * kWave;
    S.waves_per_block = waves_per_block;
    const size_t lds = (size_t)S.lds_wave * waves_per_block * sizeof(double);
    const int J = (S.p >= 2) ? launch_J(S.Wp, S.cols_per_lane) : 1;
    const void* fn = nullptr;
    if (p2) fn = (const void*)k_split<1, 2>;
    else if (narrow == 16) fn = (const void*)k_split<1, 16>;
    else if (narrow == 32) fn = (const void*)k_split<1, 32>;
    else switch (J) {
        case 1: fn = (const void*)k_split<1, 0>; break;
        case 2: fn = (const void*)k_split<2, 0>; break;
        case 4: fn = (const void*)k_split<4, 0>; break;
        case 6: fn = (const void*)k_split<6, 0>; break;
        case 8: fn = (const void*)k_split<8, 0>; break;
        default: fn = (const void*)k_split<16, 0>; break;
    }
    L->fn = fn;
    L->threads = threads;
    L->lds = lds;
    return hipSuccess;
}

hipError_t launch_split_tasks(StepParams S, int n_cu, hipStream_t st) {
    SplitLaunch L;
    hipError_t err = split_geometry(&S, &L);
    if (err != hipSuccess) return err;
    int per_cu = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, L.fn, L.threads, L.lds);
    if (err != hipSuccess) return err;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    const int64_t total = S.n_chunks + S.n_ranges;
    int64_t blocks = (int64_t)per_cu * n_cu;
    const int64_t need = (total + S.waves_per_block - 1) / S.waves_per_block;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    if (total > 0) {
        void* args[] = {&S};
        err = hipLaunchKernel(L.fn, dim3((unsigned)blocks), dim3(L.threads), args, L.lds, st);
        if (err != hipSuccess) return err;
        err = hipGetLastError();
    }
    return err;
}

hipError_t launch_hub_finish(StepParams S, int n_cu, hipStream_t st) {
    if (S.n_hubs <= 0) return hipSuccess;
    SplitLaunch L;
    hipError_t err = split_geometry(&S, &L);
    if (err != hipSuccess) return err;
    int per_cu2 = 0;
    err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, (const void*)k_hub_finish, L.threads, L.lds);
    if (err != hipSuccess) return err;
    if (per_cu2 < 1) return hipErrorInvalidConfiguration;
    int64_t b2 = (int64_t)per_cu2 * n_cu;
    const int64_t need2 = (S.n_hubs + S.waves_per_block - 1) / S.waves_per_block;
    if (b2 > need2) b2 = need2;
    hipLaunchKernelGGL(k_hub_finish, dim3((unsigned)b2), dim3(L.threads), L.lds, st, S);
    return hipGetLastError();
}

hipError_t launch_split(StepParams S, int n_cu, hipStream_t st, hipEvent_t mid) {
    hipError_t err = launch_split_tasks(S, n_cu, st);
    if (err == hipSuccess && mid) err = hipEventRecord(mid, st);
    if (err == hipSuccess) err = launch_hub_finish(S, n_cu, st);
    return err;
}

// kernel variant of a split: 0..3 = general path with 1, 2, 4, 8 doubles per lane; 4, 5 = narrow
// rows with 16 or 32 lanes per row; 6 = the 2-vertex table's path (the choice launch_split makes
// for a plain count)
int split_variant(int p, int Wp, int cols_per_lane) {
    if (p < 2) return 0;
    if (p == 2 && cols_per_lane == 0 && Wp <= 16) return 6;
    if (cols_per_lane == 0 && Wp <= 16) return 4;
    if (cols_per_lane == 0 && Wp <= 32) return 5;
    switch (pick_J(Wp, cols_per_lane)) {
        case 1: return 0;
        case 2: return 1;
        case 4: return 2;
        default: return 3;
    }
}

int variant_stage(int variant) {
    if (variant == 6) return kMaxK * 16 * (int)sizeof(uint16_t) / (int)sizeof(double);
    return variant == 4 ? 16 * kWave : variant == 5 ? 32 * kWave : 0;
}

template <int J, int NARROW>
static hipError_t launch_level_t(const SegDesc* segs_dev, int seg_lo, int seg_hi, int64_t item_lo, int64_t item_hi,
                                 int lds_wave, int n_cu, hipStream_t st) {
    const int wpb = waves_for_lds(lds_wave);
    const int threads = wpb * kWave;
    const size_t lds = (size_t)lds_wave * wpb * sizeof(double);
    int per_cu = 0;
    hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch_level<J, NARROW>, threads, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int64_t blocks = (int64_t)per_cu * n_cu;
    const int64_t need = (item_hi - item_lo + wpb - 1) / wpb;
    if (blocks > need) blocks = need;
    hipLaunchKernelGGL((k_batch_level<J, NARROW>), dim3((unsigned)blocks), dim3(threads), lds, st, segs_dev, seg_lo,
                       seg_hi, item_lo, item_hi, lds_wave, wpb);
    return hipGetLastError();
}

hipError_t launch_batch_level(const SegDesc* segs_dev, int seg_lo, int seg_hi, int64_t item_lo, int64_t item_hi,
                              int variant, int lds_wave, int n_cu, hipStream_t st) {
    if (item_hi <= item_lo || seg_hi <= seg_lo) return hipSuccess;
    if ((size_t)lds_wave * sizeof(double) > 160 * 1024) return hipErrorInvalidConfiguration;
    switch (variant) {
        case 0: return launch_level_t<1, 0>(segs_dev, seg_lo, seg_hi, item_lo, item_hi, lds_wave, n_cu, st);
        case 1: return launch_level_t<2, 0>(segs_dev, seg_lo, seg_hi, item_lo, item_hi, lds_wave, n_cu, st);
        case 2: return launch_level_t<4, 0>(segs_dev, seg_lo, seg_hi, item_lo, item_hi, lds_wave, n_cu, st);
        case 3: return launch_level_t<8, 0>(segs_dev, seg_lo, seg_hi, item_lo, item_hi, lds_wave, n_cu, st);
        case 4: return launch_level_t<1, 16>(segs_dev, seg_lo, seg_hi, item_lo, item_hi, lds_wave, n_cu, st);
        case 5: return launch_level_t<1, 32>(segs_dev, seg_lo, seg_hi, item_lo, item_hi, lds_wave, n_cu, st);
        case 6: return launch_level_t<1, 2>(segs_dev, seg_lo, seg_hi, item_lo, item_hi, lds_wave, n_cu, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_batch_inst(const SegDesc* segs_dev, const SegRange* inst_dev, int n_inst, int J, int lds_wave, int n_cu,
                             int share, hipStream_t st) {
    if (n_inst <= 0) return hipSuccess;
    if ((size_t)lds_wave * sizeof(double) > 160 * 1024) return hipErrorInvalidConfiguration;
    // up to eight wavefronts per workgroup while the LDS slices fit in 64 KB
    int wpb = 8;
    while (wpb > 1 && (size_t)lds_wave * wpb * sizeof(double) > 64 * 1024) wpb >>= 1;
    const int threads = wpb * kWave;
    const size_t lds = (size_t)lds_wave * wpb * sizeof(double);
    const void* fn = nullptr;
    switch (J) {
        case 1: fn = (const void*)k_batch_inst<1>; break;
        case 2: fn = (const void*)k_batch_inst<2>; break;
        case 4: fn = (const void*)k_batch_inst<4>; break;
        default: fn = (const void*)k_batch_inst<8>; break;
    }
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    int64_t blocks = (int64_t)per_cu * n_cu / (share > 1 ? share : 1);
    if (blocks < 1) blocks = 1;
    if (blocks > n_inst) blocks = n_inst;
    switch (J) {
        case 1: hipLaunchKernelGGL(k_batch_inst<1>, dim3((unsigned)blocks), dim3(threads), lds, st, segs_dev, inst_dev, n_inst, lds_wave); break;
        case 2: hipLaunchKernelGGL(k_batch_inst<2>, dim3((unsigned)blocks), dim3(threads), lds, st, segs_dev, inst_dev, n_inst, lds_wave); break;
        case 4: hipLaunchKernelGGL(k_batch_inst<4>, dim3((unsigned)blocks), dim3(threads), lds, st, segs_dev, inst_dev, n_inst, lds_wave); break;
        default: hipLaunchKernelGGL(k_batch_inst<8>, dim3((unsigned)blocks), dim3(threads), lds, st, segs_dev, inst_dev, n_inst, lds_wave); break;
    }
    return hipGetLastError();
}

hipError_t launch_reduce_batch(const ReduceDesc* rd_dev, int n_inst, int max_blocks, hipStream_t st) {
    if (n_inst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_batch_blocks, dim3((unsigned)max_blocks, (unsigned)n_inst), dim3(256), 0, st, rd_dev);
    hipLaunchKernelGGL(k_reduce_batch_final, dim3((unsigned)n_inst), dim3(256), 0, st, rd_dev);
    return hipGetLastError();
}

}  // namespace cc
