// Wavefront helpers shared by the device code of libcc (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

namespace cc {

__device__ __forceinline__ int lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ int bcast(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }

__device__ __forceinline__ void wave_sync_lds() {
    // order this wavefront's LDS writes before its later LDS reads by other lanes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace cc

namespace cc {

// Fixed-order blocked sum of n terms term(0..n-1): runs of 16 terms are added in order, the run
// sums of a group of 16 runs are added in order, and the group sums are added in order. Every
// term passes through at most 15 + 15 + (ceil(n / 256) - 1) roundings, which bounds the relative
// error of a sum of non-negative terms by that count times the unit roundoff, whatever n is up
// to a few thousand; the order does not depend on anything but n.
constexpr int kSumRun = 16;
template <class F>
__device__ __forceinline__ double blocked_sum(int n, F term) {
    double total = 0.0;
    for (int g = 0; g < n; g += kSumRun * kSumRun) {
        const int ge = (n - g < kSumRun * kSumRun) ? n : g + kSumRun * kSumRun;
        double gs = 0.0;
        for (int b = g; b < ge; b += kSumRun) {
            const int be = (ge - b < kSumRun) ? ge : b + kSumRun;
            double bs = 0.0;
            for (int i = b; i < be; ++i) bs += term(i);
            gs += bs;
        }
        total += gs;
    }
    return total;
}

}  // namespace cc
