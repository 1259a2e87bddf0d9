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
