// pms_device.h -- wavefront helpers shared by the search kernels (device code).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pms_dev {

typedef __attribute__((address_space(4))) const uint32_t cu32;

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Number of set bits of m below the calling lane.
__device__ __forceinline__ uint32_t rank_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0u));
}

__device__ __forceinline__ uint32_t uni(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// v_writelane_b32: lane `lane` of `old` replaced by the wave-uniform `val`
// (the LLVM intrinsic, which clang exposes under no builtin name here).  Not
// written as inline asm: v_writelane reads its SGPR operand early, so it
// needs wait states after the VALU instruction that wrote it (a ballot's
// v_cmp), which the compiler inserts for the intrinsic but not around asm.
__device__ int write_lane(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Reads a wave-uniform record of read-only data through the scalar cache.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
    static_assert(sizeof(T) % 4 == 0, "records are whole words");
    cu32* w = (cu32*)(p);
    T r;
    uint32_t* rw = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
    for (unsigned i = 0; i < sizeof(T) / 4; ++i) rw[i] = w[i];
    return r;
}

}  // namespace pms_dev
