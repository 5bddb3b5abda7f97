// Device-side helpers shared by the libpss kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pss {

constexpr uint32_t kWave = 64;

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

// Make this wave's LDS writes visible to all of its lanes (one wave works on
// one summary; the wave runs in lockstep, so a wait plus a compiler barrier
// is all that is needed).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// A word of LDS that lanes of this wave have just changed with atomics,
// read again from memory.  The access goes through an LDS pointer: a
// volatile read through a generic pointer becomes a FLAT load, and waiting
// for a FLAT load also waits for every global load and store in flight.
__device__ __forceinline__ uint32_t lds_reread(const uint32_t* p) {
    return *(const volatile __attribute__((address_space(3))) uint32_t*)p;
}

// DPP lane moves (GFX9 encodings): quad_perm, row mirrors and row broadcasts.
template <int Ctrl, int RowMask>
__device__ __forceinline__ uint32_t dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, Ctrl, RowMask, 0xF, false);
}

// Minimum over the 64 lanes, in uniform control flow with all lanes active.
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
    v = min(v, dpp<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
    v = min(v, dpp<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
    v = min(v, dpp<0x141, 0xF>(v));  // row_half_mirror
    v = min(v, dpp<0x140, 0xF>(v));  // row_mirror
    v = min(v, dpp<0x142, 0xA>(v));  // row_bcast:15 into rows 1 and 3
    v = min(v, dpp<0x143, 0xC>(v));  // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}

// Maximum, bitwise or and bitwise and over the 64 lanes, same pattern.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
    v = max(v, dpp<0xB1, 0xF>(v));
    v = max(v, dpp<0x4E, 0xF>(v));
    v = max(v, dpp<0x141, 0xF>(v));
    v = max(v, dpp<0x140, 0xF>(v));
    v = max(v, dpp<0x142, 0xA>(v));
    v = max(v, dpp<0x143, 0xC>(v));
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v) {
    v |= dpp<0xB1, 0xF>(v);
    v |= dpp<0x4E, 0xF>(v);
    v |= dpp<0x141, 0xF>(v);
    v |= dpp<0x140, 0xF>(v);
    v |= dpp<0x142, 0xA>(v);
    v |= dpp<0x143, 0xC>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint32_t wave_and_u32(uint32_t v) {
    v &= dpp<0xB1, 0xF>(v);
    v &= dpp<0x4E, 0xF>(v);
    v &= dpp<0x141, 0xF>(v);
    v &= dpp<0x140, 0xF>(v);
    v &= dpp<0x142, 0xA>(v);
    v &= dpp<0x143, 0xC>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

// Sum over the 64 lanes, same pattern.
__device__ __forceinline__ uint32_t wave_add_u32(uint32_t v) {
    v += dpp<0xB1, 0xF>(v);
    v += dpp<0x4E, 0xF>(v);
    v += dpp<0x141, 0xF>(v);
    v += dpp<0x140, 0xF>(v);
    v += dpp<0x142, 0xA>(v);
    v += dpp<0x143, 0xC>(v);
    return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
    for (int off = 32; off > 0; off >>= 1) {
        uint64_t o = __shfl_xor(v, off);
        v = o < v ? o : v;
    }
    uint32_t lo = uniform((uint32_t)v), hi = uniform((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    for (int off = 32; off > 0; off >>= 1) v += (uint32_t)__shfl_xor((int)v, off);
    return uniform(v);
}

// Fibonacci hashing of an item id into a table of 2^bits slots.
__device__ __forceinline__ uint32_t hash_slot(uint32_t x, uint32_t bits) {
    return (x * 0x9E3779B1u) >> (32u - bits);
}

}  // namespace pss
