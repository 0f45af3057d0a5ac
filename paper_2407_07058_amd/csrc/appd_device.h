// Device helpers shared by the APPD kernels (gfx950, wave64).
//
// Edge keys.  An edge (u,v) with weight w is ordered by (w, flat(u,v)),
// flat(u,v) = min(u,v)*n + max(u,v).  Packed as a 64-bit integer
//   key = ord32(w) << 32 | flat
// where ord32 maps float bits monotonically onto uint32 (negative floats are
// bit-inverted, non-negative ones get the top bit set; -0.0 is first made +0.0).
// Every real edge key is >= 2^32, so key 0 stands for "no edge" (the diagonal)
// and is the identity of max.  In widest mode every weight enters negated,
// which turns "larger weight first" into the same minimum order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace appd {

constexpr int kWave = 64;

__device__ __forceinline__ uint32_t ord32(float w) {
    uint32_t b = __float_as_uint(w);
    b = (b == 0x80000000u) ? 0u : b;  // -0.0 -> +0.0
    return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}

__device__ __forceinline__ float ord32_inv(uint32_t o) {
    uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
    return __uint_as_float(b);
}

__device__ __forceinline__ uint32_t flat_idx(uint32_t u, uint32_t v, uint32_t n) {
    return u < v ? u * n + v : v * n + u;
}

__device__ __forceinline__ uint64_t make_key(float w, uint32_t flat) {
    return ((uint64_t)ord32(w) << 32) | (uint64_t)flat;
}

// Weight of a key back in the caller's sign convention, -0.0 reported as +0.0.
template <bool WIDEST>
__device__ __forceinline__ float key_weight(uint64_t key) {
    float w = ord32_inv((uint32_t)(key >> 32));
    if (WIDEST) w = -w;
    uint32_t b = __float_as_uint(w);
    return __uint_as_float(b == 0x80000000u ? 0u : b);
}

__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return b < a ? b : a; }
__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return b > a ? b : a; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
    uint32_t lo = __shfl_xor((uint32_t)x, m);
    uint32_t hi = __shfl_xor((uint32_t)(x >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, int src) {
    uint32_t lo = __shfl((uint32_t)x, src);
    uint32_t hi = __shfl((uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t x, int d) {
    uint32_t lo = __shfl_up((uint32_t)x, d);
    uint32_t hi = __shfl_up((uint32_t)(x >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_down_u64(uint64_t x, int d) {
    uint32_t lo = __shfl_down((uint32_t)x, d);
    uint32_t hi = __shfl_down((uint32_t)(x >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}

// All lanes receive the wave-wide minimum.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) x = umin64(x, shfl_xor_u64(x, m));
    return x;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
#pragma unroll
    for (int m = 1; m < kWave; m <<= 1) x = umax64(x, shfl_xor_u64(x, m));
    return x;
}

// Inclusive running max over lanes 0..lane.
__device__ __forceinline__ uint64_t wave_incl_max_up(uint64_t x, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t y = shfl_up_u64(x, d);
        if (lane >= d) x = umax64(x, y);
    }
    return x;
}

// Inclusive running max over lanes lane..63.
__device__ __forceinline__ uint64_t wave_incl_max_down(uint64_t x, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        uint64_t y = shfl_down_u64(x, d);
        if (lane + d < kWave) x = umax64(x, y);
    }
    return x;
}

// Orders LDS traffic of one wave: writes before the fence are visible to reads
// of other lanes of the same wave after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace appd
