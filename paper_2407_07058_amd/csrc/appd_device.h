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
// Word 3 of a buffer resource on gfx9: 32-bit data format, no swizzle; with
// stride 0 a load whose offset lies past the range returns 0.
constexpr int kBufferRsrcWord3 = 0x00020000;
// Cache-policy argument of a buffer store: non-temporal (nt).
constexpr int kBufferNontemporal = 2;

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

// Lane `src` (wave-uniform) of x, to every lane, without going through LDS.
__device__ __forceinline__ uint64_t readlane_u64(uint64_t x, int src) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)x, src);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

// Lane l receives lane l-1 of x within each row of 16 lanes (DPP row_shr:1);
// the first lane of a row keeps its own value.
__device__ __forceinline__ uint64_t row_shr1_u64(uint64_t x) {
    const int lo = (int)(uint32_t)x, hi = (int)(uint32_t)(x >> 32);
    const uint32_t rlo = __builtin_amdgcn_update_dpp(lo, lo, 0x111, 0xf, 0xf, false);
    const uint32_t rhi = __builtin_amdgcn_update_dpp(hi, hi, 0x111, 0xf, 0xf, false);
    return ((uint64_t)rhi << 32) | rlo;
}

// ---- cross-lane operations on DPP (data-parallel primitives: lane moves
// inside the VALU, no LDS round trip) and readlane.
// dpp_u64<CTRL>: DPP move of x with `fill` where the source lane is outside
// the row.  row_shr:k (0x110 + k): lane l takes lane l-k of its row of 16;
// row_shl:k (0x100 + k): lane l takes lane l+k.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x, uint64_t fill) {
    const uint32_t lo = __builtin_amdgcn_update_dpp((int)(uint32_t)fill, (int)(uint32_t)x, CTRL,
                                                    0xf, 0xf, false);
    const uint32_t hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(fill >> 32),
                                                    (int)(uint32_t)(x >> 32), CTRL, 0xf, 0xf, false);
    return ((uint64_t)hi << 32) | lo;
}

// All lanes receive the wave-wide minimum: running minima inside each row of
// 16 lanes (shifts 1, 2, 4, 8), then the four row results by readlane.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
    constexpr uint64_t I = ~0ull;
    x = umin64(x, dpp_u64<0x111>(x, I));
    x = umin64(x, dpp_u64<0x112>(x, I));
    x = umin64(x, dpp_u64<0x114>(x, I));
    x = umin64(x, dpp_u64<0x118>(x, I));
    return umin64(umin64(readlane_u64(x, 15), readlane_u64(x, 31)),
                  umin64(readlane_u64(x, 47), readlane_u64(x, 63)));
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
    x = umax64(x, dpp_u64<0x111>(x, 0));
    x = umax64(x, dpp_u64<0x112>(x, 0));
    x = umax64(x, dpp_u64<0x114>(x, 0));
    x = umax64(x, dpp_u64<0x118>(x, 0));
    return umax64(umax64(readlane_u64(x, 15), readlane_u64(x, 31)),
                  umax64(readlane_u64(x, 47), readlane_u64(x, 63)));
}

// Exclusive running max over lanes 0..lane-1 (0 for lane 0).
__device__ __forceinline__ uint64_t wave_excl_max_up(uint64_t x, int lane) {
    x = umax64(x, dpp_u64<0x111>(x, 0));
    x = umax64(x, dpp_u64<0x112>(x, 0));
    x = umax64(x, dpp_u64<0x114>(x, 0));
    x = umax64(x, dpp_u64<0x118>(x, 0));  // inclusive within the row
    const uint64_t r0 = readlane_u64(x, 15), r1 = readlane_u64(x, 31),
                   r2 = readlane_u64(x, 47);
    const int row = lane >> 4;
    const uint64_t carry = row == 0 ? 0ull
                           : row == 1 ? r0
                           : row == 2 ? umax64(r0, r1)
                                      : umax64(umax64(r0, r1), r2);
    const uint64_t prev = dpp_u64<0x111>(x, 0);  // lane l-1 of the row
    return (lane & 15) == 0 ? carry : umax64(prev, carry);
}

// Exclusive running max over lanes lane+1..63 (0 for lane 63).
__device__ __forceinline__ uint64_t wave_excl_max_down(uint64_t x, int lane) {
    x = umax64(x, dpp_u64<0x101>(x, 0));
    x = umax64(x, dpp_u64<0x102>(x, 0));
    x = umax64(x, dpp_u64<0x104>(x, 0));
    x = umax64(x, dpp_u64<0x108>(x, 0));  // inclusive within the row, downwards
    const uint64_t h1 = readlane_u64(x, 16), h2 = readlane_u64(x, 32),
                   h3 = readlane_u64(x, 48);
    const int row = lane >> 4;
    const uint64_t carry = row == 3 ? 0ull
                           : row == 2 ? h3
                           : row == 1 ? umax64(h2, h3)
                                      : umax64(umax64(h1, h2), h3);
    const uint64_t next = dpp_u64<0x101>(x, 0);  // lane l+1 of the row
    return (lane & 15) == 15 ? carry : umax64(next, carry);
}

// 32-bit forms of the scans above (one DPP move per step).
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x, uint32_t fill) {
    return __builtin_amdgcn_update_dpp((int)fill, (int)x, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_excl_max_up_u32(uint32_t x, int lane) {
    x = max(x, dpp_u32<0x111>(x, 0));
    x = max(x, dpp_u32<0x112>(x, 0));
    x = max(x, dpp_u32<0x114>(x, 0));
    x = max(x, dpp_u32<0x118>(x, 0));
    const uint32_t r0 = __builtin_amdgcn_readlane(x, 15), r1 = __builtin_amdgcn_readlane(x, 31),
                   r2 = __builtin_amdgcn_readlane(x, 47);
    const int row = lane >> 4;
    const uint32_t carry = row == 0 ? 0u : row == 1 ? r0 : row == 2 ? max(r0, r1) : max(max(r0, r1), r2);
    const uint32_t prev = dpp_u32<0x111>(x, 0);
    return (lane & 15) == 0 ? carry : max(prev, carry);
}

__device__ __forceinline__ uint32_t wave_excl_max_down_u32(uint32_t x, int lane) {
    x = max(x, dpp_u32<0x101>(x, 0));
    x = max(x, dpp_u32<0x102>(x, 0));
    x = max(x, dpp_u32<0x104>(x, 0));
    x = max(x, dpp_u32<0x108>(x, 0));
    const uint32_t h1 = __builtin_amdgcn_readlane(x, 16), h2 = __builtin_amdgcn_readlane(x, 32),
                   h3 = __builtin_amdgcn_readlane(x, 48);
    const int row = lane >> 4;
    const uint32_t carry = row == 3 ? 0u : row == 2 ? h3 : row == 1 ? max(h2, h3) : max(max(h1, h2), h3);
    const uint32_t next = dpp_u32<0x101>(x, 0);
    return (lane & 15) == 15 ? carry : max(next, carry);
}

// Orders LDS traffic of one wave: writes before the fence are visible to reads
// of other lanes of the same wave after it.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace appd
