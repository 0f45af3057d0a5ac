// The K smallest entries of one row of W, found by one wave: the candidate
// lists of the Boruvka trees (single graph and batched).
#pragma once

#include "appd_device.h"

namespace appd {

constexpr int kK = 16;  // candidate list length
constexpr uint64_t kTopkNone = ~0ull;

// One wave per row.  Lanes 0..K-1 hold the row's K smallest entries seen so
// far, in ascending order; tau is the K-th.  The row is read in blocks of
// kPassElems columns per lane.  Before a block is offered, its threshold is
// set to the K-th smallest of the 64 lane minima (a bitwise search over the
// ord32 values with ballots): at least K eligible entries of the block lie at
// or below it, so nothing above it can enter the list.  Groups of four entries
// whose minimum lies above min(threshold, tau) cost one compare; an entry that
// passes is broadcast, its rank among the list (a ballot) gives its slot, and
// the lanes above shift up by one.
// All comparisons are made on s = w (minimax) or s = -w (widest); ties at the
// threshold are offered and ordered by the full key.
// VEC: rows are 16-byte aligned (n % 4 == 0), each lane reads 4 columns at once.
constexpr int kPassElems = 32;

// The K smallest entries of row u (u wave-uniform) by one wave: lane l < K
// returns the l-th smallest as ord32(s) << 32 | column (kTopkNone past the
// row's eligible entries).  Column c is skipped when c == u, or, with FILTER,
// when comp_of(c) == comp_of(u); comp_of is only called with FILTER, and
// with VEC it is also called through comp4 (four columns from c, c % 4 == 0).
// E: columns per lane per block (a multiple of 4; short rows take fewer).
// KK: entries kept (at most 16: the list lives in one 16-lane DPP row).
template <bool WIDEST, bool FILTER, bool VEC, int E = kPassElems, int KK = kK, class CompOf,
          class Comp4>
__device__ __forceinline__ uint64_t row_topk(const float* __restrict__ row, int n, int u,
                                             CompOf comp_of, Comp4 comp4) {
    static_assert(E % 4 == 0 && E >= 4, "groups of four columns per lane");
    static_assert(KK >= 1 && KK <= 16, "the list lives in lanes 0..15");
    constexpr uint64_t kNone = kTopkNone;
    const int lane = threadIdx.x & (kWave - 1);
    const int cu = FILTER ? comp_of(u) : u;
    uint64_t mine = kNone;    // this lane's slot of the sorted list (lanes < K)
    uint64_t tau = kNone;     // the K-th smallest so far (wave-uniform)
    float tau_s = INFINITY;   // its s value (+inf while the list is not full)
    auto offer = [&](float sv, int v, bool skip) {
        const uint64_t e = skip ? kNone : (((uint64_t)ord32(sv) << 32) | (uint32_t)v);
        uint64_t bal = __ballot(e < tau);
        while (bal) {
            const int src = __ffsll((unsigned long long)bal) - 1;
            bal &= bal - 1;
            const uint64_t x = readlane_u64(e, src);
            if (x < tau) {
                const int pos = __popcll(__ballot(lane < KK && mine < x));
                const uint64_t below = row_shr1_u64(mine);  // the list is lanes 0..15
                if (lane < KK) mine = lane > pos ? below : (lane == pos ? x : mine);
                tau = readlane_u64(mine, KK - 1);
            }
        }
        tau_s = tau == kNone ? INFINITY : ord32_inv((uint32_t)(tau >> 32));
    };
    constexpr int STEP = kWave * E;
    // the trip counts are the same for every lane (offer() is wave-wide)
    for (int b0 = 0; b0 < n; b0 += STEP) {
        float sv[E];
        int col[E];
        bool skip[E];
        if (VEC) {
#pragma unroll
            for (int j = 0; j < E / 4; ++j) {
                const int c0 = b0 + j * (kWave * 4) + lane * 4;
                float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                int4 cv = make_int4(cu, cu, cu, cu);
                if (c0 < n) {
                    x = *(const float4*)(row + c0);
                    if (FILTER) cv = comp4(c0);
                }
                const float xs[4] = {x.x, x.y, x.z, x.w};
                const int cs[4] = {cv.x, cv.y, cv.z, cv.w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int e = 4 * j + q;
                    col[e] = c0 + q;
                    sv[e] = WIDEST ? -xs[q] : xs[q];
                    skip[e] = c0 >= n || (FILTER ? cs[q] == cu : c0 + q == u);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int c = b0 + e * kWave + lane;
                const bool in = c < n;
                const float x = in ? row[c] : 0.0f;
                const int cv = (FILTER && in) ? comp_of(c) : cu;
                col[e] = c;
                sv[e] = WIDEST ? -x : x;
                skip[e] = !in || (FILTER ? cv == cu : c == u);
            }
        }
        // K-th smallest lane minimum of this block
        float lm = INFINITY;
#pragma unroll
        for (int e = 0; e < E; ++e) lm = fminf(lm, skip[e] ? INFINITY : sv[e]);
        // (skipped when fewer than K lane minima lie below tau: it could not
        // improve on tau).  The search runs over the top 16 bits of the ord32
        // values, which rounds the threshold up: still a valid bound.
        float tblk = INFINITY;
        if (__popcll(__ballot(lm < tau_s)) >= KK) {
            const uint32_t km = ord32(lm) >> 16;
            uint32_t res = 0;
            for (int b = 15; b >= 0; --b) {
                const uint32_t c = res | (1u << b);
                if (__popcll(__ballot(km < c)) < KK) res = c;
            }
            tblk = res == 0xffffu ? INFINITY : ord32_inv((res << 16) | 0xffffu);
        }
#pragma unroll
        for (int g = 0; g < E / 4; ++g) {
            const float thr = fminf(tblk, tau_s);
            float m4 = INFINITY;
#pragma unroll
            for (int q = 0; q < 4; ++q) m4 = fminf(m4, skip[4 * g + q] ? INFINITY : sv[4 * g + q]);
            if (!__ballot(m4 <= thr)) continue;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int e = 4 * g + q;
                offer(sv[e], col[e], skip[e] || !(sv[e] <= thr));
            }
        }
    }
    return mine;
}


// Set bits of a wave mask as a 32-bit count on the scalar unit (a count of a
// 64-bit mask compared directly would be widened to a 64-bit vector compare).
__device__ __forceinline__ int mask_count(uint64_t b) {
    int r;
    asm("s_bcnt1_i32_b64 %0, %1" : "=s"(r) : "s"(b));
    return r;
}

__device__ __forceinline__ int wave_count(bool p) { return mask_count(__ballot(p)); }

// a where the lane's bit of the wave mask is set, else b (one select; written
// out so that the operands are computed for every lane rather than under a
// changed exec mask)
__device__ __forceinline__ uint32_t select_by_mask(uint64_t mask, uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(b), "v"(a), "s"(mask));
    return r;
}

// The loads of a short row (n <= 64 * E) for row_topk_rank_vals: column
// e * 64 + lane into x[e], by buffer loads whose range is the row (loads past
// it return 0 and touch no memory).
template <int E>
__device__ __forceinline__ void rank_row_load(const float* __restrict__ row, int n, float (&x)[E]) {
    const int lane = threadIdx.x & (kWave - 1);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(row), (short)0, n * 4, kBufferRsrcWord3);
#pragma unroll
    for (int e = 0; e < E; ++e)
        x[e] = __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(rs, lane * 4 + e * (kWave * 4), 0, 0));
}

// The KK smallest entries of a short row u (n <= 64 * E, diagonal left out)
// by one wave, from the values rank_row_load read: lane l < KK gets the l-th
// smallest as ord32(s) << 32 | column (kTopkNone past the row's n - 1
// entries), with no sort and few instructions per entry:
//  - columns past n become NaN, which is never a candidate and which the lane
//    minimum ignores;
//  - the threshold is the (KK+1)-th smallest lane minimum, to 12 bits of the
//    order key and rounded up, the diagonal taking part: one lane minimum may
//    be the diagonal, so at least KK entries that are not lie at or below it;
//  - each column block's candidates are a ballot; their count decides (more
//    than 64: false, the caller falls back to row_topk); every lane writes its
//    entry of each block to the wave's LDS buffer, a candidate at the block's
//    base plus the candidates below it (mbcnt), any other lane to a slot of
//    its own past the candidates' 64;
//  - each candidate's rank is the number of smaller candidates (the diagonal
//    dropped), counted against every candidate read back by broadcast, and
//    the KK smallest are placed by rank.
// wbuf: 128 entries of LDS owned by the calling wave.
template <bool WIDEST, int E, int KK>
__device__ __forceinline__ bool row_topk_rank_vals(const float (&xr)[E], int n, int u,
                                                   uint64_t* wbuf, uint64_t* out) {
    static_assert(KK >= 1 && KK <= 16, "the list lives in lanes 0..15");
    constexpr uint64_t kNone = kTopkNone;
    constexpr int kBits = 12;  // order-key bits the threshold search resolves
    const int lane = threadIdx.x & (kWave - 1);
    float sv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) sv[e] = WIDEST ? -xr[e] : xr[e];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int rem = n - e * kWave;  // wave-uniform: only the last blocks take the branch
        if (rem < kWave) {
            asm volatile("");  // keeps the branch (no select for the whole blocks)
            sv[e] = lane < rem ? sv[e] : __builtin_nanf("");
        }
    }
    float lm = INFINITY;
#pragma unroll
    for (int e = 0; e < E; ++e) lm = fminf(lm, sv[e]);
    float thr = INFINITY;
    if (wave_count(lm < INFINITY) > KK) {
        const uint32_t km = ord32(lm) >> (32 - kBits);
        uint32_t res = 0;
#pragma unroll
        for (int b = kBits - 1; b >= 0; --b) {
            const uint32_t c = res | (1u << b);
            if (wave_count(km < c) <= KK) res = c;
        }
        // res is the bucket of a finite lane minimum, so its top is a number
        thr = ord32_inv((res << (32 - kBits)) | ((1u << (32 - kBits)) - 1));
    }
    uint64_t m[E];
    int first[E];  // candidates before block e
    int total = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        m[e] = __ballot(sv[e] <= thr);
        first[e] = total;
        total += mask_count(m[e]);
    }
    if (total > kWave) return false;
    // columns at wcol[slot], values at wcol[128 + slot]; slots 64 .. 127 are
    // the other lanes' (one per lane).  The slot addresses are LDS (32-bit)
    // addresses.
    typedef __attribute__((address_space(3))) uint32_t lds_u32;
    uint32_t* wcol = (uint32_t*)wbuf;
    const uint32_t wbase = (uint32_t)(size_t)(lds_u32*)wcol;
    const uint32_t dump = wbase + 4u * (kWave + lane);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m[e] >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m[e], 0u));
        const uint32_t cb = __builtin_amdgcn_readfirstlane(wbase + 4u * (uint32_t)first[e]);
        const uint32_t at = select_by_mask(m[e], cb + 4u * below, dump);
        lds_u32* p = (lds_u32*)(size_t)at;
        p[0] = (uint32_t)(e * kWave + lane);
        p[2 * kWave] = __float_as_uint(sv[e]);
    }
    wave_lds_sync();
    uint64_t x = kNone;
    if (lane < total) {
        const uint32_t col = wcol[lane];
        const uint32_t bits = wcol[2 * kWave + lane];
        if ((int)col != u) x = ((uint64_t)ord32(__uint_as_float(bits)) << 32) | col;
    }
    const int valid = total - wave_count(lane < total && x == kNone);
    wave_lds_sync();
    if (lane < total) wbuf[lane] = x;
    wave_lds_sync();
    int rank = 0;
    for (int j = 0; j < total; ++j) rank += wbuf[j] < x ? 1 : 0;
    wave_lds_sync();
    if (x != kNone && rank < KK) wbuf[rank] = x;
    wave_lds_sync();
    *out = lane < KK && lane < valid ? wbuf[lane] : kNone;
    wave_lds_sync();  // the buffer may be written again for the next row
    return true;
}

}  // namespace appd
