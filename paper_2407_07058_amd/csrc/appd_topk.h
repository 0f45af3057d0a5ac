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


// The same KK smallest entries for a short row (n <= 64 * E, no column
// filter) without inserting entries one at a time.  The threshold is taken as
// above (at least KK lane minima, hence at least KK entries, lie at or below
// it, so the KK smallest entries all do); every entry at or below it is
// written to the wave's LDS buffer (a prefix sum over the lanes gives each
// lane its place), one per lane is read back, and a bitonic sort across the
// lanes orders them.  Returns false, leaving *out alone, when more than 64
// entries lie at or below the threshold (then row_topk does the work).
// wbuf: 64 entries of LDS owned by the calling wave.
// The loads of a short row: column e * 64 + lane into x[e] (0 past the row).
template <int E>
__device__ __forceinline__ void short_row_load(const float* __restrict__ row, int n, float (&x)[E]) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int c = e * kWave + lane;
        x[e] = c < n ? row[c] : 0.0f;
    }
}

// row_topk_compact on values already loaded by short_row_load.
template <bool WIDEST, int E, int KK>
__device__ __forceinline__ bool topk_compact_vals(const float (&xr)[E], int n, int u,
                                                  uint64_t* wbuf, uint64_t* out) {
    static_assert(KK >= 1 && KK <= 16, "the list lives in lanes 0..15");
    constexpr uint64_t kNone = kTopkNone;
    const int lane = threadIdx.x & (kWave - 1);
    float sv[E];
    bool skip[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int c = e * kWave + lane;
        sv[e] = WIDEST ? -xr[e] : xr[e];
        skip[e] = c >= n || c == u;
    }
    float lm = INFINITY;
#pragma unroll
    for (int e = 0; e < E; ++e) lm = fminf(lm, skip[e] ? INFINITY : sv[e]);
    float thr = INFINITY;
    if (__popcll(__ballot(lm < INFINITY)) >= KK) {
        const uint32_t km = ord32(lm) >> 16;
        uint32_t res = 0;
        for (int b = 15; b >= 0; --b) {
            const uint32_t c = res | (1u << b);
            if (__popcll(__ballot(km < c)) < KK) res = c;
        }
        thr = res == 0xffffu ? INFINITY : ord32_inv((res << 16) | 0xffffu);
    }
    int cnt = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) cnt += (!skip[e] && sv[e] <= thr) ? 1 : 0;
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    const int total = __builtin_amdgcn_readlane(incl, kWave - 1);
    if (total > kWave) return false;
    int off = incl - cnt;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (!skip[e] && sv[e] <= thr) {
            wbuf[off] = ((uint64_t)ord32(sv[e]) << 32) | (uint32_t)(e * kWave + lane);
            ++off;
        }
    }
    wave_lds_sync();
    uint64_t x = lane < total ? wbuf[lane] : kNone;
    wave_lds_sync();  // the buffer may be written again for the next row
    // ascending bitonic sort of lanes 0 .. P-1 (P: a power of two >= total, >= 16)
    int P = 16;
    while (P < total) P <<= 1;
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const uint64_t y = shfl_xor_u64(x, stride);
            const bool up = (lane & size) == 0;
            const bool lower = (lane & stride) == 0;
            x = (lower == up) ? umin64(x, y) : umax64(x, y);
        }
    }
    *out = lane < KK ? x : kNone;
    return true;
}

template <bool WIDEST, int E, int KK>
__device__ __forceinline__ bool row_topk_compact(const float* __restrict__ row, int n, int u,
                                                 uint64_t* wbuf, uint64_t* out) {
    float x[E];
    short_row_load<E>(row, n, x);
    return topk_compact_vals<WIDEST, E, KK>(x, n, u, wbuf, out);
}

}  // namespace appd
