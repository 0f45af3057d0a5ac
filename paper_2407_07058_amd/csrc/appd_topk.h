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


}  // namespace appd
