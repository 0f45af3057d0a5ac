// The calculation-and-copy fill (arXiv 2407.07058, Section 3 and the argument
// of Section 5), restated over Prim's attachment order.
//
// Prim attaches v_0 = 0, v_1, ..., v_{n-1}; ek[k] is the key of the edge that
// attached v_k.  For a < b the minimax key of the pair (v_a, v_b) is
//     max(ek[a+1], ..., ek[b]).
// (>=: when v_b is attached... more precisely, at step c = argmax the attached
// set {v_0..v_{c-1}} holds v_a but not v_b, and ek[c] is the smallest edge
// leaving it, so every a-b path pays at least ek[c].  <=: take the last step
// t <= a whose key exceeds that maximum; no edge of weight below it leaves
// {v_0..v_{t-1}}, so v_t..v_b all hang off one another through edges no larger
// than the maximum.)  This is the removal order of Algorithm 4 read the other
// way round: the removed edge that first separates two vertices is the largest
// key between their attachment positions.  A row of M is therefore a running
// maximum over ek, outward from the row's own position, gathered back into
// column order.
//
// Columns are processed in blocks of CB original indices.  A prep kernel sorts
// each block's columns by attachment position (slots sp[0..cnt)) and stores
// gap[k] = max ek over (sp[k-1], sp[k]].  For a row at position a, with k* the
// first slot whose position is >= a:
//   slot k >= k*:  max(ek over (a, sp[k*]],  gap[k*+1..k])      (running max up)
//   slot k <  k*:  max(gap[k+1..k*-1], ek over (sp[k*-1], a])    (running max down)
// The two partial ranges next to a are read from ek directly (a wave-wide max);
// when the row's own column lies in the block (sp[k*] == a) it is the diagonal
// and both boundaries are gap entries.  One wave owns a row of one block: a
// running max within each lane's S = CB/64 consecutive slots, a cross-lane
// inclusive scan, a write into the wave's LDS row buffer, then a gather through
// slot_of_col to coalesced stores of M and idx.
#pragma once

#include "appd_device.h"

namespace appd {

// Block prep: one workgroup (256 threads) per column block.
template <int CB>
__device__ __forceinline__ void fill_prep_block(const int32_t* __restrict__ pos,
                                                const uint64_t* __restrict__ ek, int n, int blk,
                                                uint16_t* __restrict__ blk_sp,
                                                uint16_t* __restrict__ blk_slot,
                                                uint64_t* __restrict__ blk_gap, uint32_t* keys) {
    const int j0 = blk * CB;
    const int cnt = min(CB, n - j0);
    for (int c = threadIdx.x; c < CB; c += blockDim.x)
        keys[c] = c < cnt ? (((uint32_t)pos[j0 + c] << 16) | (uint32_t)c) : 0xffffffffu;
    __syncthreads();
    // bitonic sort, ascending
    for (int size = 2; size <= CB; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < CB / 2; i += blockDim.x) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool asc = (lo & size) == 0;
                const uint32_t x = keys[lo], y = keys[hi];
                if ((x > y) == asc) {
                    keys[lo] = y;
                    keys[hi] = x;
                }
            }
            __syncthreads();
        }
    }
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
        const uint32_t kk = keys[k];
        const int sp = (int)(kk >> 16);
        const int col = (int)(kk & 0xffffu);
        blk_sp[j0 + k] = (uint16_t)sp;
        blk_slot[j0 + col] = (uint16_t)k;
        uint64_t g = 0;
        if (k > 0) {
            const int lo = (int)(keys[k - 1] >> 16) + 1;
            for (int s = lo; s <= sp; ++s) g = umax64(g, ek[s]);
        }
        blk_gap[j0 + k] = g;
    }
}

// One column block, rows [r0, r1), waves of the workgroup take rows in turn.
// s_R: this wave's row buffer of CB keys.
template <int CB, bool WIDEST>
__device__ __forceinline__ void fill_rows_block(const int32_t* __restrict__ pos,
                                                const uint64_t* __restrict__ ek, int n,
                                                int j0, int cnt, int r0, int r1,
                                                const uint16_t* s_sp, const uint16_t* s_slot,
                                                const uint64_t* s_gap, uint64_t* s_R,
                                                float* __restrict__ M, int32_t* __restrict__ idx,
                                                int nwaves) {
    constexpr int S = CB / kWave;
    static_assert(S >= 1 && S <= kWave, "CB must be in [64, 4096]");
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    for (int i = r0 + wid; i < r1; i += nwaves) {
        const int a = pos[i];
        // k* = number of slots whose position is below a
        const int last = lane * S + S - 1;
        const bool below = s_sp[last] < a;  // padded slots hold 0xffff
        const int nbl = __popcll(__ballot(below));
        const int base = nbl * S;
        const bool part = (lane < S) && (base + lane < CB) && (s_sp[min(base + lane, CB - 1)] < a);
        const int ks = base + __popcll(__ballot(part));
        const bool diag = ks < cnt && (int)s_sp[ks] == a;

        uint64_t bl = 0, br = 0;
        if (diag) {
            bl = ks > 0 ? s_gap[ks] : 0ull;
        } else {
            const int lo = ks > 0 ? (int)s_sp[ks - 1] + 1 : a + 1;
            const int hi = ks < cnt ? (int)s_sp[ks] : a;
            for (int s = lo + lane; s <= hi; s += kWave) {
                const uint64_t e = ek[s];
                if (s <= a) bl = umax64(bl, e);
                else br = umax64(br, e);
            }
            bl = wave_max_u64(bl);
            br = wave_max_u64(br);
        }

        // E[k]: the key crossed when stepping from slot k toward the row
        // (k >= k*: the step from slot k-1, or from a, to slot k;
        //  k <  k*: the step from slot k to slot k+1, or to a).
        auto E = [&](int k) -> uint64_t {
            if (k > ks) return k < cnt ? s_gap[k] : 0ull;
            if (k == ks) return diag ? 0ull : br;
            if (k == ks - 1) return bl;
            return s_gap[k + 1];
        };
        const int k0 = lane * S;
        uint64_t up = 0, dn = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int k = k0 + q;
            const uint64_t e = E(k);
            if (k >= ks) up = umax64(up, e);
            else dn = umax64(dn, e);
        }
        uint64_t up_in = wave_incl_max_up(up, lane);
        up_in = shfl_up_u64(up_in, 1);
        if (lane == 0) up_in = 0;
        uint64_t dn_in = wave_incl_max_down(dn, lane);
        dn_in = shfl_down_u64(dn_in, 1);
        if (lane == kWave - 1) dn_in = 0;
        uint64_t run = up_in;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int k = k0 + q;
            if (k >= ks) {
                run = umax64(run, E(k));
                s_R[k] = run;
            }
        }
        run = dn_in;
#pragma unroll
        for (int q = S - 1; q >= 0; --q) {
            const int k = k0 + q;
            if (k < ks) {
                run = umax64(run, E(k));
                s_R[k] = run;
            }
        }
        wave_lds_sync();

        float* mrow = M + (size_t)i * (size_t)n + j0;
        int32_t* irow = idx + (size_t)i * (size_t)n + j0;
        for (int c = lane; c < cnt; c += kWave) {
            const uint64_t key = s_R[s_slot[c]];
            mrow[c] = key ? key_weight<WIDEST>(key) : 0.0f;
            irow[c] = key ? (int32_t)(uint32_t)key : -1;
        }
        wave_lds_sync();
    }
}

}  // namespace appd
