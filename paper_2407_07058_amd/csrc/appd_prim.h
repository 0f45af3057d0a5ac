// Prim's minimum spanning tree on a dense weight matrix, run by one workgroup
// (arXiv 2407.07058, Section 3: the first step of the implementation is a
// minimum spanning tree built with Prim's algorithm in O(n^2)).
//
// Layout: NT threads cooperate on one graph; thread t owns vertices
// v = t + NT*j (j < CH), so one row of W is read with fully coalesced dword
// loads (each wave reads 256 contiguous bytes per instruction).  For every
// owned unvisited vertex the thread keeps, in registers, the best edge to the
// tree found so far as (weight, parent).  For a fixed vertex v the flat index
// flat(x,v) grows with x, so "smaller weight, then smaller flat index" is
// "smaller weight, then smaller parent id" -- the tie rule needs no flat index
// during the update.  A visited vertex holds NaN, which no comparison selects.
//
// With more than 24 vertices per thread the parents of the best edges live in
// LDS as 16-bit ids (kp_lds, NT * CH entries, one per owned vertex slot; n <=
// 46340 fits), so that the weights and the streamed row stay in registers
// without spilling; they are read only on a tie, a rescan and an attachment.
//
// Each step: the thread's best key (packed 64-bit, see appd_device.h) is
// reduced across the wave with DPP moves and across waves through LDS (one
// barrier per step, double-buffered slots); the winner p is recorded; row p is
// streamed and the keys updated.  Only the thread that owned p rescans its
// vertices; the others fold the best improved vertex into their running best.
#pragma once

#include "appd_device.h"

namespace appd {

struct PrimOut {
    int32_t* order;   // order[k] = vertex attached at step k (order[0] = 0)
    uint64_t* ek;     // ek[k] = key of the edge that attached order[k]; ek[0] = 0
    int32_t* pos;     // pos[v] = k with order[k] = v
    int32_t* parent;  // parent[v] = tree vertex v attached to; parent[0] = -1
};

// Whether prim_run keeps the parents in LDS (the caller then passes kp_lds).
template <int CH>
constexpr bool prim_parents_in_lds() {
    return CH > 24;
}

template <int NT, int CH, bool WIDEST>
__device__ __forceinline__ void prim_run(const float* __restrict__ W, int n, PrimOut out,
                                         uint64_t* red_key, int32_t* red_v,
                                         uint16_t* kp_lds = nullptr) {
    static_assert((NT & (NT - 1)) == 0 && NT >= kWave, "NT must be a power of two >= 64");
    constexpr int NW = NT / kWave;
    constexpr bool KPL = prim_parents_in_lds<CH>();
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int wid = t / kWave;
    const uint32_t un = (uint32_t)n;
    const float qnan = __uint_as_float(0x7fc00000u);

    float kw[CH];
    int32_t kp[KPL ? 1 : CH];
    auto getkp = [&](int j) -> int32_t { return KPL ? (int32_t)kp_lds[t + NT * j] : kp[j]; };
    auto setkp = [&](int j, int32_t p) {
        if (KPL) kp_lds[t + NT * j] = (uint16_t)p;
        else kp[j] = p;
    };
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int v = t + NT * j;
        setkp(j, 0);
        if (v < n && v != 0) {
            const float w = W[v];
            kw[j] = WIDEST ? -w : w;
        } else {
            kw[j] = qnan;
        }
    }

    uint64_t bkey;
    int32_t bv;
    auto rescan = [&]() {
        bkey = ~0ull;
        bv = -1;
        // the vertex ids are recomputed here, not kept live across the steps
        // (CH of them would take as many registers)
        int tt = t;
        asm volatile("" : "+v"(tt));
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            if (kw[j] == kw[j]) {
                const uint32_t v = (uint32_t)(tt + NT * j);
                const uint64_t k = make_key(kw[j], flat_idx((uint32_t)getkp(j), v, un));
                if (k < bkey) {
                    bkey = k;
                    bv = (int32_t)v;
                }
            }
        }
    };
    rescan();
    if (t == 0) {
        out.order[0] = 0;
        out.ek[0] = 0;
        out.pos[0] = 0;
        out.parent[0] = -1;
    }

    for (int k = 1; k < n; ++k) {
        // ---- argmin over all unvisited vertices
        const uint64_t wk = wave_min_u64(bkey);
        const uint64_t bal = __ballot(bkey == wk);
        const int src = __ffsll((unsigned long long)bal) - 1;
        const int32_t wv = __builtin_amdgcn_readlane(bv, src);
        const int slot = (k & 1) * NW;
        if (lane == 0) {
            red_key[slot + wid] = wk;
            red_v[slot + wid] = wv;
        }
        __syncthreads();
        uint64_t gk = red_key[slot];
        int32_t p = red_v[slot];
#pragma unroll
        for (int w = 1; w < NW; ++w) {
            const uint64_t kk = red_key[slot + w];
            if (kk < gk) {
                gk = kk;
                p = red_v[slot + w];
            }
        }

        // A NaN weight (a violated precondition) can leave no selectable
        // vertex; keep every address in bounds and carry on deterministically.
        if (p < 0 || p >= n) p = 0;

        // ---- stream row p: buffer loads over the row's range (columns past n
        // read 0 and touch no memory), one offset register for all of them.
        // Above 32 vertices per thread the row goes through a ring of RB
        // registers: the load of slot j + RB is issued as slot j is used.
        const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(W + (size_t)p * (size_t)n), (short)0, n * 4, 0x00020000);
        constexpr int RB = CH > 32 ? (CH + 1) / 2 : CH;
        auto load = [&](int j) {
            return __builtin_bit_cast(float,
                                      __builtin_amdgcn_raw_buffer_load_b32(rs, 4 * t, 4 * NT * j, 0));
        };
        float r[RB];
#pragma unroll
        for (int j = 0; j < RB; ++j) r[j] = load(j);

        if (t == 0) {
            out.order[k] = p;
            out.ek[k] = gk;
            out.pos[p] = k;
        }
        const bool mine = (p & (NT - 1)) == t;
        if (mine) {
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                if (t + NT * j == p) {
                    out.parent[p] = getkp(j);
                    kw[j] = qnan;
                }
            }
        }

        // ---- key update with row p
        bool have = false;
        float cw = 0.0f;
        int32_t cv = 0;
        int tu = t;
        asm volatile("" : "+v"(tu));
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const float x = r[j % RB];
            if (j + RB < CH) r[j % RB] = load(j + RB);
            const float w = WIDEST ? -x : x;
            const float cur = kw[j];
            bool upd = w < cur;
            if (!upd && w == cur) upd = p < getkp(j);  // a tie: the smaller parent id
            if (upd) {
                kw[j] = w;
                setkp(j, p);
                if (!have || w < cw) {  // v grows with j: ties keep the smaller v
                    have = true;
                    cw = w;
                    cv = tu + NT * j;
                }
            }
        }
        if (mine) {
            rescan();
        } else if (have) {
            const uint64_t c = make_key(cw, flat_idx((uint32_t)p, (uint32_t)cv, un));
            if (c < bkey) {
                bkey = c;
                bv = cv;
            }
        }
    }
}

}  // namespace appd
