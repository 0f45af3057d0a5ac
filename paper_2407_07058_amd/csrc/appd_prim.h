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

template <int NT, int CH, bool WIDEST>
__device__ __forceinline__ void prim_run(const float* __restrict__ W, int n, PrimOut out,
                                         uint64_t* red_key, int32_t* red_v) {
    static_assert((NT & (NT - 1)) == 0 && NT >= kWave, "NT must be a power of two >= 64");
    constexpr int NW = NT / kWave;
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    const int wid = t / kWave;
    const uint32_t un = (uint32_t)n;
    const float qnan = __uint_as_float(0x7fc00000u);

    float kw[CH];
    int32_t kp[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
        const int v = t + NT * j;
        kp[j] = 0;
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
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            if (kw[j] == kw[j]) {
                const uint32_t v = (uint32_t)(t + NT * j);
                const uint64_t k = make_key(kw[j], flat_idx((uint32_t)kp[j], v, un));
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

        // ---- stream row p
        const float* row = W + (size_t)p * (size_t)n;
        float r[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const int v = t + NT * j;
            r[j] = v < n ? row[v] : 0.0f;
        }

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
                    out.parent[p] = kp[j];
                    kw[j] = qnan;
                }
            }
        }

        // ---- key update with row p
        bool have = false;
        float cw = 0.0f;
        int32_t cv = 0;
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            const float w = WIDEST ? -r[j] : r[j];
            const float cur = kw[j];
            const bool upd = (w < cur) || (w == cur && p < kp[j]);
            if (upd) {
                kw[j] = w;
                kp[j] = p;
                if (!have || w < cw) {  // v grows with j: ties keep the smaller v
                    have = true;
                    cw = w;
                    cv = t + NT * j;
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
