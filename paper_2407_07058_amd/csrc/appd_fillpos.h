// The position-space fill of one graph's rows (the batched Boruvka classes and
// the persistent batched forward): see fill_pos_rows.
#pragma once

#include "appd_device.h"
#include "appd_internal.h"
#include "appd_wcount.h"

namespace appd {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));

// The fill of graphs whose trees came from bt_finish_graph, which leaves
// per graph (at its noff offset) the rank code of each attachment position
// (blk.slot: 1 + the rank of the position's key among the graph's n - 1 keys,
// 0 at position 0) and each code's weight and flat index (blk.dM, blk.dI; code
// 0 is the diagonal).  A graph is one block of 64 * S slots in position order
// (S = the class's largest n / 64): lane l owns slots S l .. S l + S - 1 and
// keeps the row-independent running maxima of their codes in registers.  For
// the row of the vertex at position a, the code of column c is the largest
// code strictly after a up to pos(c) (or from pos(c) + 1 up to a); the lane
// that holds slot a scans its own slots, the others combine their maxima
// with the maxima of the lanes between them and a (cross-lane scans).  Each
// lane writes its slots' codes to the wave's LDS row buffer at the columns of
// the slots' vertices, so the buffer is the row's codes in column order,
// shifted by the row's misalignment so that every 16-byte group of outputs
// reads its four codes with one 8-byte LDS load.  A code's output pair is one
// 8-byte LDS entry.  Rows are written four columns per 16-byte store where M
// and idx align alike.  The stores are ordinary (write-back) ones: packed rows
// start anywhere in a 128-byte line, and L2 merges the part lines at the ends
// of neighbouring rows before they go to HBM (non-temporal stores sent them as
// part-line writes, about a quarter slower).
// Rows r0 .. r1 - 1 of the graph at position gi of perm, by the NT threads of
// the calling workgroup (every thread calls it); lds: fill_pos_lds_bytes(S, NT)
// bytes, 16-byte aligned.  The caller synchronises the workgroup before
// reusing it.
__host__ __device__ constexpr size_t fill_pos_lds_bytes(int S, int NT) {
    return (size_t)12 * (kWave * S) + (size_t)(NT / kWave) * 2 * (kWave * S + 8);
}

template <int S, int NT, bool WIDEST>
__device__ __forceinline__ void fill_pos_rows(const int64_t* __restrict__ offsets,
                                              const int32_t* __restrict__ ns,
                                              const int32_t* __restrict__ perm,
                                              const int64_t* __restrict__ noff, int gi, int r0,
                                              int r1, BatchTree tree, BatchBlk blk,
                                              float* __restrict__ M, int32_t* __restrict__ idx,
                                              char* lds) {
    constexpr int CB = kWave * S;
    constexpr int NWV = NT / kWave;
    constexpr int RB = CB + 8;  // row buffer: columns 0 .. CB, shifted by up to 3
    int2* s_mi = (int2*)lds;                          // 8 * CB
    uint16_t* s_rk = (uint16_t*)(lds + 8 * CB);       // 2 * CB
    uint16_t* s_pos = (uint16_t*)(lds + 10 * CB);     // 2 * CB
    uint16_t* s_Rall = (uint16_t*)(lds + 12 * CB);    // NWV rows of RB, each 16-byte aligned
    const int g = perm[gi];
    const int n = ns[g];
    const int64_t o = noff[g];
    for (int k = threadIdx.x; k < CB; k += NT) {
        const bool in = k < n;
        s_rk[k] = in ? blk.slot[o + k] : (uint16_t)0;
        s_pos[k] = in ? (uint16_t)tree.pos[o + k] : (uint16_t)0;
        s_mi[k] = in ? make_int2(__float_as_int(blk.dM[o + k]), blk.dI[o + k]) : make_int2(0, -1);
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int k0 = lane * S;
    // the vertices at this lane's slots (slots past n: column n, which no
    // store reads)
    int vt[S];
#pragma unroll
    for (int q = 0; q < S; ++q) vt[q] = k0 + q < n ? tree.order[o + k0 + q] : n;
    __syncthreads();
    // row-independent maxima of this lane's codes: pre[q] over slots k0 .. k0+q,
    // suf[q] over k0+q+1 .. k0+S-1
    uint32_t pre[S], suf[S];
    {
        uint32_t gq[S];
#pragma unroll
        for (int q = 0; q < S; ++q) gq[q] = s_rk[k0 + q];
        uint32_t run = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            run = max(run, gq[q]);
            pre[q] = run;
        }
        run = 0;
#pragma unroll
        for (int q = S - 1; q >= 0; --q) {
            suf[q] = run;
            run = max(run, gq[q]);
        }
    }
    const uint32_t tot = pre[S - 1];
    float* Mg = M + offsets[g];
    int32_t* Ig = idx + offsets[g];
    for (int i = r0 + wid; i < r1; i += NWV) {
        float* mrow = Mg + (size_t)i * n;
        int32_t* irow = Ig + (size_t)i * n;
        const int mis = (int)(((uintptr_t)mrow >> 2) & 3u);
        // column c's code at R[c]; the 16-byte groups of the row start at
        // columns c with c + mis a multiple of 4
        uint16_t* R = s_Rall + wid * RB + mis;
        const int a = s_pos[i];
        const int la = a / S, j = a % S;
        // lane la: its own slots, and what it contributes to the lanes above
        // (codes after a) and below (codes up to a)
        uint32_t upp = 0, dnp = 0;
        if (lane == la) {
            uint32_t gq[S];
#pragma unroll
            for (int q = 0; q < S; ++q) gq[q] = s_rk[k0 + q];
            uint32_t run = 0;
#pragma unroll
            for (int q = 0; q < S; ++q) {
                if (q > j) {
                    run = max(run, gq[q]);
                    R[vt[q]] = (uint16_t)run;
                }
                if (q <= j) dnp = max(dnp, gq[q]);
            }
            upp = run;
            run = 0;
#pragma unroll
            for (int q = S - 1; q >= 0; --q) {
                if (q < j) {
                    run = max(run, gq[q + 1 < S ? q + 1 : q]);
                    R[vt[q]] = (uint16_t)run;
                }
            }
            R[i] = 0;  // the diagonal: the vertex at slot a is i
        }
        upp = (uint32_t)__builtin_amdgcn_readlane((int)upp, la);
        dnp = (uint32_t)__builtin_amdgcn_readlane((int)dnp, la);
        const uint32_t cu = max(upp, wave_excl_max_up_u32(lane > la ? tot : 0u, lane));
        const uint32_t cd = max(dnp, wave_excl_max_down_u32(lane < la ? tot : 0u, lane));
        if (lane > la) {
#pragma unroll
            for (int q = 0; q < S; ++q) R[vt[q]] = (uint16_t)max(pre[q], cu);
        } else if (lane < la) {
#pragma unroll
            for (int q = 0; q < S; ++q) R[vt[q]] = (uint16_t)max(suf[q], cd);
        }
        wave_lds_sync();
        auto put1 = [&](int c) {
            const int2 e = s_mi[R[c]];
            mrow[c] = __int_as_float(e.x);
            irow[c] = e.y;
            count_writes(mrow + c, 1);
            count_writes(irow + c, 1);
        };
        if (mis == (int)(((uintptr_t)irow >> 2) & 3u)) {
            const int h = min(n, (4 - mis) & 3);
            const int nq = (n - h) >> 2;
            const int tail0 = h + 4 * nq;
            if (lane < h) put1(lane);
            if (lane < n - tail0) put1(tail0 + lane);
            for (int m = lane; m < nq; m += kWave) {
                const int c = h + 4 * m;
                const uint2 w = *(const uint2*)(R + c);
                const int2 e0 = s_mi[w.x & 0xffffu], e1 = s_mi[w.x >> 16];
                const int2 e2 = s_mi[w.y & 0xffffu], e3 = s_mi[w.y >> 16];
                const f4v mv = {__int_as_float(e0.x), __int_as_float(e1.x), __int_as_float(e2.x),
                                __int_as_float(e3.x)};
                const i4v iv = {e0.y, e1.y, e2.y, e3.y};
                *(f4v*)(mrow + c) = mv;
                *(i4v*)(irow + c) = iv;
                count_writes(mrow + c, 4);
                count_writes(irow + c, 4);
            }
        } else {
            for (int c = lane; c < n; c += kWave) put1(c);
        }
        wave_lds_sync();
    }
}

}  // namespace appd
