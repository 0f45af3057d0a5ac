// Batched APPD over many independent graphs of uneven size, packed back to
// back: graph g's W, M and idx start at element offsets[g] (= sum of n_h^2 over
// h < g) and its O(n) tree arrays at noff[g] (= sum of n_h).
//
// Graphs are grouped into size classes and, within the whole batch, listed by
// decreasing n (longest processing time first): workgroups are dispatched in
// blockIdx order, so the largest graphs -- whose Prim chains are the longest --
// start first and the small ones fill in behind them.  Each class is one Prim
// launch and one fill launch in order on one stream; classes are spread over
// up to plan.streams streams (forked from and joined back into the caller's
// stream with events), so the short classes' Prim and fill run beside the
// longest class's Prim chains: the largest class alone on the caller's
// stream, the others in turn on the side streams.
//
// Phase 1, one workgroup per graph: Prim (appd_prim.h) with the class's
// workgroup size (plan.class_threads) and ceil(class max / threads) vertices
// per thread.
// Phase 2, many workgroups per graph: each takes plan.class_rows rows of one
// graph.  Every graph fits in a single column block (n <= CB), so the block's
// sorted slots are the attachment positions themselves (slot k = position k,
// gap[k] = ek[k], slot_of_col = pos) and no prep kernel is needed.
#include <mutex>

#include "appd.h"
#include "appd_fill.h"
#include "appd_internal.h"
#include "appd_prim.h"

namespace appd {

constexpr int kBatchFillThreads = 256;

template <int NT, int CH, bool WIDEST>
__global__ __launch_bounds__(NT) void prim_batched_kernel(const float* __restrict__ W,
                                                          const int64_t* __restrict__ offsets,
                                                          const int32_t* __restrict__ ns,
                                                          const int32_t* __restrict__ perm,
                                                          const int64_t* __restrict__ noff,
                                                          int first, BatchTree tree,
                                                          int32_t* __restrict__ tstats) {
    __shared__ uint64_t red_key[2 * (NT / kWave)];
    __shared__ int32_t red_v[2 * (NT / kWave)];
    const int g = perm[first + blockIdx.x];
    if (threadIdx.x == 0) tstats[g] = -1;  // Prim's algorithm
    const int n = ns[g];
    const int64_t o = noff[g];
    PrimOut out{tree.order + o, tree.ek + o, tree.pos + o, tree.parent + o};
    prim_run<NT, CH, WIDEST>(W + offsets[g], n, out, red_key, red_v);
}

template <int CB, bool WIDEST>
__global__ __launch_bounds__(kBatchFillThreads) void fill_batched_kernel(
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ perm, const int64_t* __restrict__ noff,
    const int32_t* __restrict__ chunk_start, int first, int count, int chunk_base, int rows,
    BatchTree tree, float* __restrict__ M, int32_t* __restrict__ idx) {
    constexpr int NWV = kBatchFillThreads / kWave;
    __shared__ uint16_t s_sp[CB];
    __shared__ __align__(16) uint16_t s_slot[CB];
    __shared__ uint64_t s_gap[CB];
    __shared__ uint64_t s_R[NWV][CB];
    // which graph of this class, and which chunk of its rows (chunk numbers
    // count from the class's first graph; this launch covers graphs
    // first .. first + count - 1, from chunk chunk_base on)
    const int b = chunk_base + (int)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {  // last gi with chunk_start[first+gi] <= b
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_start[first + mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int gi = first + lo;
    const int g = perm[gi];
    const int n = ns[g];
    const int chunk = b - chunk_start[gi];
    // a work table that does not match this launch (never for a plan the host
    // checks accepted) must not turn into writes outside the graph
    if (chunk < 0 || (int64_t)chunk * rows >= n) return;
    const int64_t o = noff[g];
    const int32_t* pos = tree.pos + o;
    const uint64_t* ek = tree.ek + o;
    for (int k = threadIdx.x; k < CB; k += kBatchFillThreads) {
        const bool in = k < n;
        s_sp[k] = in ? (uint16_t)k : (uint16_t)0xffff;
        s_slot[k] = in ? (uint16_t)pos[k] : (uint16_t)0;
        s_gap[k] = in ? ek[k] : 0ull;
    }
    __syncthreads();
    const int r0 = chunk * rows;
    const int r1 = min(n, r0 + rows);
    fill_rows_block<CB, WIDEST, false>(pos, ek, n, 0, n, r0, r1, s_sp, s_slot, s_gap,
                                       s_R[threadIdx.x / kWave], M + offsets[g],
                                       idx + offsets[g], NWV);
}

// Classes of graphs with n > 256 are filled on 32-bit slot codes like the
// single-graph path: one prep workgroup per (graph, column block of 1024)
// builds the block's tables (fill_prep_block), then the coded fill writes the
// rows.  Its per-row work does not grow with the 64-bit keys, and rows whose M
// and idx starts are misaligned alike are written four columns per 16-byte
// store.  Smaller graphs keep the 64-bit fill above (a 1024-column block would
// be mostly padding for them).
constexpr int kCodedCB = 1024;
constexpr int kCodedMinClass = 3;  // n in (256, 512] and above
constexpr int kCodedBits = (2048 + 31) / 32;

template <bool WIDEST>
__global__ __launch_bounds__(kCodedCB) void fill_prep_batched_kernel(
    const int32_t* __restrict__ ns, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ noff, int first, int bpg, BatchTree tree, BatchBlk blk) {
    __shared__ uint32_t keys[kCodedCB];
    __shared__ uint32_t bits[kCodedBits];
    __shared__ int32_t wpre[kCodedBits];
    __shared__ uint64_t gap[kCodedCB];
    __shared__ uint64_t srt[kCodedCB];
    const int gi = first + (int)blockIdx.x / bpg, b = (int)blockIdx.x % bpg;
    const int g = perm[gi];
    const int n = ns[g];
    if (b * kCodedCB >= n) return;  // whole workgroup: no barrier is skipped by part of it
    const int64_t o = noff[g];
    fill_prep_block<kCodedCB, WIDEST>(tree.pos + o, tree.ek + o, n, b, blk.sp + o, blk.slot + o,
                                      blk.code + o, blk.dM + o, blk.dI + o, blk.sorted + o, keys,
                                      bits, wpre, gap, srt);
}

template <bool WIDEST>
__global__ __launch_bounds__(kBatchFillThreads) void fill_coded_batched_kernel(
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ perm, const int64_t* __restrict__ noff,
    const int32_t* __restrict__ chunk_start, int first, int count, int chunk_base, int rows,
    BatchTree tree, BatchBlk blk, float* __restrict__ M, int32_t* __restrict__ idx) {
    constexpr int CB = kCodedCB;
    constexpr int NWV = kBatchFillThreads / kWave;
    __shared__ uint16_t s_sp[CB];
    __shared__ __align__(16) uint16_t s_slot[CB];
    __shared__ uint64_t s_sorted[CB];
    __shared__ float s_dM[CB + 2 * NWV];
    __shared__ int32_t s_dI[CB + 2 * NWV];
    __shared__ uint32_t s_R[NWV][CB];
    // graph and row chunk as in fill_batched_kernel; blockIdx.y = column block
    const int b = chunk_base + (int)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_start[first + mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int gi = first + lo;
    const int g = perm[gi];
    const int n = ns[g];
    const int chunk = b - chunk_start[gi];
    const int j0 = (int)blockIdx.y * CB;
    if (chunk < 0 || (int64_t)chunk * rows >= n || j0 >= n) return;
    const int cnt = min(CB, n - j0);
    const int64_t o = noff[g];
    for (int k = threadIdx.x; k < CB; k += kBatchFillThreads) {
        const bool in = k < cnt;
        s_sp[k] = in ? blk.sp[o + j0 + k] : (uint16_t)0xffff;
        s_slot[k] = in ? blk.slot[o + j0 + k] : (uint16_t)0;
        s_sorted[k] = in ? blk.sorted[o + j0 + k] : ~0ull;
        s_dM[k] = in ? blk.dM[o + j0 + k] : 0.0f;
        s_dI[k] = in ? blk.dI[o + j0 + k] : -1;
    }
    __syncthreads();
    const int r0 = chunk * rows;
    const int r1 = min(n, r0 + rows);
    float* Mg = M + offsets[g];
    int32_t* Ig = idx + offsets[g];
    const bool vec = (n % 4 == 0) && ((((uintptr_t)Mg) | ((uintptr_t)Ig)) & 15u) == 0;
    uint32_t* row_buf = s_R[threadIdx.x / kWave];
    if (vec)
        fill_rows_block_coded<CB, WIDEST, true, true>(tree.pos + o, tree.ek + o, n, j0, cnt, r0, r1, s_sp,
                                                s_slot, blk.code + o + j0, s_sorted, s_dM, s_dI,
                                                row_buf, Mg, Ig, NWV);
    else
        fill_rows_block_coded<CB, WIDEST, false, true>(tree.pos + o, tree.ek + o, n, j0, cnt, r0, r1,
                                                 s_sp, s_slot, blk.code + o + j0, s_sorted, s_dM,
                                                 s_dI, row_buf, Mg, Ig, NWV);
}

// The fill of graphs whose trees came from btree_finish_kernel, which leaves
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
template <int S, bool WIDEST>
__global__ __launch_bounds__(kBatchFillThreads) void fill_pos_kernel(
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ perm, const int64_t* __restrict__ noff,
    const int32_t* __restrict__ chunk_start, int first, int count, int chunk_base, int rows,
    BatchTree tree, BatchBlk blk, float* __restrict__ M, int32_t* __restrict__ idx) {
    constexpr int CB = kWave * S;
    constexpr int NWV = kBatchFillThreads / kWave;
    constexpr int RB = CB + 8;  // row buffer: columns 0 .. CB, shifted by up to 3
    __shared__ uint16_t s_rk[CB];
    __shared__ uint16_t s_pos[CB];
    __shared__ int2 s_mi[CB];
    __shared__ __align__(16) uint16_t s_R[NWV][RB];
    const int b = chunk_base + (int)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_start[first + mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int gi = first + lo;
    const int g = perm[gi];
    const int n = ns[g];
    const int chunk = b - chunk_start[gi];
    if (chunk < 0 || (int64_t)chunk * rows >= n || n > CB) return;
    const int64_t o = noff[g];
    for (int k = threadIdx.x; k < CB; k += kBatchFillThreads) {
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
    const int r0 = chunk * rows, r1 = min(n, r0 + rows);
    for (int i = r0 + wid; i < r1; i += NWV) {
        float* mrow = Mg + (size_t)i * n;
        int32_t* irow = Ig + (size_t)i * n;
        const int mis = (int)(((uintptr_t)mrow >> 2) & 3u);
        // column c's code at R[c]; the 16-byte groups of the row start at
        // columns c with c + mis a multiple of 4
        uint16_t* R = s_R[wid] + mis;
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
            }
        } else {
            for (int c = lane; c < n; c += kWave) put1(c);
        }
        wave_lds_sync();
    }
}

int batch_class_of(int n) {
    for (int c = 0; c < kBatchClasses; ++c)
        if (n <= kClassMaxN[c]) return c;
    return -1;
}

// Prim workgroup sizes a class supports: 64..1024 threads, at most 8 vertices
// per thread, no more threads than twice the class's largest n.
bool batch_threads_ok(int c, int threads) {
    if (c < 0 || c >= kBatchClasses) return false;
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024)
        return false;
    const int ch = (kClassMaxN[c] + threads - 1) / threads;
    return ch <= 8 && threads <= 2 * kClassMaxN[c];
}

template <bool WIDEST>
static hipError_t launch_prim_class(int c, int threads, int first, int count, const float* W,
                                    const int64_t* offsets, const int32_t* ns,
                                    const BatchPlan& plan, const BatchTree& tree,
                                    hipStream_t s) {
    const int ch = (kClassMaxN[c] + threads - 1) / threads;
#define APPD_PRIM_B(NT, CH)                                                      \
    if (threads == NT && ch == CH) {                                             \
        APPD_LAUNCH("prim_batched_kernel", s,                                    \
                    prim_batched_kernel<NT, CH, WIDEST><<<count, NT, 0, s>>>(    \
                        W, offsets, ns, plan.perm, plan.noff, first, tree,       \
                        plan.tstats));                                           \
        return hipGetLastError();                                                \
    }
    APPD_PRIM_B(64, 1)
    APPD_PRIM_B(64, 2)
    APPD_PRIM_B(64, 4)
    APPD_PRIM_B(64, 8)
    APPD_PRIM_B(128, 1)
    APPD_PRIM_B(128, 2)
    APPD_PRIM_B(128, 4)
    APPD_PRIM_B(128, 8)
    APPD_PRIM_B(256, 1)
    APPD_PRIM_B(256, 2)
    APPD_PRIM_B(256, 4)
    APPD_PRIM_B(256, 8)
    APPD_PRIM_B(512, 1)
    APPD_PRIM_B(512, 2)
    APPD_PRIM_B(512, 4)
    APPD_PRIM_B(1024, 1)
    APPD_PRIM_B(1024, 2)
#undef APPD_PRIM_B
    return hipErrorInvalidValue;
}

template <bool WIDEST>
static hipError_t launch_fill_class(int c, int first, int count, int chunk_base, int chunks,
                                    int rows,
                                    const int64_t* offsets, const int32_t* ns,
                                    const BatchPlan& plan, const BatchTree& tree,
                                    const BatchBlk& blk, float* M, int32_t* idx, hipStream_t s) {
    if (plan.class_tree[c] == APPD_BATCH_TREE_BORUVKA) {
        // rank tables written by the tree kernel: no prep launch
#define APPD_FILL_P(CC, SS)                                                                     \
        if (c == CC) {                                                                          \
            APPD_LAUNCH("fill_pos_kernel", s,                                                   \
                        fill_pos_kernel<SS, WIDEST><<<chunks, kBatchFillThreads, 0, s>>>(       \
                            offsets, ns, plan.perm, plan.noff, plan.chunk_start, first, count,  \
                            chunk_base, rows, tree, blk, M, idx));                              \
            return hipGetLastError();                                                           \
        }
        APPD_FILL_P(0, 1)
        APPD_FILL_P(1, 2)
        APPD_FILL_P(2, 4)
        APPD_FILL_P(3, 8)
        APPD_FILL_P(4, 16)
        APPD_FILL_P(5, 32)
#undef APPD_FILL_P
        return hipErrorInvalidValue;
    }
    if (c >= kCodedMinClass) {
        const int bpg = (kClassMaxN[c] + kCodedCB - 1) / kCodedCB;
        APPD_LAUNCH("fill_prep_batched_kernel", s,
                    fill_prep_batched_kernel<WIDEST><<<count * bpg, kCodedCB, 0, s>>>(
                        ns, plan.perm, plan.noff, first, bpg, tree, blk));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        APPD_LAUNCH("fill_coded_batched_kernel", s,
                    fill_coded_batched_kernel<WIDEST><<<dim3(chunks, bpg), kBatchFillThreads, 0, s>>>(
                        offsets, ns, plan.perm, plan.noff, plan.chunk_start, first, count,
                        chunk_base, rows, tree, blk, M, idx));
        return hipGetLastError();
    }
#define APPD_FILL_B(CC, CB)                                                           \
    if (c == CC) {                                                                    \
        APPD_LAUNCH("fill_batched_kernel", s,                                         \
                    fill_batched_kernel<CB, WIDEST><<<chunks, kBatchFillThreads, 0, s>>>( \
                        offsets, ns, plan.perm, plan.noff, plan.chunk_start, first,   \
                        count, chunk_base, rows, tree, M, idx));                      \
        return hipGetLastError();                                                     \
    }
    APPD_FILL_B(0, 64)
    APPD_FILL_B(1, 128)
    APPD_FILL_B(2, 256)
    APPD_FILL_B(3, 512)
    APPD_FILL_B(4, 1024)
    APPD_FILL_B(5, 2048)
#undef APPD_FILL_B
    return hipErrorInvalidValue;
}

// Library streams and events for the class fork/join, created once per device
// and kept for the life of the process (default priority).
namespace {
struct SideStreams {
    hipStream_t side[kBatchClasses - 1];
    hipEvent_t fork;
    hipEvent_t join[kBatchClasses - 1];
    bool ready = false;
};
std::mutex g_side_mu;
SideStreams g_side[64];
// Held from the fork record to the last join wait of one batched forward: the
// fork and join events are shared, so two host threads must not interleave
// their record / wait sequences.
std::mutex g_fork_mu;

hipError_t side_streams(SideStreams** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_side_mu);
    SideStreams& ss = g_side[dev];
    if (!ss.ready) {
        for (int k = 0; k < kBatchClasses - 1; ++k) {
            if ((e = hipStreamCreateWithFlags(&ss.side[k], hipStreamNonBlocking)) != hipSuccess)
                return e;
            if ((e = hipEventCreateWithFlags(&ss.join[k], hipEventDisableTiming)) != hipSuccess)
                return e;
        }
        if ((e = hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming)) != hipSuccess) return e;
        ss.ready = true;
    }
    *out = &ss;
    return hipSuccess;
}
}  // namespace

template <bool WIDEST>
static hipError_t run_batched_t(const float* W, const int64_t* offsets, const int32_t* ns,
                                const BatchPlan& plan, const BatchTree& tree,
                                const BatchBlk& blk, float* M, int32_t* idx, hipStream_t s) {
    // classes in launch order: largest first
    int cls[kBatchClasses], nc = 0;
    for (int c = kBatchClasses - 1; c >= 0; --c)
        if (plan.class_count[c]) cls[nc++] = c;
    const int nstreams = max(1, min(plan.streams, nc));
    hipStream_t st[kBatchClasses];
    st[0] = s;
    SideStreams* ss = nullptr;
    hipError_t e;
    std::unique_lock<std::mutex> fork_lock(g_fork_mu, std::defer_lock);
    if (nstreams > 1) {
        fork_lock.lock();
        if ((e = side_streams(&ss)) != hipSuccess) return e;
        if ((e = hipEventRecord(ss->fork, s)) != hipSuccess) return e;
        for (int k = 1; k < nstreams; ++k) {
            st[k] = ss->side[k - 1];
            if ((e = hipStreamWaitEvent(st[k], ss->fork, 0)) != hipSuccess) return e;
        }
    }
    // The largest class (the longest Prim chains and most of the entries) has
    // the caller's stream to itself; the others take the side streams in turn,
    // so that they finish while it still runs.  Split, the largest class's
    // biggest graphs keep the caller's stream, the rest of it takes the first
    // side stream, and the other classes the side streams after it.
    const bool split = nstreams >= 2 && plan.split_count > 0;
    const int others0 = split && nstreams >= 3 ? 2 : 1;
    for (int j = 0; j < nc; ++j) {
        const int c = cls[j];
        const int first = plan.class_first[c], count = plan.class_count[c];
        const int rows = plan.class_rows[c], chunks = plan.class_chunks[c];
        // trees of graphs first .. first + cnt - 1 of class c (rows: their
        // total n, the rows of the Boruvka pass)
        auto trees = [&](int f0, int cnt, int rows_bound, hipStream_t cs) -> hipError_t {
            return plan.class_tree[c] == APPD_BATCH_TREE_BORUVKA
                       ? launch_btree(c, f0, cnt, rows_bound, WIDEST ? 1 : 0, W, offsets, ns, plan,
                                      tree, blk, plan.lists, cs)
                       : launch_prim_class<WIDEST>(c, plan.class_threads[c], f0, cnt, W, offsets,
                                                   ns, plan, tree, cs);
        };
        if (j == 0 && split) {
            const int h = plan.split_count, hc = plan.split_chunks;
            e = trees(first, h, plan.split_vertices, st[0]);
            if (e != hipSuccess) return e;
            e = launch_fill_class<WIDEST>(c, first, h, 0, hc, rows, offsets, ns, plan, tree, blk,
                                          M, idx, st[0]);
            if (e != hipSuccess) return e;
            e = trees(first + h, count - h, plan.class_vertices[c] - plan.split_vertices, st[1]);
            if (e != hipSuccess) return e;
            e = launch_fill_class<WIDEST>(c, first + h, count - h, hc, chunks - hc, rows,
                                          offsets, ns, plan, tree, blk, M, idx, st[1]);
            if (e != hipSuccess) return e;
            continue;
        }
        hipStream_t cs =
            (j == 0 || nstreams == 1) ? st[0] : st[others0 + (j - 1) % (nstreams - others0)];
        e = trees(first, count, plan.class_vertices[c], cs);
        if (e != hipSuccess) return e;
        e = launch_fill_class<WIDEST>(c, first, count, 0, chunks, rows, offsets, ns, plan, tree,
                                      blk, M, idx, cs);
        if (e != hipSuccess) return e;
    }
    if (nstreams > 1) {
        for (int k = 1; k < nstreams; ++k) {
            if ((e = hipEventRecord(ss->join[k - 1], st[k])) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(s, ss->join[k - 1], 0)) != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

hipError_t run_batched(const float* W, const int64_t* offsets, const int32_t* ns,
                       const BatchPlan& plan, const BatchTree& tree, const BatchBlk& blk,
                       int mode, float* M, int32_t* idx, hipStream_t s) {
    return mode == 1 ? run_batched_t<true>(W, offsets, ns, plan, tree, blk, M, idx, s)
                     : run_batched_t<false>(W, offsets, ns, plan, tree, blk, M, idx, s);
}

}  // namespace appd
