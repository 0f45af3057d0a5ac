// Batched APPD over many independent graphs of uneven size, packed back to
// back: graph g's W, M and idx start at element offsets[g] (= sum of n_h^2 over
// h < g) and its O(n) tree arrays at noff[g] (= sum of n_h).
//
// Graphs are grouped into size classes and, within the whole batch, listed by
// decreasing n (longest processing time first): workgroups are dispatched in
// blockIdx order, so the largest graphs -- whose Prim chains are the longest --
// start first and the small ones fill in behind them.
//
// Phase 1, one workgroup per graph: Prim (appd_prim.h) with NT threads and CH
// vertices per thread, chosen by the graph's class.
// Phase 2, many workgroups per graph: each takes kBatchRows rows of one graph.
// Every graph here fits in a single column block (n <= CB), so the block's
// sorted slots are the attachment positions themselves (slot k = position k,
// gap[k] = ek[k], slot_of_col = pos) and no prep kernel is needed.
#include "appd_fill.h"
#include "appd_internal.h"
#include "appd_prim.h"

namespace appd {

constexpr int kBatchFillThreads = 256;
constexpr int kBatchRows = 16;

// size classes: n <= 64, 256, 1024, 2048
constexpr int kClassMaxN[kBatchClasses] = {64, 256, 1024, 2048};

template <int NT, int CH, bool WIDEST>
__global__ __launch_bounds__(NT) void prim_batched_kernel(const float* __restrict__ W,
                                                          const int64_t* __restrict__ offsets,
                                                          const int32_t* __restrict__ ns,
                                                          const int32_t* __restrict__ perm,
                                                          const int64_t* __restrict__ noff,
                                                          int first, BatchTree tree) {
    __shared__ uint64_t red_key[2 * (NT / kWave)];
    __shared__ int32_t red_v[2 * (NT / kWave)];
    const int g = perm[first + blockIdx.x];
    const int n = ns[g];
    const int64_t o = noff[g];
    PrimOut out{tree.order + o, tree.ek + o, tree.pos + o, tree.parent + o};
    prim_run<NT, CH, WIDEST>(W + offsets[g], n, out, red_key, red_v);
}

template <int CB, bool WIDEST>
__global__ __launch_bounds__(kBatchFillThreads) void fill_batched_kernel(
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ perm, const int64_t* __restrict__ noff,
    const int32_t* __restrict__ chunk_start, int first, int count, BatchTree tree,
    float* __restrict__ M, int32_t* __restrict__ idx) {
    constexpr int NWV = kBatchFillThreads / kWave;
    __shared__ uint16_t s_sp[CB];
    __shared__ __align__(16) uint16_t s_slot[CB];
    __shared__ uint64_t s_gap[CB];
    __shared__ uint64_t s_R[NWV][CB];
    // which graph of this class, and which chunk of its rows
    const int b = blockIdx.x;
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
    const int r0 = chunk * kBatchRows;
    const int r1 = min(n, r0 + kBatchRows);
    fill_rows_block<CB, WIDEST, false>(pos, ek, n, 0, n, r0, r1, s_sp, s_slot, s_gap,
                                s_R[threadIdx.x / kWave], M + offsets[g], idx + offsets[g], NWV);
}

int batch_class_of(int n) {
    for (int c = 0; c < kBatchClasses; ++c)
        if (n <= kClassMaxN[c]) return c;
    return -1;
}

int batch_rows_per_chunk() { return kBatchRows; }

template <bool WIDEST>
static hipError_t run_batched_t(const float* W, const int64_t* offsets, const int32_t* ns,
                                const BatchPlan& plan, const BatchTree& tree, float* M,
                                int32_t* idx, hipStream_t s) {
    // phase 1: Prim per graph, one launch per class (largest first)
    for (int c = kBatchClasses - 1; c >= 0; --c) {
        const int first = plan.class_first[c], count = plan.class_count[c];
        if (!count) continue;
        switch (c) {
            case 0:
                APPD_LAUNCH("prim_batched_kernel", s,
                    prim_batched_kernel<64, 1, WIDEST><<<count, 64, 0, s>>>(W, offsets, ns,
                        plan.perm, plan.noff, first, tree));
                break;
            case 1:
                APPD_LAUNCH("prim_batched_kernel", s,
                    prim_batched_kernel<64, 4, WIDEST><<<count, 64, 0, s>>>(W, offsets, ns,
                        plan.perm, plan.noff, first, tree));
                break;
            case 2:
                APPD_LAUNCH("prim_batched_kernel", s,
                    prim_batched_kernel<256, 4, WIDEST><<<count, 256, 0, s>>>(W, offsets, ns,
                        plan.perm, plan.noff, first, tree));
                break;
            default:
                APPD_LAUNCH("prim_batched_kernel", s,
                    prim_batched_kernel<256, 8, WIDEST><<<count, 256, 0, s>>>(W, offsets, ns,
                        plan.perm, plan.noff, first, tree));
                break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // phase 2: fill, one launch per class
    for (int c = kBatchClasses - 1; c >= 0; --c) {
        const int first = plan.class_first[c], count = plan.class_count[c];
        if (!count) continue;
        const int blocks = plan.class_chunks[c];
        switch (c) {
            case 0:
                APPD_LAUNCH("fill_batched_kernel", s,
                    fill_batched_kernel<64, WIDEST><<<blocks, kBatchFillThreads, 0, s>>>(offsets,
                        ns, plan.perm, plan.noff, plan.chunk_start, first, count, tree, M, idx));
                break;
            case 1:
                APPD_LAUNCH("fill_batched_kernel", s,
                    fill_batched_kernel<256, WIDEST><<<blocks, kBatchFillThreads, 0, s>>>(offsets,
                        ns, plan.perm, plan.noff, plan.chunk_start, first, count, tree, M, idx));
                break;
            case 2:
                APPD_LAUNCH("fill_batched_kernel", s,
                    fill_batched_kernel<1024, WIDEST><<<blocks, kBatchFillThreads, 0, s>>>(offsets,
                        ns, plan.perm, plan.noff, plan.chunk_start, first, count, tree, M, idx));
                break;
            default:
                APPD_LAUNCH("fill_batched_kernel", s,
                    fill_batched_kernel<2048, WIDEST><<<blocks, kBatchFillThreads, 0, s>>>(offsets,
                        ns, plan.perm, plan.noff, plan.chunk_start, first, count, tree, M, idx));
                break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t run_batched(const float* W, const int64_t* offsets, const int32_t* ns,
                       const BatchPlan& plan, const BatchTree& tree, int mode, float* M,
                       int32_t* idx, hipStream_t s) {
    return mode == 1 ? run_batched_t<true>(W, offsets, ns, plan, tree, M, idx, s)
                     : run_batched_t<false>(W, offsets, ns, plan, tree, M, idx, s);
}

}  // namespace appd
