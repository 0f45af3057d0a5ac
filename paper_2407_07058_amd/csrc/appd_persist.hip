// The batched forward as one persistent launch over a work queue.
//
// The graphs of a batch are independent (Algorithm 4 per graph), and each goes
// through three steps with a dependency between them: the candidate lists of
// its rows (a pass over its W), its tree, Prim order and fill tables (one
// workgroup), and the fill of its rows.  Here one launch of as many workgroups
// as the GPU holds at once takes work items from a queue in a fixed order:
//
//   pass items  -- kPersistThreads / 64 consecutive rows of the batch (rows of
//                  the graphs in perm order, largest graphs first), one row per
//                  wave; the tree item of a graph follows the pass item that
//                  holds its last row;
//   tree items  -- one graph: waits until all its rows are counted, then
//                  bt_finish_graph;
//   fill items  -- after every pass and tree item, `rows` rows of one graph:
//                  waits until its tree is done, then fill_pos_rows.
//
// A workgroup takes the next run of kPersistGrab items only when it has
// finished its current run, takes a run's items in order, and an item only
// waits for items earlier in the queue, which running workgroups hold (or
// which come earlier in its own run): the earliest unfinished item never
// waits, so the queue always drains.  The waits are bounded all the same (kPersistSpin polls with
// a sleep between them); one that gives up skips its item and marks the
// GPU's status record, which appd_sync reports.  The latency-bound tree of a
// graph runs while other workgroups stream rows of later graphs, and nothing
// waits for a launch boundary.
//
// Memory order: the waves of a pass item wait for their list stores, and one
// thread releases at device scope for the workgroup before the rows are
// counted; a tree workgroup does the same before the flag of its graph is set
// (a release store); a waiter polls the count or flag with relaxed loads and,
// once it is reached, the whole workgroup acquires at device scope.  (One
// release and one acquire per item: on this GPU a device-scope release writes
// back and an acquire invalidates the caches of the issuing die, so a fence
// per row or per poll would cost more than the work.)
#include <algorithm>

#include "appd.h"
#include "appd_btree.h"
#include "appd_fillpos.h"
#include "appd_internal.h"

namespace appd {
namespace {

constexpr int kPersistSpin = 1 << 20;  // polls before a wait gives up (about a second)
constexpr int kPersistGrab = 8;        // queue items taken per atomic on the queue head

// Polls *p until it reaches `target`; false if kPersistSpin polls pass first,
// or at once when another wait of this launch has given up (*abort set: the
// launch then only drains its queue).  A wait that gives up sets *abort and
// marks the GPU's status record.
__device__ __forceinline__ bool wait_count(const int* p, int target, int* abort, uint32_t* status) {
    for (int k = 0; k < kPersistSpin; ++k) {
        // relaxed polls (an acquiring load would invalidate caches each time);
        // the caller acquires once the count is reached
        if (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) return true;
        if (__hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return false;
        __builtin_amdgcn_s_sleep(2);
    }
    atomicOr(status, kStatusWaitTimeout);
    atomicExch(abort, 1);
    return false;
}

// This wave's stores have completed (reached the device's caches); a release
// fence at device scope by one thread after a barrier then covers the stores
// of the whole workgroup.
__device__ __forceinline__ void wave_stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

__global__ void persist_reset_kernel(int* __restrict__ ctr, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) ctr[i] = 0;
}

// Class limit of a graph of n vertices (the LDS tables of its tree and fill
// are sized by it).
__device__ __forceinline__ int class_max_of(int n) {
    return n <= 64 ? 64 : n <= 128 ? 128 : n <= 256 ? 256 : n <= 512 ? 512 : 1024;
}

template <bool WIDEST>
__global__ __launch_bounds__(kPersistThreads) void batch_persistent_kernel(
    const float* __restrict__ W, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ ns, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ noff, const int32_t* __restrict__ rstart,
    const int32_t* __restrict__ rgraph, uint64_t* __restrict__ lists, BatchTree tree,
    BatchBlk blk, int32_t* __restrict__ tstats, float* __restrict__ M, int32_t* __restrict__ idx,
    const uint2* __restrict__ items, int nitems, int* __restrict__ ctr, int G, int total_rows,
    uint32_t* __restrict__ status) {
    constexpr int NT = kPersistThreads;
    extern __shared__ __align__(16) char s_lds[];
    __shared__ uint64_t s_aux[(bt_aux_bytes<NT>() + 7) / 8];
    __shared__ int s_item, s_ok;
    int* pass_done = ctr + 1;
    int* tree_done = ctr + 1 + G;
    int* abort = ctr + 1 + 2 * G;
    const int t = threadIdx.x, lane = t & (kWave - 1);
    const int wid = __builtin_amdgcn_readfirstlane(t / kWave);
    for (int it = 0, grab_end = 0;; ++it) {
        if (it >= grab_end) {
            // the next kPersistGrab items of the queue (one atomic on the
            // queue head per run, not per item: all workgroups contend for it)
            if (t == 0) s_item = atomicAdd(ctr, kPersistGrab);
            __syncthreads();
            it = s_item;
            grab_end = it + kPersistGrab;
            __syncthreads();
        }
        if (it >= nitems) break;  // workgroup-uniform
        const uint2 d = items[it];
        const uint32_t type = d.x >> 30;
        const int a = (int)(d.x & 0x3fffffffu);
        if (type == kItemPass) {
            // the item's rows, one per wave; then one release for all of them
            const int r = a + wid;
            if (r < total_rows) {
                const int gi = rgraph[r];
                const int n = ns[perm[gi]];
                uint64_t* wbuf = (uint64_t*)s_lds + wid * (2 * kWave);
                if (n <= 256)
                    bt_pass_row<WIDEST, 4>(W, offsets, ns, perm, noff, rstart, rgraph, r, lists, wbuf);
                else if (n <= 512)
                    bt_pass_row<WIDEST, 8>(W, offsets, ns, perm, noff, rstart, rgraph, r, lists, wbuf);
                else
                    bt_pass_row<WIDEST, 16>(W, offsets, ns, perm, noff, rstart, rgraph, r, lists, wbuf);
            }
            wave_stores_done();
            __syncthreads();
            if (t == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                // count the item's rows, one atomic per graph among them
                const int r1 = min(total_rows, a + kPersistThreads / kWave);
                for (int q = a; q < r1;) {
                    const int gq = rgraph[q];
                    int e = q + 1;
                    while (e < r1 && rgraph[e] == gq) ++e;
                    atomicAdd(&pass_done[gq], e - q);
                    q = e;
                }
            }
        } else if (type == kItemTree) {
            const int gi = a;
            const int n = ns[perm[gi]];
            if (t == 0) {
                s_ok = wait_count(&pass_done[gi], n, abort, status) ? 1 : 0;
            }
            __syncthreads();
            if (s_ok) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const BtAux aux = bt_aux_carve<NT>((char*)s_aux);
                const int nmax = class_max_of(n);
                if (nmax <= 512)
                    bt_finish_graph<NT, 1, WIDEST>(W, offsets, ns, perm, noff, gi, nmax, lists, tree,
                                                   tstats, blk, s_lds, aux);
                else
                    bt_finish_graph<NT, 2, WIDEST>(W, offsets, ns, perm, noff, gi, nmax, lists, tree,
                                                   tstats, blk, s_lds, aux);
                wave_stores_done();
                __syncthreads();
                if (t == 0)
                    __hip_atomic_store(&tree_done[gi], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            const int gi = a;
            const int r0 = (int)(d.y & 0xffffu), r1 = r0 + (int)(d.y >> 16);
            if (t == 0) {
                s_ok = wait_count(&tree_done[gi], 1, abort, status) ? 1 : 0;
            }
            __syncthreads();
            if (s_ok) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                switch (class_max_of(ns[perm[gi]])) {
                    case 64:
                        fill_pos_rows<1, NT, WIDEST>(offsets, ns, perm, noff, gi, r0, r1, tree, blk, M,
                                                     idx, s_lds);
                        break;
                    case 128:
                        fill_pos_rows<2, NT, WIDEST>(offsets, ns, perm, noff, gi, r0, r1, tree, blk, M,
                                                     idx, s_lds);
                        break;
                    case 256:
                        fill_pos_rows<4, NT, WIDEST>(offsets, ns, perm, noff, gi, r0, r1, tree, blk, M,
                                                     idx, s_lds);
                        break;
                    case 512:
                        fill_pos_rows<8, NT, WIDEST>(offsets, ns, perm, noff, gi, r0, r1, tree, blk, M,
                                                     idx, s_lds);
                        break;
                    default:
                        fill_pos_rows<16, NT, WIDEST>(offsets, ns, perm, noff, gi, r0, r1, tree, blk, M,
                                                      idx, s_lds);
                        break;
                }
            }
        }
        __syncthreads();  // the item's LDS and s_item are free again
    }
}

// Dynamic LDS of the launch: the largest of a tree's tables, a fill's tables
// and the pass waves' buffers, for the largest class present.
size_t persist_lds_bytes(int nmax) {
    const int S = nmax / kWave;
    size_t b = btree_lds_bytes(nmax);
    b = b > fill_pos_lds_bytes(S, kPersistThreads) ? b : fill_pos_lds_bytes(S, kPersistThreads);
    const size_t pass = (size_t)(kPersistThreads / kWave) * 2 * kWave * 8;
    b = b > pass ? b : pass;
    return (b + 15) & ~(size_t)15;
}

template <bool WIDEST>
hipError_t run_persistent_t(const float* W, const int64_t* offsets, const int32_t* ns,
                            const BatchPlan& plan, const BatchTree& tree, const BatchBlk& blk,
                            float* M, int32_t* idx, hipStream_t s) {
    int nmax = 64;
    for (int c = 0; c < kBatchClasses; ++c)
        if (plan.class_count[c]) nmax = kClassMaxN[c];
    if (nmax > kPersistMaxN || plan.persist_items < 1) return hipErrorInvalidValue;
    uint32_t* status = device_status_word();
    if (!status) return hipErrorUnknown;
    const size_t lds = persist_lds_bytes(nmax);
    auto kern = batch_persistent_kernel<WIDEST>;
    hipError_t e;
    if (lds > 64 * 1024 &&
        (e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds)) != hipSuccess)
        return e;
    int dev = 0, cus = 0, per_cu = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess ||
        (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)kern,
                                                          kPersistThreads, lds)) != hipSuccess)
        return e;
    const int blocks = std::max(1, std::min(plan.persist_items, std::max(1, per_cu) * cus));
    const int nctr = 2 + 2 * plan.num_graphs;
    APPD_LAUNCH("persist_reset_kernel", s,
                persist_reset_kernel<<<(nctr + 255) / 256, 256, 0, s>>>(plan.ctr, nctr));
    APPD_LAUNCH("batch_persistent_kernel", s,
                kern<<<blocks, kPersistThreads, lds, s>>>(
                    W, offsets, ns, plan.perm, plan.noff, plan.rstart, plan.rgraph, plan.lists,
                    tree, blk, plan.tstats, M, idx, plan.items, plan.persist_items, plan.ctr,
                    plan.num_graphs, plan.total_n, status));
    return hipGetLastError();
}

}  // namespace

hipError_t run_persistent(const float* W, const int64_t* offsets, const int32_t* ns,
                          const BatchPlan& plan, const BatchTree& tree, const BatchBlk& blk,
                          int mode, float* M, int32_t* idx, hipStream_t s) {
    return mode == 1 ? run_persistent_t<true>(W, offsets, ns, plan, tree, blk, M, idx, s)
                     : run_persistent_t<false>(W, offsets, ns, plan, tree, blk, M, idx, s);
}

// This unit's copy of the write-count switch (appd_wcount.h).
hipError_t set_write_count_persist(const WriteCount& wc, hipStream_t s) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_write_count), &wc, sizeof wc, 0,
                                  hipMemcpyHostToDevice, s);
}

}  // namespace appd
