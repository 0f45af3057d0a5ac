// Spanning tree and Prim order of many small graphs (n <= 2048) without
// Prim's sequential chain.
//
// Prim's algorithm (Section 3) takes n - 1 dependent steps per graph, each
// waiting for a row of W; for a batch that chain, not bandwidth, sets the time.
// Under the edge total order the minimum spanning tree is unique and Prim's
// attachment order from vertex 0 is a function of that tree alone (the
// single-graph Boruvka path in appd_tree.hip relies on the same two facts), so
// here, per size class:
//
//  1. btree_pass_kernel: one wave per row of every graph of the class keeps
//     the row's K smallest entries (row_topk_rank_vals, appd_topk.h) as that
//     vertex's candidate list: one pass over the class's W.
//  2. btree_finish_kernel: one workgroup per graph.  Boruvka rounds on the
//     lists, all state in LDS: a vertex's first list entry outside its
//     component is its exact cheapest outgoing edge; a vertex whose list is
//     used up bounds its outgoing edges from below by its last entry, and a
//     component hooks along its best candidate only when that beats every
//     bound of the component (cut property).  After a round in which no
//     component can decide, the workgroup itself refreshes the lists of the
//     smallest component's vertices (their entries outside it), which then
//     decides; after kBtRefreshes refreshes the workgroup runs Prim's
//     algorithm instead (same outputs).  Each hooking component is re-rooted at its endpoint, so the
//     merged forest stays rooted; at the end it is re-rooted at vertex 0.
//     Then Prim's order: with link(v) the nearest ancestor whose edge is larger
//     than v's own (or vertex 0), Prim takes every vertex hanging below a
//     through edges smaller than e(a) before crossing a larger edge, cheapest
//     first, so the order is the preorder of the link tree with children by
//     increasing edge key: pos(v) = pos(link(v)) + 1 + the link-subtree sizes
//     of v's siblings with smaller keys.
//
// Outputs per graph (at its noff offset): order, ek (attachment keys in Prim
// order), pos and parent -- what the sequential kernel writes.
#include "appd_btree.h"

namespace appd {

constexpr int kBtPassThreads = 256;  // 4 waves, one row each

// One wave per row of the class.
template <bool WIDEST, int E>
__global__ __launch_bounds__(kBtPassThreads) void btree_pass_kernel(
    const float* __restrict__ W, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ ns, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ noff, const int32_t* __restrict__ rstart,
    const int32_t* __restrict__ rgraph, int first, int count, uint64_t* __restrict__ lists) {
    __shared__ uint64_t s_buf[kBtPassThreads / kWave][2 * kWave];
    const int wid = __builtin_amdgcn_readfirstlane((int)threadIdx.x / kWave);
    const int r = rstart[first] + (int)blockIdx.x * (kBtPassThreads / kWave) + wid;
    const int rend = rstart[first + count - 1] + ns[perm[first + count - 1]];
    if (r >= rend) return;  // whole wave (r is wave-uniform); no barrier in this kernel
    bt_pass_row<WIDEST, E>(W, offsets, ns, perm, noff, rstart, rgraph, r, lists, s_buf[wid]);
}

// One workgroup per graph of the class.
template <int NT, int CH, bool WIDEST>
__global__ __launch_bounds__(NT) void btree_finish_kernel(
    const float* __restrict__ Wall, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ ns, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ noff, int first, int nmax, uint64_t* __restrict__ lists_all,
    BatchTree tree, int32_t* __restrict__ tstats, BatchBlk blk) {
    extern __shared__ uint64_t s_dyn[];
    __shared__ uint64_t s_aux[(bt_aux_bytes<NT>() + 7) / 8];
    const BtAux aux = bt_aux_carve<NT>((char*)s_aux);
    bt_finish_graph<NT, CH, WIDEST>(Wall, offsets, ns, perm, noff, first + (int)blockIdx.x, nmax,
                                    lists_all, tree, tstats, blk, s_dyn, aux);
}

template <bool WIDEST>
hipError_t launch_btree_t(int c, int first, int count, int rows_in_class, const float* W,
                          const int64_t* offsets, const int32_t* ns, const BatchPlan& plan,
                          const BatchTree& tree, const BatchBlk& blk, uint64_t* lists,
                          hipStream_t s, hipEvent_t after_pass) {
    if (count <= 0) return hipSuccess;
    const int nmax = kClassMaxN[c];
    const int blocks = (rows_in_class + kBtPassThreads / kWave - 1) / (kBtPassThreads / kWave);
    // columns per lane: one block of 64 * E columns covers the class's rows
#define APPD_BT_PASS(EE)                                                                    \
    APPD_LAUNCH("btree_pass_kernel", s,                                                     \
                btree_pass_kernel<WIDEST, EE><<<blocks, kBtPassThreads, 0, s>>>(            \
                    W, offsets, ns, plan.perm, plan.noff, plan.rstart, plan.rgraph, first, count,  \
                    lists))
    if (blocks > 0) {
        if (nmax <= 256) APPD_BT_PASS(4);
        else if (nmax <= 512) APPD_BT_PASS(8);
        else if (nmax <= 1024) APPD_BT_PASS(16);
        else APPD_BT_PASS(32);
    }
#undef APPD_BT_PASS
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // the point other streams may wait for: the class's lists are written
    if (after_pass && (e = hipEventRecord(after_pass, s)) != hipSuccess) return e;
    const size_t lds = btree_lds_bytes(nmax);
    // workgroup size: 256 threads, 1024 for the largest class (few graphs of
    // up to 2048 vertices: the per-graph latency is the launch's time)
#define APPD_BT_FIN(NTT, NM)                                                                   \
    if (nmax == NM) {                                                                          \
        constexpr int CC = (NM + NTT - 1) / NTT;                                               \
        if (lds > 64 * 1024) {                                                                 \
            e = hipFuncSetAttribute((const void*)btree_finish_kernel<NTT, CC, WIDEST>,         \
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);     \
            if (e != hipSuccess) return e;                                                     \
        }                                                                                      \
        APPD_LAUNCH("btree_finish_kernel", s,                                                  \
                    btree_finish_kernel<NTT, CC, WIDEST><<<count, NTT, lds, s>>>(              \
                        W, offsets, ns, plan.perm, plan.noff, first, nmax, lists, tree,        \
                        plan.tstats, blk));                                                    \
        return hipGetLastError();                                                              \
    }
    APPD_BT_FIN(256, 64)
    APPD_BT_FIN(256, 128)
    APPD_BT_FIN(256, 256)
    APPD_BT_FIN(256, 512)
    APPD_BT_FIN(256, 1024)
    APPD_BT_FIN(1024, 2048)
#undef APPD_BT_FIN
    return hipErrorInvalidValue;
}

hipError_t launch_btree(int c, int first, int count, int rows_in_class, int mode, const float* W,
                        const int64_t* offsets, const int32_t* ns, const BatchPlan& plan,
                        const BatchTree& tree, const BatchBlk& blk, uint64_t* lists,
                        hipStream_t s, hipEvent_t after_pass) {
    return mode == 1 ? launch_btree_t<true>(c, first, count, rows_in_class, W, offsets, ns, plan,
                                            tree, blk, lists, s, after_pass)
                     : launch_btree_t<false>(c, first, count, rows_in_class, W, offsets, ns, plan,
                                             tree, blk, lists, s, after_pass);
}

}  // namespace appd
