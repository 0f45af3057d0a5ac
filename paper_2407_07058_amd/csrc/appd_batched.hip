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
#include "appd_fillpos.h"
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
    __shared__ uint16_t s_R[NWV][CB];  // slot part of each column's code
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
    uint16_t* row_buf = s_R[threadIdx.x / kWave];
    if (vec)
        fill_rows_block_coded<CB, WIDEST, true, true>(tree.pos + o, tree.ek + o, n, j0, cnt, r0, r1, s_sp,
                                                s_slot, blk.code + o + j0, s_sorted, s_dM, s_dI,
                                                row_buf, Mg, Ig, NWV);
    else
        fill_rows_block_coded<CB, WIDEST, false, true>(tree.pos + o, tree.ek + o, n, j0, cnt, r0, r1,
                                                 s_sp, s_slot, blk.code + o + j0, s_sorted, s_dM,
                                                 s_dI, row_buf, Mg, Ig, NWV);
}

// One work item: `rows` rows of one graph of the class (the chunk tables give
// the graph and the item's first row).
template <int S, bool WIDEST>
__global__ __launch_bounds__(kBatchFillThreads) void fill_pos_kernel(
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ perm, const int64_t* __restrict__ noff,
    const int32_t* __restrict__ chunk_start, int first, int count, int chunk_base, int rows,
    BatchTree tree, BatchBlk blk, float* __restrict__ M, int32_t* __restrict__ idx) {
    __shared__ __align__(16) char s_lds[fill_pos_lds_bytes(S, kBatchFillThreads)];
    const int b = chunk_base + (int)blockIdx.x;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_start[first + mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    const int gi = first + lo;
    const int n = ns[perm[gi]];
    const int chunk = b - chunk_start[gi];
    if (chunk < 0 || (int64_t)chunk * rows >= n || n > kWave * S) return;
    fill_pos_rows<S, kBatchFillThreads, WIDEST>(offsets, ns, perm, noff, gi, chunk * rows,
                                                min(n, chunk * rows + rows), tree, blk, M, idx,
                                                s_lds);
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
        for (int k = 1; k < nstreams; ++k) st[k] = ss->side[k - 1];
    }
    // Staggered: the fork is recorded after the largest class's candidate-list
    // pass, which then streams its W with the GPU to itself, and the other
    // classes run beside that class's per-graph trees (bound by latency) and
    // its fill.  Otherwise every class starts at once.
    const bool stagger = nstreams > 1 && plan.stagger && plan.split_count <= 0 &&
                         plan.class_tree[cls[0]] == APPD_BATCH_TREE_BORUVKA;
    auto fork = [&]() -> hipError_t {
        hipError_t fe;
        for (int k = 1; k < nstreams; ++k)
            if ((fe = hipStreamWaitEvent(st[k], ss->fork, 0)) != hipSuccess) return fe;
        return hipSuccess;
    };
    if (nstreams > 1 && !stagger) {
        if ((e = hipEventRecord(ss->fork, s)) != hipSuccess) return e;
        if ((e = fork()) != hipSuccess) return e;
    }
    // The largest class (the longest Prim chains and most of the entries) has
    // the caller's stream to itself; each other class, largest first, takes
    // the side stream with the least work so far, so that they finish while
    // it still runs.  Split, the largest class's
    // biggest graphs keep the caller's stream, the rest of it takes the first
    // side stream, and the other classes the side streams after it.
    const bool split = nstreams >= 2 && plan.split_count > 0;
    const int others0 = split && nstreams >= 3 ? 2 : 1;
    double load[kBatchClasses] = {};
    for (int j = 0; j < nc; ++j) {
        const int c = cls[j];
        const int first = plan.class_first[c], count = plan.class_count[c];
        const int rows = plan.class_rows[c], chunks = plan.class_chunks[c];
        // trees of graphs first .. first + cnt - 1 of class c (rows: their
        // total n, the rows of the Boruvka pass)
        auto trees = [&](int f0, int cnt, int rows_bound, hipStream_t cs) -> hipError_t {
            return plan.class_tree[c] == APPD_BATCH_TREE_BORUVKA
                       ? launch_btree(c, f0, cnt, rows_bound, WIDEST ? 1 : 0, W, offsets, ns, plan,
                                      tree, blk, plan.lists, cs,
                                      stagger && j == 0 ? ss->fork : nullptr)
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
        hipStream_t cs = st[0];
        if (j > 0 && nstreams > 1) {
            // the side stream with the least work so far (work of a class:
            // its vertices times its largest n, about its n^2 entries), so
            // that small classes pile up behind each other rather than behind
            // a large one
            int best = others0;
            for (int k = others0 + 1; k < nstreams; ++k)
                if (load[k] < load[best]) best = k;
            load[best] += (double)plan.class_vertices[c] * (double)kClassMaxN[c];
            cs = st[best];
        }
        e = trees(first, count, plan.class_vertices[c], cs);
        if (e != hipSuccess) return e;
        if (stagger && j == 0 && (e = fork()) != hipSuccess) return e;
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
    if (plan.persistent) return run_persistent(W, offsets, ns, plan, tree, blk, mode, M, idx, s);
    return mode == 1 ? run_batched_t<true>(W, offsets, ns, plan, tree, blk, M, idx, s)
                     : run_batched_t<false>(W, offsets, ns, plan, tree, blk, M, idx, s);
}

// This unit's copy of the write-count switch (appd_wcount.h).
hipError_t set_write_count_batched(const WriteCount& wc, hipStream_t s) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_write_count), &wc, sizeof wc, 0,
                                  hipMemcpyHostToDevice, s);
}

}  // namespace appd
