// Parallel spanning tree and Prim order for one large graph.
//
// Prim's algorithm (Section 3) attaches one vertex per step, each step waiting
// for a dependent row load; for large n that chain, not bandwidth, bounds the
// time.  Under the edge total order the minimum spanning tree is unique, and
// Prim's attachment order from vertex 0 is a function of that tree alone.  So
// here the tree is found with Boruvka rounds and Prim's order is rebuilt from
// it; the outputs (order, attachment keys, positions, parents) are the ones the
// sequential Prim kernel produces.
//
// Tree.  A pass over W keeps, for every row u, its K smallest keys towards
// vertices outside u's component (sorted).  Boruvka rounds then run on these
// lists in one workgroup: a vertex's first list entry outside its component is
// its exact cheapest outgoing edge; a vertex whose list is used up only bounds
// its outgoing edges from below by its K-th entry.  A component whose best exact
// candidate is below every such bound has found its cheapest outgoing edge,
// which is a tree edge (cut property), and hooks along it.  When no component can
// decide, another pass refreshes the lists (entries inside the row's own
// component skipped), or, once at most kCmat components are left, computes the
// smallest edge key between every pair of components, from which the rounds
// finish the tree exactly.  Each hooking component is re-rooted
// at its endpoint (the parent pointers on the path to its old root are
// reversed), so the merged tree stays rooted; at the end it is re-rooted at
// vertex 0.  If the tree is not complete after kPasses passes, the sequential
// Prim kernel runs instead (same outputs).
//
// Order.  For a vertex v with tree edge e(v) to its parent, let link(v) be the
// nearest ancestor a whose own edge is larger than e(v) (or vertex 0).  Prim,
// having reached a, takes every vertex hanging below a through edges smaller
// than e(a) before crossing any larger edge, cheapest edge first; so the Prim
// order is the preorder of the tree of links, children taken by increasing edge
// key.  Positions follow from link-subtree sizes and, among siblings, the sizes
// of the siblings with smaller keys.
#include "appd_device.h"
#include "appd_internal.h"
#include "appd.h"
#include "appd_prim.h"
#include "appd_topk.h"

namespace appd {

constexpr int kPasses = 4;         // passes over W before falling back to Prim
constexpr int kPassThreads = 256;  // 4 waves, one row each
constexpr int kRoundThreads = 1024;
constexpr int kRankTile = 256;
constexpr int kMaxLdsN = 32768;    // comp + parent as 16-bit values in LDS
constexpr int kLdsBytes = 150 * 1024;  // dynamic LDS the rounds kernel may take
constexpr int kTableBytes = 28;        // per-component table entry
constexpr uint64_t kNone = ~0ull;
// A vertex's list is stored as K/4 groups of four consecutive entries, in two
// planes: the vertex ids of group g of vertex u (4 x u16) at word
// (g * n + u) * 2, their ord32 weights (4 x u32) at word K/2 * n + (g * n + u) * 4.
// A wave of the rounds kernel, whose lanes hold consecutive vertices, then
// reads 512 and 1024 contiguous bytes for one group of 64 vertices (and touches
// 12 cache lines, not the 32 of an interleaved 32-byte record).  The edge key of
// an entry is ord32 << 32 | flat(u, id).  The planes take 96 of the 128 bytes
// per vertex the workspace reserves for the lists.  A list shorter than K
// (only when n <= K: a refresh pass runs with more than K components, so every
// row then has K entries outside its own) is padded with the vertex itself,
// which every walk sees as internal.
__device__ __forceinline__ size_t grp_ids(int n, int g, int u) { return ((size_t)g * n + u) * 2; }
__device__ __forceinline__ size_t grp_ords(int n, int g, int u) {
    return (size_t)(kK / 2) * n + ((size_t)g * n + u) * 4;
}

// control block (int32 words); word 32 holds the number of rank tiles
enum { C_DONE = 0, C_NCOMP, C_NEED_PASS, C_FALLBACK, C_ROUNDS, C_ORDERED, C_PASSES, C_CMAT,
       C_TABLES, C_WORDS };  // C_TABLES: component-table passes that ran
// With at most kCmat components left, a refresh pass computes the smallest
// edge key between every pair of components instead of candidate lists
// (C_CMAT = the number of components it saw); the next rounds call then
// finishes the tree from that exact kCmat x kCmat table.
constexpr int kCmat = 16;
// Up to this n a round that leaves at most kCmat components, some of which
// could not decide (their lists are running dry), hands over to the component
// table at once: its pass reads 2n^2 bytes, which costs no more than the list
// rounds it replaces.  Above it the rounds carry on while they can.
constexpr int kEarlyTableMaxN = 16384;
constexpr int C_TILES = 32;

// List entries are ord32(w) << 32 | v: within one row the flat index of (u, v)
// grows with v, so this orders a row exactly like the global edge key.
__device__ __forceinline__ uint64_t edge_key_of(uint64_t entry, uint32_t u, uint32_t n) {
    const uint32_t v = (uint32_t)entry;
    return (entry & 0xffffffff00000000ull) | (uint64_t)flat_idx(u, v, n);
}

// Values updated by device-scope atomics (performed in L2) are read past L1.
__device__ __forceinline__ uint64_t ld_l2(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_l2(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- pass
// One wave per row: the row's K smallest entries (row_topk, appd_topk.h),
// stored as the vertex's candidate list.
template <bool WIDEST, bool FILTER, bool VEC>
__device__ __forceinline__ void pass_row(const float* __restrict__ W, int n,
                                         const int32_t* __restrict__ comp,
                                         int32_t* __restrict__ lptr,
                                         uint32_t* __restrict__ groups, int u) {
    const int lane = threadIdx.x & (kWave - 1);
    const float* row = W + (size_t)u * (size_t)n;
    const uint64_t mine = row_topk<WIDEST, FILTER, VEC>(
        row, n, u, [&](int c) { return comp[c]; },
        [&](int c0) { return *(const int4*)(comp + c0); });
    if (lane < kK) {  // group lane/4, slot lane%4 (layout: see grp_ids)
        ((uint16_t*)(groups + grp_ids(n, lane >> 2, u)))[lane & 3] =
            (uint16_t)(mine == kNone ? (uint32_t)u : (uint32_t)mine);
        groups[grp_ords(n, lane >> 2, u) + (lane & 3)] = (uint32_t)(mine >> 32);
    }
    if (lane == 0) lptr[u] = 0;
}

// First pass over W (every row, no component filter).  It also sets up the
// rounds' state, which nothing reads before the first rounds call: every
// vertex its own component, empty minima, the control words.
template <bool WIDEST, bool VEC>
__global__ __launch_bounds__(kPassThreads) void tree_pass_kernel(const float* __restrict__ W,
                                                                 int n, int32_t* __restrict__ comp,
                                                                 uint64_t* __restrict__ best,
                                                                 uint64_t* __restrict__ lb,
                                                                 int32_t* __restrict__ lptr,
                                                                 uint32_t* __restrict__ groups,
                                                                 int32_t* __restrict__ ctrl) {
    const int t = threadIdx.x;
    const int i = blockIdx.x * kPassThreads + t;
    if (i < n) {
        comp[i] = i;
        best[i] = kNone;
        lb[i] = kNone;
    }
    if (blockIdx.x == 0 && t < 64)
        ctrl[t] = t == C_NCOMP ? n : (t == C_PASSES || (t == C_DONE && n == 1)) ? 1 : 0;
    const int u = blockIdx.x * (kPassThreads / kWave) + t / kWave;
    if (u >= n) return;  // no barrier in this kernel
    pass_row<WIDEST, false, VEC>(W, n, nullptr, lptr, groups, u);
}

// ---------------------------------------------------------------- component table
// Refresh pass, one launch whose mode follows the number C of components left
// (dense ids 0..C-1).  C > kCmat: the list pass again over every row, entries
// inside the row's own component skipped (a persistent grid, one row per wave
// at a time).  C <= kCmat: the component table, the smallest edge key between
// every pair of components.  By the cut property the
// spanning tree of the components under these minima is exactly the rest of
// the minimum spanning tree.
//
// A persistent grid of kCmatBlocks(n) workgroups of 16 waves, one row per wave
// at a time.  Each lane keeps, per component c, the smallest weight it has
// seen towards c and its column in a private LDS column ({s, v}; s = w, or -w
// when widest).  W is NaN-free, so a float compare orders weights exactly like
// ord32 (both take -0.0 = +0.0); the empty slot holds a NaN, which every
// weight beats, and a lane walks its columns in increasing order, so the first
// of equal weights (the smaller edge key within the row) is kept.  At the end
// of a row lane l reduces slot l & 15 over a quarter of the wave's lanes as
// full edge keys and two shuffles finish the row; the 16 row minima fold into
// the workgroup's table with LDS atomics.  Each workgroup writes its table to
// part[blockIdx]; the next rounds call combines the tables (the kernel
// boundary publishes them, so no workgroup waits on or fences for another).
constexpr int kCmatThreads = 1024;
constexpr int kCmatMaxBlocks = 256;
__host__ __device__ inline int kCmatBlocks(int n) {
    const int b = (n + kCmatThreads / kWave - 1) / (kCmatThreads / kWave);
    return b < kCmatMaxBlocks ? b : kCmatMaxBlocks;
}

__device__ __forceinline__ void cmat_fold_slot(uint2* slot, float s, uint32_t v) {
    const uint2 cur = *slot;
    if (!(s >= __uint_as_float(cur.x))) *slot = make_uint2(__float_as_uint(s), v);
}

template <bool WIDEST, bool VEC>
__global__ __launch_bounds__(kCmatThreads) void tree_refresh_kernel(
    const float* __restrict__ W, int n, const int32_t* __restrict__ comp,
    int32_t* __restrict__ lptr, uint32_t* __restrict__ groups, uint64_t* __restrict__ part,
    int32_t* __restrict__ ctrl) {
    constexpr int NW = kCmatThreads / kWave;
    __shared__ uint2 tab[NW][kCmat][kWave];
    __shared__ uint64_t pair[kCmat * kCmat];
    if (ctrl[C_DONE]) return;
    const int C = ctrl[C_NCOMP];
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    if (C > kCmat) {
        // candidate lists again, entries inside the own component skipped
        if (blockIdx.x == 0 && t == 0) atomicAdd(&ctrl[C_PASSES], 1);
        const int u0 = __builtin_amdgcn_readfirstlane(blockIdx.x * NW + wid);
        for (int u = u0; u < n; u += gridDim.x * NW)
            pass_row<WIDEST, true, VEC>(W, n, comp, lptr, groups, u);
        return;
    }
    if (blockIdx.x == 0 && t == 0) {
        atomicAdd(&ctrl[C_PASSES], 1);
        atomicAdd(&ctrl[C_TABLES], 1);
        ctrl[C_CMAT] = C;
    }
    if (t < kCmat * kCmat) pair[t] = kNone;
    uint2* col = &tab[wid][0][lane];  // slot c at col[c * kWave]
    const uint2 empty = make_uint2(0x7fc00000u, 0xffffffffu);
#pragma unroll
    for (int c = 0; c < kCmat; ++c) col[c * kWave] = empty;
    __syncthreads();
    // W is symmetric: row u offers only its columns v > u, so edge (u, v) lands
    // under the component of its smaller endpoint (the rounds take the minimum
    // of both orientations).  A wave takes rows q and n - 1 - q together, which
    // makes every wave's share n - 1 columns.
    auto row_minima = [&](int u) {
        const float* row = W + (size_t)u * (size_t)n;
        const int cu = comp[u] & (kCmat - 1);
        if (VEC) {
            // a ring of kRing 16-byte loads of W (and of comp) per lane in
            // flight; the slot just consumed is refilled kRing steps ahead
            // (clamped to the row's last 16 bytes past the end)
            constexpr int kRing = 4;
            constexpr int S = kWave * 4;  // columns per wave step
            const int base = (u + 1) & ~3;  // 16-byte aligned; columns <= u skipped
            const int c0 = base + lane * 4;
            float4 xb[kRing];
            int4 cb[kRing];
#pragma unroll
            for (int d = 0; d < kRing; ++d) {
                const int c = min(c0 + d * S, n - 4);
                xb[d] = *(const float4*)(row + c);
                cb[d] = *(const int4*)(comp + c);
            }
            for (int cc = c0; cc < n; cc += kRing * S) {
#pragma unroll
                for (int d = 0; d < kRing; ++d) {
                    const int c = cc + d * S;
                    const float4 x = xb[d];
                    const int4 c4 = cb[d];
                    const int cn = min(c + kRing * S, n - 4);
                    xb[d] = *(const float4*)(row + cn);
                    cb[d] = *(const int4*)(comp + cn);
                    if (c < n) {  // columns in increasing order, as the ties need
                        if (c > u) cmat_fold_slot(&col[(c4.x & (kCmat - 1)) * kWave], WIDEST ? -x.x : x.x, c);
                        if (c + 1 > u)
                            cmat_fold_slot(&col[(c4.y & (kCmat - 1)) * kWave], WIDEST ? -x.y : x.y, c + 1);
                        if (c + 2 > u)
                            cmat_fold_slot(&col[(c4.z & (kCmat - 1)) * kWave], WIDEST ? -x.z : x.z, c + 2);
                        cmat_fold_slot(&col[(c4.w & (kCmat - 1)) * kWave], WIDEST ? -x.w : x.w, c + 3);
                    }
                }
            }
        } else {
            for (int c = u + 1 + lane; c < n; c += kWave) {
                const float x = row[c];
                cmat_fold_slot(&col[(comp[c] & (kCmat - 1)) * kWave], WIDEST ? -x : x, c);
            }
        }
        // slot (lane & 15) over lanes 16 q .. 16 q + 15, then across the quarters
        const int c = lane & (kCmat - 1), q = lane / kCmat;
        uint64_t m = kNone;
#pragma unroll
        for (int j = 0; j < kWave / 4; ++j) {
            const uint2 e = tab[wid][c][q * (kWave / 4) + j];
            const uint64_t key = ((uint64_t)ord32(__uint_as_float(e.x)) << 32) |
                                 (uint64_t)flat_idx((uint32_t)u, e.y, (uint32_t)n);
            m = umin64(m, e.y == 0xffffffffu ? kNone : key);
        }
        m = umin64(m, shfl_xor_u64(m, 16));
        m = umin64(m, shfl_xor_u64(m, 32));
#pragma unroll
        for (int c2 = 0; c2 < kCmat; ++c2) col[c2 * kWave] = empty;
        if (lane < kCmat && m != kNone)
            atomicMin((unsigned long long*)&pair[cu * kCmat + c], (unsigned long long)m);
    };
    const int nw = gridDim.x * NW;
    const int npairs = (n + 1) / 2;
    for (int q = __builtin_amdgcn_readfirstlane(blockIdx.x * NW + wid); q < npairs; q += nw) {
        row_minima(q);
        if (n - 1 - q != q) row_minima(n - 1 - q);
    }
    __syncthreads();
    if (t < kCmat * kCmat) part[(size_t)blockIdx.x * kCmat * kCmat + t] = pair[t];
}

// ---------------------------------------------------------------- rounds
struct RoundArgs {
    const float* W;
    int n;
    int32_t* comp;  // global copy of the component labels (read by the passes)
    uint64_t* best;
    uint64_t* lb;
    int32_t* lptr;
    const uint32_t* groups;  // candidate lists (layout: see grp_ids)
    int32_t* hook;
    int32_t* hx;  // hooking endpoint inside the component
    int32_t* hy;  // endpoint outside
    int32_t* par;
    int32_t* ctrl;
    const uint64_t* cmpart;  // component-table pass: kCmatBlocks(n) tables of kCmat^2 keys
    int cm;  // capacity of the per-component LDS tables
};

// Block-wide exclusive scan (one workgroup of kRoundThreads threads): wave
// scans by shuffles, then one scan over the 16 wave totals.  s: kRoundThreads ints.
__device__ __forceinline__ int block_excl_scan(int x, int* s) {
    constexpr int NW = kRoundThreads / kWave;
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1), wid = t / kWave;
    int incl = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) s[wid] = incl;
    __syncthreads();
    if (t < kWave) {
        const int v = t < NW ? s[t] : 0;
        int w = v;
#pragma unroll
        for (int d = 1; d < NW; d <<= 1) {
            const int y = __shfl_up(w, d);
            if (t >= d) w += y;
        }
        if (t < NW) s[NW + t] = w - v;
    }
    __syncthreads();
    const int r = s[NW + wid] + incl - x;
    __syncthreads();
    return r;
}

// One workgroup.  Components are numbered densely 0..C-1 and renumbered after
// every round.  Per vertex: component and parent, as 16-bit values in LDS when
// n <= kMaxLdsN (else the global arrays).  Per component: best candidate, lower
// bound, hook target and hooking edge -- in LDS tables once C <= cm (so that
// the many vertices of a large component meet in LDS atomics, not at one L2
// address), in the global arrays before that.
template <bool LDS, bool WIDEST>
__global__ __launch_bounds__(kRoundThreads) void tree_rounds_kernel(RoundArgs a) {
    extern __shared__ uint64_t s_dyn[];
    __shared__ int s_flag[4];
    __shared__ int s_scan[kRoundThreads];
    const int n = a.n;
    const int cm = a.cm;
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    int32_t* ctrl = a.ctrl;
    if (ctrl[C_ORDERED] || ctrl[C_FALLBACK]) return;
    // control words read once; this workgroup alone updates them until it
    // ends, so they live in registers (uniform) and are written at the end
    bool done = ctrl[C_DONE] != 0;
    int rounds = ctrl[C_ROUNDS];
    bool need_pass = false;
    // LDS layout: [per-component tables: best, lb (u64) | hook, hx, hy (i32)]
    //             [per-vertex: component, parent (u16)]
    uint64_t* t_best = s_dyn;
    uint64_t* t_lb = t_best + cm;
    int32_t* t_hook = (int32_t*)(t_lb + cm);
    int32_t* t_hx = t_hook + cm;
    int32_t* t_hy = t_hx + cm;
    uint16_t* v_comp = (uint16_t*)(t_hy + cm);
    uint16_t* v_par = v_comp + n;
    constexpr uint16_t NIL = 0xffff;
    auto getc = [&](int v) -> int { return LDS ? (int)v_comp[v] : a.comp[v]; };
    auto setc = [&](int v, int c) {
        if (LDS) v_comp[v] = (uint16_t)c;
        else a.comp[v] = c;
    };
    auto getp = [&](int v) -> int {
        if (LDS) {
            const uint16_t x = v_par[v];
            return x == NIL ? -1 : (int)x;
        }
        return a.par[v];
    };
    auto setp = [&](int v, int p) {
        if (LDS) v_par[v] = p < 0 ? NIL : (uint16_t)p;
        else a.par[v] = p;
    };
    if (t == 0) s_flag[3] = 0;  // pending walks of the current round
    int C = ctrl[C_NCOMP];
    bool small = C <= cm;
    auto get_best = [&](int d) { return small ? t_best[d] : ld_l2(&a.best[d]); };
    auto get_lb = [&](int d) { return small ? t_lb[d] : ld_l2(&a.lb[d]); };
    auto min_best = [&](int d, uint64_t k) {
        if (small) atomicMin((unsigned long long*)&t_best[d], (unsigned long long)k);
        else atomicMin((unsigned long long*)&a.best[d], (unsigned long long)k);
    };
    auto min_lb = [&](int d, uint64_t k) {
        if (small) atomicMin((unsigned long long*)&t_lb[d], (unsigned long long)k);
        else atomicMin((unsigned long long*)&a.lb[d], (unsigned long long)k);
    };
    auto geth = [&](int d) { return small ? t_hook[d] : a.hook[d]; };
    auto seth = [&](int d, int h) {
        if (small) t_hook[d] = h;
        else a.hook[d] = h;
    };
    auto gethx = [&](int d) { return small ? t_hx[d] : a.hx[d]; };
    auto sethx = [&](int d, int x) {
        if (small) t_hx[d] = x;
        else a.hx[d] = x;
    };
    auto gethy = [&](int d) { return small ? t_hy[d] : a.hy[d]; };
    auto sethy = [&](int d, int y) {
        if (small) t_hy[d] = y;
        else a.hy[d] = y;
    };
    // the rooted forest built so far (first call: every vertex its own root)
    const bool first = rounds == 0;
    // after a component-table pass: c0 components, table entry (a, b) names the
    // smallest edge between them; s_cmap follows each one's current number
    __shared__ int s_cmap[kCmat];
    __shared__ uint64_t s_cm[kCmat * kCmat];
    const int c0 = first ? 0 : ctrl[C_CMAT];
    const bool dmode = c0 > 0 && c0 == C;
    if (t < kCmat) s_cmap[t] = t;
    if (dmode) {
        // combine the component-table pass's workgroup tables: thread t takes
        // entries 2p, 2p + 1 (p = t % 128) of every eighth table, one 16-byte
        // load per table, sixteen in flight at a time
        constexpr int kPairs = kCmat * kCmat / 2;
        constexpr int kQ = kRoundThreads / kPairs;
        constexpr int kInFlight = 16;
        static_assert(kRoundThreads % kPairs == 0, "whole table pairs per thread group");
        const int e = 2 * (t % kPairs), q = t / kPairs;
        const int nparts = kCmatBlocks(n);
        if (t < kCmat * kCmat) s_cm[t] = kNone;
        uint64_t m0 = kNone, m1 = kNone;
        // only entries between the c0 components are ever set (e is even, so
        // e and e + 1 share a row)
        const bool used = e / kCmat < c0 && e % kCmat < c0;
        for (int g0 = q; used && g0 < nparts; g0 += kQ * kInFlight) {
            ulonglong2 v[kInFlight];
#pragma unroll
            for (int i = 0; i < kInFlight; ++i) {
                const int g = g0 + kQ * i;  // past the end: table q again
                v[i] = *(const ulonglong2*)(a.cmpart + (size_t)(g < nparts ? g : q) * kCmat * kCmat + e);
            }
#pragma unroll
            for (int i = 0; i < kInFlight; ++i) {
                m0 = umin64(m0, v[i].x);
                m1 = umin64(m1, v[i].y);
            }
        }
        __syncthreads();
        if (used) {
            atomicMin((unsigned long long*)&s_cm[e], (unsigned long long)m0);
            atomicMin((unsigned long long*)&s_cm[e + 1], (unsigned long long)m1);
        }
        __syncthreads();
        // an edge was recorded under its smaller endpoint's component only
        uint64_t sym = kNone;
        if (t < kCmat * kCmat) sym = umin64(s_cm[t], s_cm[(t % kCmat) * kCmat + t / kCmat]);
        __syncthreads();
        if (t < kCmat * kCmat) s_cm[t] = sym;
        __syncthreads();
    }
    if (LDS && first && !done) {
        // Round 1, all in LDS.  Every vertex is its own component and its list's
        // first entry is its cheapest edge, so it hooks along it; the only
        // cycles are pairs that chose the same edge, whose smaller vertex stays
        // the root.  parent = hook target for every other vertex.
        constexpr int kV = 8;
        for (int base = 0; base < n; base += kV * kRoundThreads) {
            uint16_t e[kV];
#pragma unroll
            for (int i = 0; i < kV; ++i) {
                const int u = base + i * kRoundThreads + t;
                e[i] = u < n ? *(const uint16_t*)(a.groups + grp_ids(n, 0, u)) : 0;
            }
#pragma unroll
            for (int i = 0; i < kV; ++i) {
                const int u = base + i * kRoundThreads + t;
                if (u < n) v_par[u] = e[i];  // an empty list holds u itself
            }
        }
        __syncthreads();
        // roots: vertices hooked to themselves, and the smaller end of a pair.
        // The per-vertex loops below go kB vertices at a time, every LDS read
        // of a batch issued before the first is used (and before any store).
        constexpr int kB = 8;
        uint32_t rootbits = 0;  // bit i: vertex t + i * kRoundThreads (n <= 32 * 1024)
        for (int i0 = 0; i0 * kRoundThreads < n; i0 += kB) {
            int h[kB], hh[kB];
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int u = (i0 + j) * kRoundThreads + t;
                h[j] = u < n ? v_par[u] : 0;
            }
#pragma unroll
            for (int j = 0; j < kB; ++j) hh[j] = v_par[h[j]];
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int u = (i0 + j) * kRoundThreads + t;
                const bool r = u < n && (h[j] == u || (hh[j] == u && u < h[j]));
                rootbits |= r ? 1u << (i0 + j) : 0u;
            }
        }
        __syncthreads();
        for (int i = 0, u = t; u < n; ++i, u += kRoundThreads) {
            const bool r = (rootbits >> i) & 1u;
            v_comp[u] = r ? (uint16_t)u : v_par[u];
            if (r) v_par[u] = NIL;
        }
        __syncthreads();
        // component = root of the hook forest.  Every vertex follows its chain
        // of hook targets up to the root (which holds itself), storing each
        // step in its own entry, so that chains through it shorten for the
        // other threads.  An entry read mid-update holds an earlier or later
        // point of the same chain, so every thread reaches the same root; the
        // forest is acyclic (edge keys are distinct, mutual pairs were broken
        // above), which bounds every chain by n.
        for (int u0 = t; u0 < n; u0 += kB * kRoundThreads) {
            int c[kB];
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int u = u0 + j * kRoundThreads;
                c[j] = u < n ? v_comp[u] : 0;  // vertex 0's chain stands in past n
            }
            bool more = true;
            for (int it = 0; more && it < n; ++it) {
                int cc[kB];
#pragma unroll
                for (int j = 0; j < kB; ++j) cc[j] = v_comp[c[j]];
                more = false;
#pragma unroll
                for (int j = 0; j < kB; ++j) {
                    const int u = u0 + j * kRoundThreads;
                    if (cc[j] != c[j]) {
                        c[j] = cc[j];
                        if (u < n) v_comp[u] = (uint16_t)cc[j];
                        more = true;
                    }
                }
            }
        }
        __syncthreads();
        // dense numbers: id(root r) = number of roots below r, from a bitmap of
        // the roots (64 per word) and the exclusive prefix of its word counts
        uint64_t* bits = s_dyn;  // n/64 words, then n/64 prefix counts
        int32_t* wpre = (int32_t*)(bits + (n + kWave - 1) / kWave);
        const int nw = (n + kWave - 1) / kWave;
        for (int w = t / kWave; w < nw; w += kRoundThreads / kWave) {
            const int u = w * kWave + lane;
            const uint64_t m = __ballot(u < n && v_par[u] == NIL);
            if (lane == 0) bits[w] = m;
        }
        __syncthreads();
        // nw <= 512 < kRoundThreads: one word per thread
        const int pre = block_excl_scan(t < nw ? __popcll(bits[t]) : 0, s_scan);
        if (t < nw) wpre[t] = pre;
        if (t == nw - 1) s_flag[2] = pre + __popcll(bits[t]);
        __syncthreads();
        C = s_flag[2];
        for (int u0 = t; u0 < n; u0 += kB * kRoundThreads) {
            int r[kB], pre_w[kB];
            uint64_t bw[kB];
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int u = u0 + j * kRoundThreads;
                r[j] = u < n ? v_comp[u] : 0;
            }
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                pre_w[j] = wpre[r[j] / kWave];
                bw[j] = bits[r[j] / kWave];
            }
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int u = u0 + j * kRoundThreads;
                const uint64_t below = (1ull << (r[j] & (kWave - 1))) - 1;
                if (u < n) v_comp[u] = (uint16_t)(pre_w[j] + __popcll(bw[j] & below));
            }
        }
        __syncthreads();
        small = C <= cm;
        rounds = 1;
        done = C == 1;
        for (int d = t; d < C; d += kRoundThreads) {
            if (small) t_best[d] = t_lb[d] = kNone;
            else a.best[d] = a.lb[d] = kNone;
        }
    } else if (LDS) {
        // the forest so far into LDS, eight vertices per thread at a time
        constexpr int kB = 8;
        for (int v0 = t; v0 < n; v0 += kB * kRoundThreads) {
            int c[kB], p[kB];
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int v = v0 + j * kRoundThreads;
                c[j] = v < n ? (first ? v : a.comp[v]) : 0;
                p[j] = v < n ? (first ? -1 : a.par[v]) : 0;
            }
#pragma unroll
            for (int j = 0; j < kB; ++j) {
                const int v = v0 + j * kRoundThreads;
                if (v < n) {
                    setc(v, c[j]);
                    setp(v, p[j]);
                }
            }
        }
        if (small)
            for (int d = t; d < C; d += kRoundThreads) t_best[d] = t_lb[d] = kNone;
    } else {
        if (first)
            for (int v = t; v < n; v += kRoundThreads) a.par[v] = -1;
        if (small)
            for (int d = t; d < C; d += kRoundThreads) t_best[d] = t_lb[d] = kNone;
    }
    __syncthreads();

    // 1. cheapest outgoing candidate (or lower bound) of every vertex.  Each
    //    round a vertex reads a window of eight list entries: the group of four
    //    that holds its list pointer and the group after it (ids and weights,
    //    two independent loads each), and checks the entries from the pointer
    //    on, endpoint components from LDS.  The first entry leaving its
    //    component is its exact cheapest outgoing edge.  If every entry checked
    //    is internal, every outgoing edge of the vertex is larger than the
    //    window's last entry, which becomes a lower bound, and the pointer moves
    //    past the window (the vertex is "pending": its walk continues next
    //    round); an exhausted list bounds by its entry K-1.  A round in which no
    //    component decides but some vertex is pending is followed by another
    //    round on the same lists.  A wave whose vertices share one component
    //    sends one atomic per minimum.
    constexpr int kW = 4;  // vertices per thread
    constexpr int kStride = kW * kRoundThreads;
    constexpr int kLastGroup = kK / 4 - 1;
    // list pointers of the next batch of vertices, loaded one batch ahead (and
    // for the next round's first batch while the round's later steps run)
    int ppn[kW];
#pragma unroll
    for (int i = 0; i < kW; ++i) {
        const int u = i * kRoundThreads + t;
        ppn[i] = (!dmode && u < n) ? a.lptr[u] : kK;
    }
    for (int guard = 0; guard < 128 && !done; ++guard) {
        if (t == 0) s_flag[0] = 0;  // components that decided this round
        ++rounds;
        if (dmode) {
            // exact: every component's cheapest edge to any other one
            for (int e = t; e < c0 * c0; e += kRoundThreads) {
                const int x = e / c0, y = e % c0;
                const int cx = s_cmap[x], cy = s_cmap[y];
                const uint64_t k = s_cm[x * kCmat + y];
                if (cx != cy && k != kNone) min_best(cx, k);
            }
        }
        for (int base = 0; !dmode && base < n; base += kStride) {
            int pp[kW];
            uint2 gi[kW][2];  // ids of the window's two groups (u16 pairs)
            uint4 go[kW][2];  // their ord32 weights
#pragma unroll
            for (int i = 0; i < kW; ++i) pp[i] = ppn[i];
#pragma unroll
            for (int i = 0; i < kW; ++i) {
                const int u = base + i * kRoundThreads + t;
                // an exhausted list reads its last group (for the bound); the
                // window's second group past the end repeats the last one
                const int g0 = min(pp[i] >> 2, kLastGroup);
                const int g1 = min(g0 + 1, kLastGroup);
                gi[i][0] = gi[i][1] = make_uint2(0u, 0u);
                go[i][0] = go[i][1] = make_uint4(0u, 0u, 0u, 0u);
                if (u < n) {
                    gi[i][0] = *(const uint2*)(a.groups + grp_ids(n, g0, u));
                    go[i][0] = *(const uint4*)(a.groups + grp_ords(n, g0, u));
                    gi[i][1] = *(const uint2*)(a.groups + grp_ids(n, g1, u));
                    go[i][1] = *(const uint4*)(a.groups + grp_ords(n, g1, u));
                }
            }
            // the next batch's pointers (this round's next, or the next round's
            // first, whose stores came earlier in this round); a single batch
            // keeps its own, updated below
            const int nb = base + kStride < n ? base + kStride : 0;
            if (nb != base) {
#pragma unroll
                for (int i = 0; i < kW; ++i) {
                    const int u = nb + i * kRoundThreads + t;
                    ppn[i] = u < n ? a.lptr[u] : kK;
                }
            }
            int npend = 0;
            uint64_t key[kW];
            int cuv[kW];
            uint32_t isb = 0, pendm = 0, moved = 0;  // bit i: vertex i
#pragma unroll
            for (int i = 0; i < kW; ++i) {
                const int u = base + i * kRoundThreads + t;
                const bool act = u < n;
                const int cu = getc(act ? u : 0);
                cuv[i] = cu;
                // window entry w is list entry 4 * g0 + w; its id is half w & 1
                // of word w >> 1.  Lookups unconditional (ids are always < n),
                // combined bitwise: no branch separates the LDS reads.
                uint32_t idw[4] = {gi[i][0].x, gi[i][0].y, gi[i][1].x, gi[i][1].y};
                uint32_t ow[8] = {go[i][0].x, go[i][0].y, go[i][0].z, go[i][0].w,
                                  go[i][1].x, go[i][1].y, go[i][1].z, go[i][1].w};
                // opaque register values: the selects below must stay selects
                // (folded into an index they would put the window in scratch)
#pragma unroll
                for (int w = 0; w < 4; ++w) asm("" : "+v"(idw[w]));
#pragma unroll
                for (int w = 0; w < 8; ++w) asm("" : "+v"(ow[w]));
                uint32_t ext = 0;
#pragma unroll
                for (int w = 0; w < 8; ++w) {
                    const uint32_t id = (w & 1) ? idw[w >> 1] >> 16 : idw[w >> 1] & 0xffffu;
                    ext |= (uint32_t)(getc((int)id) != cu) << w;
                }
                const int p = pp[i];
                const int g0 = min(p >> 2, kLastGroup);
                // entries at or after the pointer and inside the list (p = K:
                // none; the bound is then the entry K-1, window entry 3)
                const uint32_t inlist = g0 == kLastGroup ? 0x0fu : 0xffu;
                const uint32_t live = (0xffu << (p - 4 * g0)) & inlist;
                const uint32_t stop = live & ext;
                const int last = g0 == kLastGroup ? 3 : 7;
                const int first = stop ? __builtin_ctz(stop) : last;
                // select entry `first` by its three bits
                const bool b0 = first & 1, b1 = first & 2, b2 = first & 4;
                const uint32_t wlo = b1 ? idw[1] : idw[0], whi = b1 ? idw[3] : idw[2];
                const uint32_t word = b2 ? whi : wlo;
                const uint32_t v = b0 ? word >> 16 : word & 0xffffu;
                const uint32_t o01 = b0 ? ow[1] : ow[0], o23 = b0 ? ow[3] : ow[2];
                const uint32_t o45 = b0 ? ow[5] : ow[4], o67 = b0 ? ow[7] : ow[6];
                const uint32_t o = b2 ? (b1 ? o67 : o45) : (b1 ? o23 : o01);
                const bool found = act && stop != 0;
                // padding (the vertex itself) bounds nothing: the list held
                // every outgoing edge of the vertex
                const bool bound = act && !stop && v != (uint32_t)u;
                const int np = stop ? 4 * g0 + first : min(4 * g0 + 8, kK);
                key[i] = (found || bound) ? (((uint64_t)o << 32) | flat_idx(u, v, n)) : kNone;
                const uint32_t bit = 1u << i;
                isb |= bound ? bit : 0u;
                moved |= (act && np != p) ? bit : 0u;
                pendm |= (act && !stop && np < kK) ? bit : 0u;
                pp[i] = np;
                if (nb == base) ppn[i] = np;
            }
#pragma unroll
            for (int i = 0; i < kW; ++i) {
                const int u = base + i * kRoundThreads + t;
                const bool act = u < n;
                const int cu = cuv[i];
                const bool isbi = (isb >> i) & 1u;
                const uint64_t kc = isbi ? kNone : key[i];
                const uint64_t kb = isbi ? key[i] : kNone;
                const bool pend = (pendm >> i) & 1u;
                if ((moved >> i) & 1u) a.lptr[u] = pp[i];
                npend += __popcll(__ballot(pend));
                const int cw = __builtin_amdgcn_readfirstlane(cu);
                const uint64_t same = __ballot(act && cu == cw);
                const uint64_t acts = __ballot(act);
                if (same == acts) {
                    if (__ballot(kc != kNone)) {
                        const uint64_t mc = wave_min_u64(kc);
                        if (lane == 0) min_best(cw, mc);
                    }
                    if (__ballot(kb != kNone)) {
                        const uint64_t mb = wave_min_u64(kb);
                        if (lane == 0) min_lb(cw, mb);
                    }
                } else if (act) {
                    if (kc != kNone) min_best(cu, kc);
                    if (kb != kNone) min_lb(cu, kb);
                }
            }
            if (lane == 0 && npend) atomicAdd(&s_flag[3], npend);
        }
        __syncthreads();
        // 2. decide: a component hooks when its best exact candidate beats every bound
        for (int d = t; d < C; d += kRoundThreads) {
            const uint64_t b = get_best(d);
            const uint64_t l = get_lb(d);
            seth(d, d);
            if (b != kNone && b < l) {
                const uint32_t f = (uint32_t)b;
                const int x0 = (int)(f / (uint32_t)n), y0 = (int)(f % (uint32_t)n);
                const bool xin = getc(x0) == d;
                const int x = xin ? x0 : y0, y = xin ? y0 : x0;
                sethx(d, x);
                sethy(d, y);
                seth(d, getc(y));
                atomicAdd(&s_flag[0], 1);
            }
        }
        __syncthreads();
        const int decided = s_flag[0];
        const int pending = s_flag[3];
        const int c_before = C;
        __syncthreads();  // every thread has read the counters
        if (t == 0) s_flag[3] = 0;  // ordered before the next round by the barriers below
        if (decided == 0) {
            // minima of this round are stale either way: clear them
            for (int d = t; d < C; d += kRoundThreads) {
                if (small) t_best[d] = t_lb[d] = kNone;
                else a.best[d] = a.lb[d] = kNone;
            }
            // lists still being walked: another round, unless the component
            // table can take over (at most kCmat components left)
            if (pending > 0 && C > kCmat) {
                __syncthreads();
                continue;
            }
            need_pass = true;
            break;
        }
        // 3. a mutual pair chose the same edge: the smaller id stays the root
        //    (points to itself; its partner then sees no mutual pair and hooks).
        //    Every other hooking component re-roots itself at its endpoint,
        //    whose parent becomes the endpoint outside.
        for (int d = t; d < C; d += kRoundThreads) {
            const int h = geth(d);
            if (h == d) continue;
            if (d < h && geth(h) == d && get_best(h) == get_best(d)) {
                seth(d, d);
                continue;
            }
            int cur = gethx(d), prev = gethy(d);
            while (cur >= 0) {  // reverse the parent pointers on hx -> old root
                const int nxt = getp(cur);
                setp(cur, prev);
                prev = cur;
                cur = nxt;
            }
        }
        __syncthreads();
        // 4. pointer jumping: every component -> the root it now belongs to
        for (int it = 0; it < 64; ++it) {
            if (t == 0) s_flag[1] = 0;
            __syncthreads();
            for (int d = t; d < C; d += kRoundThreads) {
                const int h = geth(d);
                const int hh = geth(h);
                if (hh != h) {
                    seth(d, hh);
                    s_flag[1] = 1;
                }
            }
            __syncthreads();
            const int again = s_flag[1];
            __syncthreads();  // every thread has read the flag before it is reset
            if (!again) break;
        }
        // 5. number the roots densely (hx of a root now holds its new number)
        const int per = (C + kRoundThreads - 1) / kRoundThreads;
        const int d0 = min(C, t * per), d1 = min(C, d0 + per);
        int cnt = 0;
        for (int d = d0; d < d1; ++d) cnt += geth(d) == d ? 1 : 0;
        int id = block_excl_scan(cnt, s_scan);
        for (int d = d0; d < d1; ++d)
            if (geth(d) == d) sethx(d, id++);
        if (t == kRoundThreads - 1) s_flag[2] = id;
        __syncthreads();
        const int Cn = s_flag[2];
        // 6. every component's new number (the number of its root), kept in
        //    its hook slot, so that relabelling a vertex takes one lookup
        constexpr int kRB = 8;  // entries per batch: every read of a step in flight
        for (int d0 = t; d0 < C; d0 += kRB * kRoundThreads) {
            int h[kRB];
#pragma unroll
            for (int j = 0; j < kRB; ++j) {
                const int d = d0 + j * kRoundThreads;
                h[j] = d < C ? geth(d) : 0;
            }
#pragma unroll
            for (int j = 0; j < kRB; ++j) h[j] = gethx(h[j]);
#pragma unroll
            for (int j = 0; j < kRB; ++j) {
                const int d = d0 + j * kRoundThreads;
                if (d < C) seth(d, h[j]);
            }
        }
        __syncthreads();
        //    relabel every vertex; clear the tables for the next round
        for (int u0 = t; u0 < n; u0 += kW * kRoundThreads) {
            int c[kW];
#pragma unroll
            for (int j = 0; j < kW; ++j) {
                const int u = u0 + j * kRoundThreads;
                c[j] = u < n ? getc(u) : 0;
            }
#pragma unroll
            for (int j = 0; j < kW; ++j) c[j] = geth(c[j]);
#pragma unroll
            for (int j = 0; j < kW; ++j) {
                const int u = u0 + j * kRoundThreads;
                if (u < n) setc(u, c[j]);
            }
        }
        const int cmap_new = (dmode && t < c0) ? geth(s_cmap[t]) : 0;
        __syncthreads();
        if (dmode && t < c0) s_cmap[t] = cmap_new;
        C = Cn;
        small = C <= cm;
        for (int d = t; d < C; d += kRoundThreads) {
            if (small) t_best[d] = t_lb[d] = kNone;
            else a.best[d] = a.lb[d] = kNone;
        }
        done = C == 1;
        __syncthreads();
        if (C == 1) break;
        if (!dmode && C <= kCmat && decided < c_before && n <= kEarlyTableMaxN) {
            need_pass = true;
            break;
        }
    }
    __syncthreads();
    if (t == 0) {
        ctrl[C_ROUNDS] = rounds;
        ctrl[C_NCOMP] = C;
        if (done) ctrl[C_DONE] = 1;
        if (need_pass) ctrl[C_NEED_PASS] = 1;
        if (dmode) ctrl[C_CMAT] = 0;  // the table is used up
    }
    if (done && t == 0) {  // re-root at vertex 0
        int cur = 0, prev = -1;
        while (cur >= 0) {
            const int nxt = getp(cur);
            setp(cur, prev);
            prev = cur;
            cur = nxt;
        }
    }
    __syncthreads();
    if (LDS) {
        for (int v = t; v < n; v += kRoundThreads) {
            a.comp[v] = getc(v);
            a.par[v] = getp(v);
        }
    }
    if (!done) return;
    if (t == 0) ctrl[C_ORDERED] = 1;  // tree complete and rooted at 0
}

// ---------------------------------------------------------------- order
// Every kernel below returns at once unless the rounds completed the tree
// (else the sequential fallback produced the outputs).  One thread per vertex
// wherever the work is independent, so each dependent chain is paid once.

// Workgroups are dispatched to the eight XCDs in turn and each XCD has its own
// L2.  A kernel launched kXcds times wider, in which only every kXcds-th
// workgroup works, keeps all its work on one XCD: a line that many threads'
// pointer chains share is then fetched into one L2 once and hit there, not
// missed once per XCD.  Only the speed depends on the dispatch order.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_block() {
    return blockIdx.x % kXcds ? -1 : (int)(blockIdx.x / kXcds);
}

// Edge key to the parent, link initialised to the parent.
template <bool WIDEST>
__device__ __forceinline__ void keyup_vertex(const float* __restrict__ W, int n, const int32_t* par,
                                             uint64_t* keyup, int32_t* link, int32_t* size,
                                             int32_t* gcount, int32_t* arrived, uint64_t* sa,
                                             int v) {
    const int p = par[v];
    uint64_t k = 0;
    if (p >= 0) k = make_key((WIDEST ? -1.0f : 1.0f) * W[(size_t)v * n + p], flat_idx(v, p, n));
    keyup[v] = k;
    link[v] = p;
    size[v] = 1;
    gcount[v] = 0;
    arrived[v] = 0;
    if (sa) sa[v] = 1ull << 32;  // packed (size, arrivals): size 1, none arrived
}

template <bool WIDEST>
__global__ __launch_bounds__(256) void tree_keyup_kernel(const float* __restrict__ W, int n,
                                                        const int32_t* par, uint64_t* keyup,
                                                        int32_t* link, int32_t* size,
                                                        int32_t* gcount, int32_t* arrived,
                                                        uint64_t* sa, const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    keyup_vertex<WIDEST>(W, n, par, keyup, link, size, gcount, arrived, sa, v);
}

// arr[target] += 1 for every active lane.  Lanes aiming at vertex 0 (the
// largest sibling group by far) and lanes sharing the first remaining lane's
// target are folded into one atomic each.
__device__ __forceinline__ void add_folded(int32_t* arr, int target) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint64_t m0 = __ballot(target == 0);
    if (m0 && lane == (int)(__ffsll((unsigned long long)m0) - 1)) atomicAdd(&arr[0], __popcll(m0));
    if (target == 0) return;
    const int lead = __builtin_amdgcn_readfirstlane(target);
    const uint64_t m = __ballot(target == lead);
    if (target == lead) {
        if (lane == (int)(__ffsll((unsigned long long)m) - 1)) atomicAdd(&arr[lead], __popcll(m));
    } else {
        atomicAdd(&arr[target], 1);
    }
}

// link(v): jump over ancestors whose edge is smaller than e(v).  Any value a
// link[] entry holds at any time is an ancestor reached over smaller edges
// only, so a thread may follow entries other threads are still updating, and
// it publishes its own progress as it goes.  Every jump moves up the tree, so
// each thread ends.  The chains share the upper part of the tree, so the
// kernel runs on one XCD (xcd_block; n = 8192: 20 -> 13 us).
__global__ __launch_bounds__(256) void tree_link_kernel(int n, const uint64_t* keyup,
                                                       int32_t* link, int32_t* gcount,
                                                       const int32_t* ctrl) {
    const int bid = xcd_block();
    if (bid < 0 || !ctrl[C_ORDERED]) return;
    const int v = bid * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    const uint64_t kv = keyup[v];
    int c = link[v];
    while (c > 0 && keyup[c] < kv) {
        c = link[c];
        link[v] = c;
    }
    add_folded(gcount, c);  // sibling-group sizes
}

// Link-subtree sizes, bottom-up: a thread starts at every leaf of the link
// tree and adds its subtree size to its link parent; the child that arrives
// last at a vertex (its arrival completes the count) carries that vertex's
// now final size further up.  Every add is released by the arrival that
// follows it and acquired by the last arrival, so the size it reads is final.
// The root's size (n) is never needed.
__global__ __launch_bounds__(256) void tree_sizes_kernel(int n, const int32_t* link,
                                                        int32_t* size, const int32_t* gcount,
                                                        int32_t* arrived, const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n || gcount[v] != 0) return;
    int x = v, sx = 1;
    for (int guard = 0; guard < n; ++guard) {
        const int p = link[x];
        if (p <= 0) break;
        __hip_atomic_fetch_add(&size[p], sx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int old =
            __hip_atomic_fetch_add(&arrived[p], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old + 1 != gcount[p]) break;
        sx = __hip_atomic_load(&size[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = p;
    }
}

// Exclusive scans over the n vertices in two grid launches: each block of
// kScanThreads threads owns kScanBlock consecutive elements (8 per thread);
// the first launch writes the block totals, the second adds the totals of the
// blocks before it and scans its own elements.
constexpr int kScanThreads = 256;
constexpr int kScanBlock = 8 * kScanThreads;

// Exclusive scan over the 256 threads of a block; *total gets the sum.
__device__ __forceinline__ int block256_excl_scan(int x, int* s, int* total) {
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    int incl = x;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) s[wid] = incl;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        const int v = s[w];
        before += w < wid ? v : 0;
        all += v;
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

// Link-subtree sizes and the scans over the group sizes in one launch: blocks
// [0, nsb) scan, blocks [nsb, nsb + nb) run tree_sizes_kernel's walk on packed
// words sa[x] = size << 32 | arrivals: one atomic per step adds a child's size
// and its arrival, and the child that completes the count reads x's final size
// from the value it returns.  A scan
// block of kScanThreads threads owns kScanBlock consecutive vertices (8 per
// thread) and sums the group sizes and rank-tile counts of all vertices before
// it itself (no other block is waited for).  It writes group starts, cleared
// fill counters and rank-tile starts; the last one records the number
// of rank tiles.
__global__ __launch_bounds__(kScanThreads) void tree_sizes_scan_kernel(
    int n, int nsb, const int32_t* link, uint64_t* sa, const int32_t* gcount, int32_t* gstart,
    int32_t* gfill, int32_t* tstart, int32_t* ctrl) {
    __shared__ int s_a[8], s_b[8];
    if (!ctrl[C_ORDERED]) return;
    if ((int)blockIdx.x >= nsb) {
        const int v = ((int)blockIdx.x - nsb) * kScanThreads + threadIdx.x;
        if (v == 0 || v >= n || gcount[v] != 0) return;
        int x = v;
        uint32_t sx = 1;
        for (int guard = 0; guard < n; ++guard) {
            const int p = link[x];
            if (p <= 0) break;
            const uint64_t old = __hip_atomic_fetch_add(&sa[p], ((uint64_t)sx << 32) | 1ull,
                                                        __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if ((int)(uint32_t)old + 1 != gcount[p]) break;
            sx += (uint32_t)(old >> 32);
            x = p;
        }
        return;
    }
    const int blk0 = blockIdx.x * kScanBlock;  // a multiple of 4 * kScanThreads
    int pre = 0, tpre = 0;
    auto count = [&](int m) {
        const int nt = (m + kRankTile - 1) / kRankTile;
        pre += m;
        tpre += m > 1 ? nt * nt : 0;
    };
#pragma unroll 4
    for (int i = 4 * threadIdx.x; i < blk0; i += 4 * kScanThreads) {  // 16-byte loads
        const int4 m = *(const int4*)(gcount + i);
        count(m.x);
        count(m.y);
        count(m.z);
        count(m.w);
    }
    int run, trun;
    (void)block256_excl_scan(pre, s_a, &run);
    (void)block256_excl_scan(tpre, s_b, &trun);
    const int b0 = blk0 + threadIdx.x * 8;
    int m[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) m[j] = b0 + j < n ? gcount[b0 + j] : 0;
    int s = 0, ts = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int nt = (m[j] + kRankTile - 1) / kRankTile;
        s += m[j];
        ts += m[j] > 1 ? nt * nt : 0;
    }
    int ta, tb;
    int r = run + block256_excl_scan(s, s_a, &ta);
    int tr = trun + block256_excl_scan(ts, s_b, &tb);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (b0 + j < n) {
            const int nt = (m[j] + kRankTile - 1) / kRankTile;
            gstart[b0 + j] = r;
            gfill[b0 + j] = 0;
            tstart[b0 + j] = tr;
            r += m[j];
            tr += m[j] > 1 ? nt * nt : 0;
        }
    }
    if (blockIdx.x == nsb - 1 && threadIdx.x == 0) ctrl[C_TILES] = trun + tb;
}

constexpr int kGroupThreads = 1024;

__global__ __launch_bounds__(kGroupThreads) void tree_group_kernel(int n, const int32_t* link,
                                                                  const int32_t* gstart,
                                                                  int32_t* gfill, int32_t* grouped,
                                                                  int32_t* rank,
                                                                  const int32_t* ctrl) {
    constexpr int NW = kGroupThreads / kWave;
    __shared__ int s_w0[NW];
    __shared__ int s_base0;
    if (!ctrl[C_ORDERED]) return;
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    const int v = blockIdx.x * kGroupThreads + t;
    const bool act = v > 0 && v < n;
    const int g = act ? link[v] : -1;
    // vertex 0's group (by far the largest): one atomic per workgroup
    const uint64_t m0 = __ballot(g == 0);
    if (lane == 0) s_w0[wid] = __popcll(m0);
    __syncthreads();
    if (t == 0) {
        int tot = 0;
        for (int w = 0; w < NW; ++w) tot += s_w0[w];
        s_base0 = tot ? atomicAdd(&gfill[0], tot) : 0;
    }
    __syncthreads();
    if (!act) return;
    rank[v] = 0;
    int slot;
    if (g == 0) {
        int before = s_base0;
        for (int w = 0; w < wid; ++w) before += s_w0[w];
        slot = before + __popcll(m0 & ((1ull << lane) - 1));
    } else {
        // lanes of the first other lane's group take consecutive slots from one atomic
        const uint64_t rest = __ballot(g != 0);
        const int first = __ffsll((unsigned long long)rest) - 1;
        const int lead = __builtin_amdgcn_readlane(g, first);
        const uint64_t ml = __ballot(g == lead);
        int bl = 0;
        if (lane == first) bl = atomicAdd(&gfill[lead], __popcll(ml));
        bl = __builtin_amdgcn_readlane(bl, first);
        slot = g == lead ? bl + __popcll(ml & ((1ull << lane) - 1)) : atomicAdd(&gfill[g], 1);
    }
    grouped[gstart[g] + slot] = v;
}

// Rank among siblings: tile (group, v-block, member-block) counts the members
// of the member block with a smaller key than each v of the v block.
__global__ __launch_bounds__(kRankTile) void tree_rank_kernel(int n, const int32_t* gcount,
                                                             const int32_t* gstart,
                                                             const int32_t* tstart,
                                                             const int32_t* grouped,
                                                             const uint64_t* keyup, int32_t* rank,
                                                             const int32_t* ctrl) {
    __shared__ uint64_t s_key[kRankTile];
    if (!ctrl[C_ORDERED]) return;
    const int total = ctrl[C_TILES];
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        int lo = 0, hi = n - 1;  // the group owning the tile: last g with tstart[g] <= tile
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tstart[mid] <= tile) lo = mid;
            else hi = mid - 1;
        }
        const int g = lo;
        const int m = gcount[g];
        const int nt = (m + kRankTile - 1) / kRankTile;
        const int local = tile - tstart[g];
        const int vb = local / nt, mb = local % nt;
        const int* mem = grouped + gstart[g];
        const int mi = mb * kRankTile + threadIdx.x;
        __syncthreads();
        s_key[threadIdx.x] = mi < m ? keyup[mem[mi]] : kNone;
        __syncthreads();
        const int vi = vb * kRankTile + threadIdx.x;
        if (vi < m) {
            const uint64_t kv = keyup[mem[vi]];
            int cnt = 0;
            const int lim = min(kRankTile, m - mb * kRankTile);
            for (int j = 0; j < lim; ++j) cnt += s_key[j] < kv ? 1 : 0;
            if (cnt) atomicAdd(&rank[mem[vi]], cnt);
        }
    }
}

// Each vertex's link-subtree size at (group start + rank): siblings in key order.
__global__ __launch_bounds__(256) void tree_place_kernel(int n, const int32_t* link,
                                                        const int32_t* gstart,
                                                        const int32_t* rank, const uint64_t* sa,
                                                        int32_t* sorted_size, int32_t* sorted_grp,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    const int g = link[v];
    const int slot = gstart[g] + rank[v];
    sorted_size[slot] = (int32_t)(sa[v] >> 32);
    sorted_grp[slot] = g;
}

// Segmented exclusive scan of the placed sizes (segments = sibling groups)
// -> total size of the smaller siblings of each slot, over the n-1 slots, one
// launch: a block of kScanThreads threads owns kScanBlock consecutive slots;
// its incoming carry is the sum of the sizes from the start of the group that
// holds the slot before the block up to the block (read directly).
__device__ __forceinline__ bool seg_head(const int32_t* grp, int i) {
    return i == 0 || grp[i] != grp[i - 1];
}

__global__ __launch_bounds__(kScanThreads) void tree_segscan_kernel(
    int n, const int32_t* sorted_size, const int32_t* sorted_grp, const int32_t* gstart,
    int32_t* sorted_pre, const int32_t* ctrl) {
    __shared__ int s_v[kScanThreads], s_h[kScanThreads], s_a[8];
    if (!ctrl[C_ORDERED]) return;
    const int m = n - 1;
    const int t = threadIdx.x;
    const int blk0 = blockIdx.x * kScanBlock;
    int carry = 0;
    {
        int part = 0;
        if (blk0 > 0 && blk0 <= m) {
            const int st = gstart[sorted_grp[blk0 - 1]];
            for (int i = st + t; i < blk0; i += kScanThreads) part += sorted_size[i];
        }
        (void)block256_excl_scan(part, s_a, &carry);
    }
    const int b0 = blk0 + t * 8;
    int sz[8];
    bool hd[8];
    int tot = 0, head = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = b0 + j;
        sz[j] = i < m ? sorted_size[i] : 0;
        hd[j] = i < m && seg_head(sorted_grp, i);
        if (hd[j]) {
            tot = 0;
            head = 1;
        }
        tot += sz[j];
    }
    s_v[t] = tot;
    s_h[t] = head;
    __syncthreads();
    // inclusive segmented scan: (v, h) + (v', h') = (h' ? v' : v + v', h | h')
    for (int d = 1; d < kScanThreads; d <<= 1) {
        int pv = 0, ph = 0;
        if (t >= d) {
            pv = s_v[t - d];
            ph = s_h[t - d];
        }
        __syncthreads();
        if (t >= d && !s_h[t]) {
            s_v[t] += pv;
            s_h[t] |= ph;
        }
        __syncthreads();
    }
    int run = t == 0 ? carry : (s_h[t - 1] ? s_v[t - 1] : carry + s_v[t - 1]);
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int i = b0 + j;
        if (i < m) {
            if (hd[j]) run = 0;
            sorted_pre[i] = run;
            run += sz[j];
        }
    }
}

// pos(v) = sum over v and its link ancestors x (below the root) of
// 1 + (sizes of x's smaller siblings).
__global__ __launch_bounds__(256) void tree_pos_kernel(int n, const int32_t* link,
                                                      const int32_t* gstart, const int32_t* rank,
                                                      const int32_t* sorted_pre,
                                                      const uint64_t* keyup, const int32_t* par,
                                                      PrimOut out, const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (v == 0) {
        out.pos[0] = 0;
        out.order[0] = 0;
        out.ek[0] = 0;
        out.parent[0] = -1;
        return;
    }
    int p = 0;
    for (int x = v; x > 0; x = link[x]) p += 1 + sorted_pre[gstart[link[x]] + rank[x]];
    out.pos[v] = p;
    out.order[p] = v;
    out.ek[p] = keyup[v];
    out.parent[v] = par[v];
}

// The two ends of the rounds in one launch (they exclude each other): block 0
// runs sequential Prim (the fallback) if the rounds did not finish the tree,
// blocks 1.. compute the parent-edge keys of the order phase if they did.
template <int CH, bool WIDEST>
__global__ __launch_bounds__(1024) void tree_finish_kernel(const float* __restrict__ W, int n,
                                                          PrimOut out, const int32_t* par,
                                                          uint64_t* keyup, int32_t* link,
                                                          int32_t* size, int32_t* gcount,
                                                          int32_t* arrived, uint64_t* sa,
                                                          int32_t* ctrl) {
    __shared__ uint64_t red_key[2 * 16];
    __shared__ int32_t red_v[2 * 16];
    extern __shared__ uint16_t s_parents[];  // prim_parents_in_lds<CH>(): 1024 * CH
    if (blockIdx.x == 0) {
        if (ctrl[C_DONE]) return;
        if (threadIdx.x == 0) ctrl[C_FALLBACK] = 1;
        prim_run<1024, CH, WIDEST>(W, n, out, red_key, red_v, s_parents);
        return;
    }
    if (!ctrl[C_ORDERED]) return;
    const int v = (blockIdx.x - 1) * 1024 + threadIdx.x;
    if (v < n) keyup_vertex<WIDEST>(W, n, par, keyup, link, size, gcount, arrived, sa, v);
}

// ---------------------------------------------------------------- host side
struct TreeWs {
    uint64_t* lists;  // candidate-list groups (128 bytes per vertex)
    int32_t *comp, *lptr, *hook, *hx, *hy, *par, *link, *size, *gcount, *gstart, *gfill;
    int32_t *tstart, *grouped, *rank, *sorted_size, *sorted_grp, *sorted_pre;
    uint64_t *best, *lb, *keyup;
    uint64_t* cmpart;
    int32_t* ctrl;
    size_t bytes;
};

// Order-phase arrays reuse the list storage (the lists are dead by then):
// six int arrays of n fit in the 8 * K * n bytes.
static TreeWs carve_tree(void* ws, int n) {
    const uintptr_t b = (uintptr_t)ws;  // null when only the size is wanted
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = (char*)(b + off);
        off = align_up(off + bytes);
        return p;
    };
    TreeWs w;
    w.lists = (uint64_t*)take(8 * (size_t)n * kK);
    int32_t** ints[11] = {&w.comp, &w.lptr, &w.hook, &w.hx, &w.hy, &w.par,
                          &w.link, &w.size, &w.gcount, &w.gstart, &w.gfill};
    for (int i = 0; i < 11; ++i) *ints[i] = (int32_t*)take(4 * (size_t)n);
    uint64_t** longs[3] = {&w.best, &w.lb, &w.keyup};
    for (int i = 0; i < 3; ++i) *longs[i] = (uint64_t*)take(8 * (size_t)n);
    w.ctrl = (int32_t*)take(4 * 64);
    w.cmpart = (uint64_t*)take(8 * (size_t)kCmat * kCmat * kCmatBlocks(n));
    w.bytes = off;
    const uintptr_t r = (uintptr_t)w.lists;
    w.tstart = (int32_t*)r;
    w.grouped = (int32_t*)(r + 4 * (size_t)n);
    w.rank = (int32_t*)(r + 8 * (size_t)n);
    w.sorted_size = (int32_t*)(r + 12 * (size_t)n);
    w.sorted_grp = (int32_t*)(r + 16 * (size_t)n);
    w.sorted_pre = (int32_t*)(r + 20 * (size_t)n);
    return w;
}

size_t tree_workspace_bytes(int n) { return carve_tree(nullptr, n).bytes; }

template <bool WIDEST>
static hipError_t launch_finish(const float* W, int n, PrimOut out, const TreeWs& w,
                                hipStream_t s) {
    const int ch = (n + 1023) / 1024;
    const int blocks = 1 + (n + 1023) / 1024;
#define APPD_FIN(C)                                                                        \
    if (ch <= C) {                                                                         \
        const size_t lds = prim_parents_in_lds<C>() ? (size_t)2 * 1024 * C : 0;           \
        if (lds > 0) {                                                                     \
            const hipError_t e = hipFuncSetAttribute(                                      \
                (const void*)tree_finish_kernel<C, WIDEST>,                                \
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                     \
            if (e != hipSuccess) return e;                                                 \
        }                                                                                  \
        APPD_LAUNCH("tree_finish_kernel", s,                                               \
                    tree_finish_kernel<C, WIDEST><<<blocks, 1024, lds, s>>>(W, n, out, w.par, \
                        w.keyup, w.link, w.size, w.gcount, w.hook, w.lb, w.ctrl));         \
        return hipGetLastError();                                                          \
    }
    APPD_FIN(1)
    APPD_FIN(2)
    APPD_FIN(4)
    APPD_FIN(8)
    APPD_FIN(16)
    APPD_FIN(24)
    APPD_FIN(32)
    APPD_FIN(46)
#undef APPD_FIN
    return hipErrorInvalidValue;
}

template <bool WIDEST>
static void launch_first_pass(const float* W, int n, const TreeWs& w, hipStream_t s) {
    const int blocks = (n + kPassThreads / kWave - 1) / (kPassThreads / kWave);
    const bool vec = (n % 4 == 0) && (((uintptr_t)W & 15u) == 0);
    if (vec)
        APPD_LAUNCH("tree_pass_kernel", s,
            tree_pass_kernel<WIDEST, true><<<blocks, kPassThreads, 0, s>>>(W, n, w.comp, w.best,
                w.lb, w.lptr, (uint32_t*)w.lists, w.ctrl));
    else
        APPD_LAUNCH("tree_pass_kernel", s,
            tree_pass_kernel<WIDEST, false><<<blocks, kPassThreads, 0, s>>>(W, n, w.comp, w.best,
                w.lb, w.lptr, (uint32_t*)w.lists, w.ctrl));
}

template <bool WIDEST>
static void launch_refresh(const float* W, int n, const TreeWs& w, hipStream_t s) {
    const int blocks = kCmatBlocks(n);
    const bool vec = (n % 4 == 0) && (((uintptr_t)W & 15u) == 0);
    if (vec)
        APPD_LAUNCH("tree_refresh_kernel", s,
            tree_refresh_kernel<WIDEST, true><<<blocks, kCmatThreads, 0, s>>>(W, n, w.comp,
                w.lptr, (uint32_t*)w.lists, w.cmpart, w.ctrl));
    else
        APPD_LAUNCH("tree_refresh_kernel", s,
            tree_refresh_kernel<WIDEST, false><<<blocks, kCmatThreads, 0, s>>>(W, n, w.comp,
                w.lptr, (uint32_t*)w.lists, w.cmpart, w.ctrl));
}

template <bool WIDEST>
static hipError_t run_tree_parallel_t(const float* W, int n, PrimOut out, void* tws, int passes,
                                      hipStream_t s) {
    TreeWs w = carve_tree(tws, n);
    const int nb = (n + 255) / 256;
    hipError_t e;
#define APPD_CHK()                                     \
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const bool lds = n <= kMaxLdsN;
    const size_t vbytes = lds ? 4 * (size_t)n : 0;
    int cm = (int)((kLdsBytes - vbytes) / kTableBytes);
    cm = min(4096, cm) & ~63;
    const size_t round_lds = (size_t)cm * kTableBytes + vbytes;
    if (round_lds > 64 * 1024) {
        e = hipFuncSetAttribute(lds ? (const void*)tree_rounds_kernel<true, WIDEST>
                                    : (const void*)tree_rounds_kernel<false, WIDEST>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)round_lds);
        if (e != hipSuccess) return e;
    }
    RoundArgs ra{W,      n,    w.comp, w.best, w.lb, w.lptr, (const uint32_t*)w.lists,
                 w.hook, w.hx, w.hy,   w.par,  w.ctrl, w.cmpart, cm};
    for (int p = 0; p < passes; ++p) {
        if (p == 0)
            launch_first_pass<WIDEST>(W, n, w, s);
        else  // candidate lists, or the component table once few are left
            launch_refresh<WIDEST>(W, n, w, s);
        APPD_CHK();
        if (lds)
            APPD_LAUNCH("tree_rounds_kernel", s,
                tree_rounds_kernel<true, WIDEST><<<1, kRoundThreads, round_lds, s>>>(ra));
        else
            APPD_LAUNCH("tree_rounds_kernel", s,
                tree_rounds_kernel<false, WIDEST><<<1, kRoundThreads, round_lds, s>>>(ra));
        APPD_CHK();
    }
    e = launch_finish<WIDEST>(W, n, out, w, s);
    if (e != hipSuccess) return e;
    APPD_LAUNCH("tree_link_kernel", s,
        tree_link_kernel<<<nb * kXcds, 256, 0, s>>>(n, w.keyup, w.link, w.gcount, w.ctrl));
    APPD_CHK();
    // the packed (size, arrivals) words go to lb, free by now
    const int nsb = (n + kScanBlock - 1) / kScanBlock;
    APPD_LAUNCH("tree_sizes_scan_kernel", s,
        tree_sizes_scan_kernel<<<nsb + nb, kScanThreads, 0, s>>>(n, nsb, w.link, w.lb, w.gcount,
            w.gstart, w.gfill, w.tstart, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_group_kernel", s,
        tree_group_kernel<<<(n + kGroupThreads - 1) / kGroupThreads, kGroupThreads, 0, s>>>(n,
            w.link, w.gstart, w.gfill, w.grouped, w.rank, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_rank_kernel", s,
        tree_rank_kernel<<<1024, kRankTile, 0, s>>>(n, w.gcount, w.gstart, w.tstart, w.grouped,
            w.keyup, w.rank, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_place_kernel", s,
        tree_place_kernel<<<nb, 256, 0, s>>>(n, w.link, w.gstart, w.rank, w.lb, w.sorted_size,
            w.sorted_grp, w.ctrl));
    APPD_CHK();
    const int nseg = max(1, (n - 1 + kScanBlock - 1) / kScanBlock);
    APPD_LAUNCH("tree_segscan_kernel", s,
        tree_segscan_kernel<<<nseg, kScanThreads, 0, s>>>(n, w.sorted_size, w.sorted_grp, w.gstart,
                                                          w.sorted_pre, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_pos_kernel", s,
        tree_pos_kernel<<<nb, 256, 0, s>>>(n, w.link, w.gstart, w.rank, w.sorted_pre, w.keyup,
            w.par, out, w.ctrl));
    APPD_CHK();
#undef APPD_CHK
    return hipSuccess;
}

hipError_t run_tree_parallel(const float* W, int n, int mode, const PrimOut& out, void* tws,
                             hipStream_t s) {
    const int passes = (mode & APPD_TREE_ONE_PASS) ? 1 : kPasses;
    return (mode & 1) ? run_tree_parallel_t<true>(W, n, out, tws, passes, s)
                      : run_tree_parallel_t<false>(W, n, out, tws, passes, s);
}

// ---------------------------------------------------------------- dendrogram
// The single-linkage merge table of a graph from Prim's attachment order.  With
// v_0 .. v_{n-1} the attachment order and h[k] the key of the edge that
// attached v_k, the pair (v_a, v_b), a < b, merges at max h[a+1..b] (the
// range-maximum form of Algorithm 4, see appd_fill.h), so the dendrogram is
// the max-Cartesian tree of h[1..n-1]: node k joins the vertex ranges
// [pg(k), k-1] and [k, ng(k)-1], pg / ng being the nearest positions with a
// larger key to the left (0 if none) and to the right (n if none).  From the
// link tree: pg(k) = pos(link(v_k)), because the vertices between a link
// parent and v_k hang below it through smaller keys, and ng(k) = k + size(v_k),
// the end of v_k's link subtree.  A node's parent is whichever of pg, ng holds
// the smaller key; merge j is the node with the j-th smallest key (the tree
// order).  Merge rows follow the usual linkage-matrix layout.
namespace {

__global__ void lk_flag_kernel(int32_t* ctrl) { ctrl[C_ORDERED] = 1; }

__global__ __launch_bounds__(256) void lk_ranges_kernel(int n, const int32_t* order,
                                                        const int32_t* pos, const int32_t* link,
                                                        const int32_t* size, int32_t* pg,
                                                        int32_t* ng, int32_t* lc, int32_t* rc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (k >= n) return;
    const int v = order[k];
    const int l = link[v];
    pg[k] = l > 0 ? pos[l] : 0;
    ng[k] = k + size[v];
    lc[k] = -1;
    rc[k] = -1;
}

__global__ __launch_bounds__(256) void lk_children_kernel(int n, const uint64_t* ek,
                                                          const int32_t* pg, const int32_t* ng,
                                                          int32_t* lc, int32_t* rc) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (k >= n) return;
    const int a = pg[k], b = ng[k];
    int p = -1;
    if (a >= 1 && b <= n - 1) p = ek[a] < ek[b] ? a : b;
    else if (a >= 1) p = a;
    else if (b <= n - 1) p = b;
    if (p < 0) return;  // the largest key: the root of the dendrogram
    if (k < p) lc[p] = k;
    else rc[p] = k;
}

// rank[k] = number of keys among h[1..n-1] below h[k] (all distinct)
__global__ __launch_bounds__(256) void lk_rank_kernel(int n, const uint64_t* ek, int32_t* rank) {
    __shared__ uint64_t tile[256];
    const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
    const uint64_t key = k < n ? ek[k] : kNone;
    int cnt = 0;
    for (int base = 1; base < n; base += 256) {
        const int j = base + threadIdx.x;
        tile[threadIdx.x] = j < n ? ek[j] : kNone;
        __syncthreads();
        const int lim = min(256, n - base);
        for (int q = 0; q < lim; ++q) cnt += tile[q] < key ? 1 : 0;
        __syncthreads();
    }
    if (k < n) rank[k] = cnt;
}

template <bool WIDEST>
__global__ __launch_bounds__(256) void lk_rows_kernel(int n, const int32_t* order,
                                                      const uint64_t* ek, const int32_t* pg,
                                                      const int32_t* ng, const int32_t* lc,
                                                      const int32_t* rc, const int32_t* rank,
                                                      double* Z) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
    if (k >= n) return;
    const int64_t a = lc[k] >= 0 ? (int64_t)n + rank[lc[k]] : order[k - 1];
    const int64_t b = rc[k] >= 0 ? (int64_t)n + rank[rc[k]] : order[k];
    double* z = Z + 4 * (size_t)rank[k];
    z[0] = (double)(a < b ? a : b);
    z[1] = (double)(a < b ? b : a);
    z[2] = (double)key_weight<WIDEST>(ek[k]);
    z[3] = (double)(ng[k] - pg[k]);
}

}  // namespace

hipError_t run_linkage(const float* W, int n, int mode, const PrimOut& out, void* tws, double* Z,
                       hipStream_t s) {
    if (n < 2) return hipSuccess;
    TreeWs w = carve_tree(tws, n);
    const int nb = (n + 255) / 256;
    const bool widest = (mode & 1) != 0;
    hipError_t e;
#define APPD_CHK_L()                                   \
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // link tree and its subtree sizes (from the parent array either tree path
    // leaves), then the Cartesian-tree structure and the merge order
    APPD_LAUNCH("lk_flag_kernel", s, lk_flag_kernel<<<1, 1, 0, s>>>(w.ctrl));
    APPD_CHK_L();
    if (widest)
        APPD_LAUNCH("tree_keyup_kernel", s,
            tree_keyup_kernel<true><<<nb, 256, 0, s>>>(W, n, out.parent, w.keyup, w.link, w.size,
                w.gcount, w.hook, nullptr, w.ctrl));
    else
        APPD_LAUNCH("tree_keyup_kernel", s,
            tree_keyup_kernel<false><<<nb, 256, 0, s>>>(W, n, out.parent, w.keyup, w.link, w.size,
                w.gcount, w.hook, nullptr, w.ctrl));
    APPD_CHK_L();
    APPD_LAUNCH("tree_link_kernel", s,
        tree_link_kernel<<<nb * kXcds, 256, 0, s>>>(n, w.keyup, w.link, w.gcount, w.ctrl));
    APPD_CHK_L();
    APPD_LAUNCH("tree_sizes_kernel", s,
        tree_sizes_kernel<<<nb, 256, 0, s>>>(n, w.link, w.size, w.gcount, w.hook, w.ctrl));
    APPD_CHK_L();
    // pg, ng, children, rank in arrays the tree no longer needs
    int32_t *pg = w.gstart, *ng = w.gfill, *lc = w.hx, *rc = w.hy, *rank = w.comp;
    APPD_LAUNCH("lk_ranges_kernel", s,
        lk_ranges_kernel<<<nb, 256, 0, s>>>(n, out.order, out.pos, w.link, w.size, pg, ng, lc,
            rc));
    APPD_CHK_L();
    APPD_LAUNCH("lk_children_kernel", s,
        lk_children_kernel<<<nb, 256, 0, s>>>(n, out.ek, pg, ng, lc, rc));
    APPD_CHK_L();
    APPD_LAUNCH("lk_rank_kernel", s, lk_rank_kernel<<<nb, 256, 0, s>>>(n, out.ek, rank));
    APPD_CHK_L();
    if (widest)
        APPD_LAUNCH("lk_rows_kernel", s,
            lk_rows_kernel<true><<<nb, 256, 0, s>>>(n, out.order, out.ek, pg, ng, lc, rc, rank,
                Z));
    else
        APPD_LAUNCH("lk_rows_kernel", s,
            lk_rows_kernel<false><<<nb, 256, 0, s>>>(n, out.order, out.ek, pg, ng, lc, rc, rank,
                Z));
    APPD_CHK_L();
#undef APPD_CHK_L
    return hipSuccess;
}

}  // namespace appd

namespace appd {
// Passes over W and Boruvka rounds the last parallel-tree run used, and
// whether it fell back to sequential Prim (read from the control words).
hipError_t tree_stats(const void* tws, int n, int32_t* passes, int32_t* rounds, int32_t* fallback,
                      int32_t* tables, hipStream_t s) {
    TreeWs w = carve_tree(const_cast<void*>(tws), n);
    int32_t c[C_WORDS];
    hipError_t e = hipMemcpyAsync(c, w.ctrl, sizeof(c), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    *passes = c[C_PASSES];
    *rounds = c[C_ROUNDS];
    *fallback = c[C_FALLBACK];
    *tables = c[C_TABLES];
    return hipSuccess;
}
}  // namespace appd
