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
// decide, another pass refreshes the lists.  Each hooking component is re-rooted
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
#include "appd_prim.h"

namespace appd {

constexpr int kK = 16;             // candidate list length
constexpr int kPasses = 4;         // passes over W before falling back to Prim
constexpr int kPassThreads = 256;  // 4 waves, one row each
constexpr int kRoundThreads = 1024;
constexpr int kRankTile = 256;
constexpr int kMaxLdsN = 32768;    // comp + parent as 16-bit values in LDS
constexpr int kLdsBytes = 150 * 1024;  // dynamic LDS the rounds kernel may take
constexpr int kTableBytes = 28;        // per-component table entry
constexpr uint64_t kNone = ~0ull;

// control block (int32 words); word 32 holds the number of rank tiles
enum { C_DONE = 0, C_NCOMP, C_NEED_PASS, C_FALLBACK, C_ROUNDS, C_ORDERED, C_WORDS };
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

// ---------------------------------------------------------------- init
__global__ void tree_init_kernel(int n, int32_t* comp, uint64_t* best, uint64_t* lb,
                                 int32_t* ctrl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        comp[i] = i;
        best[i] = kNone;
        lb[i] = kNone;
    }
    if (i < 64) ctrl[i] = (i == C_NCOMP) ? n : 0;
    if (i == 0 && n == 1) ctrl[C_DONE] = 1;
}

// ---------------------------------------------------------------- pass
// One wave per row.  Lanes 0..K-1 hold the row's K smallest entries seen so
// far, in ascending order; tau is the K-th.  An element is offered only when it
// beats tau, so after the first few columns almost every element costs one
// compare: a candidate is broadcast, its rank among the list (a ballot) gives
// its slot, the lanes above shift up by one.
// VEC: rows are 16-byte aligned (n % 4 == 0), each lane reads 4 columns at once.
template <bool WIDEST, bool FILTER, bool VEC>
__global__ __launch_bounds__(kPassThreads) void tree_pass_kernel(const float* __restrict__ W,
                                                                 int n,
                                                                 const int32_t* __restrict__ comp,
                                                                 int32_t* __restrict__ lptr,
                                                                 uint64_t* __restrict__ lists,
                                                                 const int32_t* __restrict__ ctrl) {
    if (ctrl[C_DONE]) return;
    const int lane = threadIdx.x & (kWave - 1);
    const int u = blockIdx.x * (kPassThreads / kWave) + threadIdx.x / kWave;
    if (u >= n) return;  // no barrier in this kernel
    const float* row = W + (size_t)u * (size_t)n;
    const int cu = FILTER ? comp[u] : u;
    uint64_t mine = kNone;  // this lane's slot of the sorted list (lanes < K)
    uint64_t tau = kNone;   // the K-th smallest so far (wave-uniform)
    auto offer = [&](float w, int v, int cv) {
        const bool skip = FILTER ? (cv == cu) : (v == u);
        const uint64_t e =
            skip ? kNone : (((uint64_t)ord32(WIDEST ? -w : w) << 32) | (uint32_t)v);
        uint64_t bal = __ballot(e < tau);
        while (bal) {
            const int src = __ffsll((unsigned long long)bal) - 1;
            bal &= bal - 1;
            const uint64_t x = shfl_u64(e, src);
            if (x < tau) {
                const int pos = __popcll(__ballot(lane < kK && mine < x));
                const uint64_t below = shfl_up_u64(mine, 1);
                if (lane < kK) mine = lane > pos ? below : (lane == pos ? x : mine);
                tau = shfl_u64(mine, kK - 1);
            }
        }
    };
    if (VEC) {
        constexpr int U = 4;
        // the trip count must be the same for every lane (offer() is wave-wide)
        for (int b0 = 0; b0 < n; b0 += kWave * 4 * U) {
            const int base = b0 + lane * 4;
            float4 x[U];
            int4 c[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave * 4;
                if (v < n) {
                    x[j] = *(const float4*)(row + v);
                    if (FILTER) c[j] = *(const int4*)(comp + v);
                } else {
                    x[j] = make_float4(0.f, 0.f, 0.f, 0.f);
                    c[j] = make_int4(cu, cu, cu, cu);
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave * 4;
                // out-of-range columns (v >= n) are offered as skipped entries
                const bool in = v < n;
                offer(x[j].x, in ? v : u, FILTER ? c[j].x : 0);
                offer(x[j].y, in ? v + 1 : u, FILTER ? c[j].y : 0);
                offer(x[j].z, in ? v + 2 : u, FILTER ? c[j].z : 0);
                offer(x[j].w, in ? v + 3 : u, FILTER ? c[j].w : 0);
            }
        }
    } else {
        constexpr int U = 8;
        for (int b0 = 0; b0 < n; b0 += kWave * U) {
            const int base = b0 + lane;
            float x[U];
            int c[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave;
                x[j] = v < n ? row[v] : 0.0f;
                c[j] = (FILTER && v < n) ? comp[v] : cu;
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave;
                offer(x[j], v < n ? v : u, FILTER ? c[j] : 0);
            }
        }
    }
    if (lane < kK) lists[(size_t)u * kK + lane] = mine;
    if (lane == 0) lptr[u] = 0;
}

// ---------------------------------------------------------------- rounds
struct RoundArgs {
    const float* W;
    int n;
    int32_t* comp;  // global copy of the component labels (read by the passes)
    uint64_t* best;
    uint64_t* lb;
    int32_t* lptr;
    const uint64_t* lists;
    int32_t* hook;
    int32_t* hx;  // hooking endpoint inside the component
    int32_t* hy;  // endpoint outside
    int32_t* par;
    int32_t* ctrl;
    int cm;  // capacity of the per-component LDS tables
};

// Block-wide exclusive scan (one workgroup of kRoundThreads threads).
__device__ __forceinline__ int block_excl_scan(int x, int* s) {
    const int t = threadIdx.x;
    s[t] = x;
    __syncthreads();
    for (int d = 1; d < kRoundThreads; d <<= 1) {
        const int y = t >= d ? s[t - d] : 0;
        __syncthreads();
        s[t] += y;
        __syncthreads();
    }
    const int r = s[t] - x;
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
    const bool first = ctrl[C_ROUNDS] == 0;
    for (int v = t; v < n; v += kRoundThreads) {
        if (LDS) {
            setc(v, first ? v : a.comp[v]);
            setp(v, first ? -1 : a.par[v]);
        } else if (first) {
            a.par[v] = -1;
        }
    }
    if (small)
        for (int d = t; d < C; d += kRoundThreads) t_best[d] = t_lb[d] = kNone;
    __syncthreads();

    constexpr int kChunk = 8;
    constexpr int kStride = kChunk * kRoundThreads;
    for (int guard = 0; guard < 64 && !ctrl[C_DONE]; ++guard) {
        if (t == 0) {
            s_flag[0] = 0;  // components that decided this round
            ctrl[C_ROUNDS] += 1;
        }
        // 1. cheapest outgoing candidate (or lower bound) of every vertex; a wave
        //    whose vertices share one component sends one atomic per minimum.
        //    The list words a vertex usually needs (its current entry, the next
        //    one and the last) are gathered for kChunk vertices before use.
        for (int base = 0; base < n; base += kStride) {
            int pp[kChunk];
            uint64_t e0[kChunk], e1[kChunk], el[kChunk];
#pragma unroll
            for (int i = 0; i < kChunk; ++i) {
                const int u = base + i * kRoundThreads + t;
                pp[i] = u < n ? a.lptr[u] : kK;
            }
#pragma unroll
            for (int i = 0; i < kChunk; ++i) {
                const int u = base + i * kRoundThreads + t;
                const uint64_t* L = a.lists + (size_t)u * kK;
                const bool ok = u < n && pp[i] < kK;
                e0[i] = ok ? L[pp[i]] : kNone;
                e1[i] = (ok && pp[i] + 1 < kK) ? L[pp[i] + 1] : kNone;
                el[i] = u < n ? L[kK - 1] : kNone;
            }
#pragma unroll
            for (int i = 0; i < kChunk; ++i) {
                const int u = base + i * kRoundThreads + t;
                const bool act = u < n;
                int cu = -1;
                uint64_t kc = kNone, kb = kNone;
                if (act) {
                    const uint64_t* L = a.lists + (size_t)u * kK;
                    cu = getc(u);
                    int p = pp[i];
                    uint64_t ent = e0[i];
                    if (p < kK && ent != kNone && getc((int)(uint32_t)ent) == cu) {
                        ++p;
                        ent = e1[i];
                        while (p < kK && ent != kNone && getc((int)(uint32_t)ent) == cu) {
                            ++p;
                            ent = p < kK ? L[p] : kNone;
                        }
                    }
                    if (p < kK && ent == kNone) p = kK;  // short list: nothing beyond it
                    if (p != pp[i]) a.lptr[u] = p;
                    if (p < kK) kc = edge_key_of(ent, u, n);
                    else if (el[i] != kNone) kb = edge_key_of(el[i], u, n);
                }
                const int c0 = __shfl(cu, 0);
                const uint64_t same = __ballot(act && cu == c0);
                const uint64_t acts = __ballot(act);
                if (same == acts) {
                    const uint64_t mc = wave_min_u64(kc), mb = wave_min_u64(kb);
                    if (lane == 0) {
                        if (mc != kNone) min_best(c0, mc);
                        if (mb != kNone) min_lb(c0, mb);
                    }
                } else if (act) {
                    if (kc != kNone) min_best(cu, kc);
                    if (kb != kNone) min_lb(cu, kb);
                }
            }
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
        if (decided == 0) {
            // the minima gathered from these lists are stale once the lists are
            // refreshed: clear them for the next call
            if (!small)
                for (int d = t; d < C; d += kRoundThreads) a.best[d] = a.lb[d] = kNone;
            if (t == 0) ctrl[C_NEED_PASS] = 1;
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
        // 6. relabel every vertex; clear the tables for the next round
        for (int u = t; u < n; u += kRoundThreads) setc(u, gethx(geth(getc(u))));
        __syncthreads();
        C = Cn;
        small = C <= cm;
        for (int d = t; d < C; d += kRoundThreads) {
            if (small) t_best[d] = t_lb[d] = kNone;
            else a.best[d] = a.lb[d] = kNone;
        }
        if (t == 0) {
            ctrl[C_NCOMP] = C;
            if (C == 1) ctrl[C_DONE] = 1;
        }
        __syncthreads();
        if (C == 1) break;
    }
    __syncthreads();
    const bool done = ctrl[C_DONE] != 0;
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

// Edge key to the parent, link initialised to the parent.
template <bool WIDEST>
__global__ __launch_bounds__(256) void tree_keyup_kernel(const float* __restrict__ W, int n,
                                                        const int32_t* par, uint64_t* keyup,
                                                        int32_t* link, int32_t* size,
                                                        int32_t* gcount, const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int p = par[v];
    uint64_t k = 0;
    if (p >= 0) k = make_key((WIDEST ? -1.0f : 1.0f) * W[(size_t)v * n + p], flat_idx(v, p, n));
    keyup[v] = k;
    link[v] = p;
    size[v] = 1;
    gcount[v] = 0;
}

// link(v): jump over ancestors whose edge is smaller than e(v).  Any value a
// link[] entry holds at any time is an ancestor reached over smaller edges
// only, so a thread may follow entries other threads are still updating, and
// it publishes its own progress as it goes.  Every jump moves up the tree, so
// each thread ends.
__global__ __launch_bounds__(256) void tree_link_kernel(int n, const uint64_t* keyup,
                                                       int32_t* link, const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    const uint64_t kv = keyup[v];
    int c = link[v];
    while (c > 0 && keyup[c] < kv) {
        c = link[c];
        link[v] = c;
    }
}

// link-subtree sizes and sibling-group sizes
__global__ __launch_bounds__(256) void tree_sizes_kernel(int n, const int32_t* link,
                                                        int32_t* size, int32_t* gcount,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    const int g = link[v];
    atomicAdd(&gcount[g], 1);
    for (int x = g; x > 0; x = link[x]) atomicAdd(&size[x], 1);
}

// One workgroup: group starts and rank-tile starts (exclusive scans over n).
__global__ __launch_bounds__(kRoundThreads) void tree_scan_kernel(int n, const int32_t* gcount,
                                                                 int32_t* gstart, int32_t* gfill,
                                                                 int32_t* tstart, int32_t* ctrl) {
    __shared__ int s_scan[kRoundThreads];
    if (!ctrl[C_ORDERED]) return;
    const int t = threadIdx.x;
    const int per = (n + kRoundThreads - 1) / kRoundThreads;
    const int b0 = min(n, t * per), b1 = min(n, b0 + per);
    int s = 0, ts = 0;
    for (int i = b0; i < b1; ++i) {
        const int m = gcount[i];
        const int nt = (m + kRankTile - 1) / kRankTile;
        s += m;
        ts += m > 1 ? nt * nt : 0;
    }
    int run = block_excl_scan(s, s_scan);
    int trun = block_excl_scan(ts, s_scan);
    for (int i = b0; i < b1; ++i) {
        const int m = gcount[i];
        const int nt = (m + kRankTile - 1) / kRankTile;
        gstart[i] = run;
        gfill[i] = 0;
        tstart[i] = trun;
        run += m;
        trun += m > 1 ? nt * nt : 0;
    }
    if (t == kRoundThreads - 1) ctrl[C_TILES] = trun;
}

__global__ __launch_bounds__(256) void tree_group_kernel(int n, const int32_t* link,
                                                        const int32_t* gstart, int32_t* gfill,
                                                        int32_t* grouped, int32_t* rank,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    const int g = link[v];
    grouped[gstart[g] + atomicAdd(&gfill[g], 1)] = v;
    rank[v] = 0;
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
        // groups without tiles share their tstart with the next group that has
        // tiles, so the last g with tstart[g] <= tile owns the tile
        int lo = 0, hi = n - 1;
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
                                                        const int32_t* rank, const int32_t* size,
                                                        int32_t* sorted_size, int32_t* sorted_grp,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_ORDERED]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    const int g = link[v];
    const int slot = gstart[g] + rank[v];
    sorted_size[slot] = size[v];
    sorted_grp[slot] = g;
}

// One workgroup: segmented exclusive scan of the placed sizes (segments =
// sibling groups) -> total size of the smaller siblings of each slot.
__global__ __launch_bounds__(kRoundThreads) void tree_segscan_kernel(
    int n, const int32_t* sorted_size, const int32_t* sorted_grp, int32_t* sorted_pre,
    const int32_t* ctrl) {
    __shared__ int s_val[kRoundThreads];
    __shared__ int s_head[kRoundThreads];
    if (!ctrl[C_ORDERED]) return;
    const int t = threadIdx.x;
    const int m = n - 1;  // slots
    const int per = (m + kRoundThreads - 1) / kRoundThreads;
    const int b = min(m, t * per), e = min(m, b + per);
    int tot = 0, head = 0;
    for (int i = b; i < e; ++i) {
        if (i == 0 || sorted_grp[i] != sorted_grp[i - 1]) {
            tot = 0;
            head = 1;
        }
        tot += sorted_size[i];
    }
    s_val[t] = tot;
    s_head[t] = head;
    __syncthreads();
    // inclusive segmented scan over the chunks: (v, h) + (v', h') = (h' ? v' : v + v', h | h')
    for (int d = 1; d < kRoundThreads; d <<= 1) {
        int pv = 0, ph = 0;
        if (t >= d) {
            pv = s_val[t - d];
            ph = s_head[t - d];
        }
        __syncthreads();
        if (t >= d && !s_head[t]) {
            s_val[t] += pv;
            s_head[t] |= ph;
        }
        __syncthreads();
    }
    int carry = t ? s_val[t - 1] : 0;
    for (int i = b; i < e; ++i) {
        if (i == 0 || sorted_grp[i] != sorted_grp[i - 1]) carry = 0;
        sorted_pre[i] = carry;
        carry += sorted_size[i];
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

// Sequential Prim, run only when the rounds could not finish the tree.
template <int CH, bool WIDEST>
__global__ __launch_bounds__(1024) void tree_fallback_kernel(const float* __restrict__ W, int n,
                                                            PrimOut out, int32_t* ctrl) {
    __shared__ uint64_t red_key[2 * 16];
    __shared__ int32_t red_v[2 * 16];
    if (ctrl[C_DONE]) return;
    if (threadIdx.x == 0) ctrl[C_FALLBACK] = 1;
    prim_run<1024, CH, WIDEST>(W, n, out, red_key, red_v);
}

// ---------------------------------------------------------------- host side
struct TreeWs {
    uint64_t* lists;
    int32_t *comp, *lptr, *hook, *hx, *hy, *par, *link, *size, *gcount, *gstart, *gfill;
    int32_t *tstart, *grouped, *rank, *sorted_size, *sorted_grp, *sorted_pre;
    uint64_t *best, *lb, *keyup;
    int32_t* ctrl;
    size_t bytes;
};

// Order-phase arrays reuse the list storage (the lists are dead by then):
// six int arrays of n fit in the 8 * K * n bytes.
static TreeWs carve_tree(void* ws, int n) {
    char* b = (char*)ws;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char* p = b + off;
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
    w.bytes = off;
    int32_t* r = (int32_t*)w.lists;
    w.tstart = r;
    w.grouped = r + n;
    w.rank = r + 2 * (size_t)n;
    w.sorted_size = r + 3 * (size_t)n;
    w.sorted_grp = r + 4 * (size_t)n;
    w.sorted_pre = r + 5 * (size_t)n;
    return w;
}

size_t tree_workspace_bytes(int n) { return carve_tree(nullptr, n).bytes; }

template <bool WIDEST>
static hipError_t launch_fallback(const float* W, int n, PrimOut out, int32_t* ctrl,
                                  hipStream_t s) {
    const int ch = (n + 1023) / 1024;
#define APPD_FB(C)                                                                   \
    if (ch <= C) {                                                                   \
        APPD_LAUNCH("tree_fallback_kernel", s,                                       \
                    tree_fallback_kernel<C, WIDEST><<<1, 1024, 0, s>>>(W, n, out, ctrl)); \
        return hipGetLastError();                                                    \
    }
    APPD_FB(1)
    APPD_FB(2)
    APPD_FB(4)
    APPD_FB(8)
    APPD_FB(16)
    APPD_FB(24)
    APPD_FB(32)
    APPD_FB(46)
#undef APPD_FB
    return hipErrorInvalidValue;
}

template <bool WIDEST, bool FILTER>
static void launch_pass(const float* W, int n, const TreeWs& w, hipStream_t s) {
    const int blocks = (n + kPassThreads / kWave - 1) / (kPassThreads / kWave);
    const bool vec = (n % 4 == 0) && (((uintptr_t)W & 15u) == 0);
    if (vec)
        APPD_LAUNCH("tree_pass_kernel", s,
            tree_pass_kernel<WIDEST, FILTER, true><<<blocks, kPassThreads, 0, s>>>(W, n, w.comp,
                w.lptr, w.lists, w.ctrl));
    else
        APPD_LAUNCH("tree_pass_kernel", s,
            tree_pass_kernel<WIDEST, FILTER, false><<<blocks, kPassThreads, 0, s>>>(W, n, w.comp,
                w.lptr, w.lists, w.ctrl));
}

template <bool WIDEST>
static hipError_t run_tree_parallel_t(const float* W, int n, PrimOut out, void* tws,
                                      hipStream_t s) {
    TreeWs w = carve_tree(tws, n);
    const int nb = (n + 255) / 256;
    hipError_t e;
#define APPD_CHK()                                     \
    if ((e = hipGetLastError()) != hipSuccess) return e;
    APPD_LAUNCH("tree_init_kernel", s,
        tree_init_kernel<<<max(nb, 1), 256, 0, s>>>(n, w.comp, w.best, w.lb, w.ctrl));
    APPD_CHK();
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
    RoundArgs ra{W,      n,    w.comp, w.best, w.lb, w.lptr, w.lists,
                 w.hook, w.hx, w.hy,   w.par,  w.ctrl, cm};
    for (int p = 0; p < kPasses; ++p) {
        if (p == 0) launch_pass<WIDEST, false>(W, n, w, s);
        else launch_pass<WIDEST, true>(W, n, w, s);
        APPD_CHK();
        if (lds)
            APPD_LAUNCH("tree_rounds_kernel", s,
                tree_rounds_kernel<true, WIDEST><<<1, kRoundThreads, round_lds, s>>>(ra));
        else
            APPD_LAUNCH("tree_rounds_kernel", s,
                tree_rounds_kernel<false, WIDEST><<<1, kRoundThreads, round_lds, s>>>(ra));
        APPD_CHK();
    }
    e = launch_fallback<WIDEST>(W, n, out, w.ctrl, s);
    if (e != hipSuccess) return e;
    APPD_LAUNCH("tree_keyup_kernel", s,
        tree_keyup_kernel<WIDEST><<<nb, 256, 0, s>>>(W, n, w.par, w.keyup, w.link, w.size, w.gcount,
            w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_link_kernel", s,
        tree_link_kernel<<<nb, 256, 0, s>>>(n, w.keyup, w.link, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_sizes_kernel", s,
        tree_sizes_kernel<<<nb, 256, 0, s>>>(n, w.link, w.size, w.gcount, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_scan_kernel", s,
        tree_scan_kernel<<<1, kRoundThreads, 0, s>>>(n, w.gcount, w.gstart, w.gfill, w.tstart,
            w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_group_kernel", s,
        tree_group_kernel<<<nb, 256, 0, s>>>(n, w.link, w.gstart, w.gfill, w.grouped, w.rank,
            w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_rank_kernel", s,
        tree_rank_kernel<<<1024, kRankTile, 0, s>>>(n, w.gcount, w.gstart, w.tstart, w.grouped,
            w.keyup, w.rank, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_place_kernel", s,
        tree_place_kernel<<<nb, 256, 0, s>>>(n, w.link, w.gstart, w.rank, w.size, w.sorted_size,
            w.sorted_grp, w.ctrl));
    APPD_CHK();
    APPD_LAUNCH("tree_segscan_kernel", s,
        tree_segscan_kernel<<<1, kRoundThreads, 0, s>>>(n, w.sorted_size, w.sorted_grp,
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
    return (mode & 1) ? run_tree_parallel_t<true>(W, n, out, tws, s)
                      : run_tree_parallel_t<false>(W, n, out, tws, s);
}

}  // namespace appd
