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
// One wave per row: each lane keeps its K smallest entries in registers
// (insertion), then K rounds of wave-minimum extraction merge the 64 lists.
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
    uint64_t top[kK];
#pragma unroll
    for (int q = 0; q < kK; ++q) top[q] = kNone;
    auto consider = [&](float w, int v, int cv) {
        const bool skip = FILTER ? (cv == cu) : (v == u);
        const uint64_t e =
            skip ? kNone : (((uint64_t)ord32(WIDEST ? -w : w) << 32) | (uint32_t)v);
        if (e < top[kK - 1]) {
            uint64_t x = e;
#pragma unroll
            for (int q = 0; q < kK; ++q) {  // insert, keeping top[] ascending
                const uint64_t t = top[q];
                const bool sw = x < t;
                top[q] = sw ? x : t;
                x = sw ? t : x;
            }
        }
    };
    if (VEC) {
        constexpr int U = 4;
        for (int base = lane * 4; base < n; base += kWave * 4 * U) {
            float4 x[U];
            int4 c[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave * 4;
                if (v < n) {
                    x[j] = *(const float4*)(row + v);
                    if (FILTER) c[j] = *(const int4*)(comp + v);
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave * 4;
                if (v < n) {
                    consider(x[j].x, v, FILTER ? c[j].x : 0);
                    consider(x[j].y, v + 1, FILTER ? c[j].y : 0);
                    consider(x[j].z, v + 2, FILTER ? c[j].z : 0);
                    consider(x[j].w, v + 3, FILTER ? c[j].w : 0);
                }
            }
        }
    } else {
        constexpr int U = 8;
        for (int base = lane; base < n; base += kWave * U) {
            float x[U];
            int c[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave;
                if (v < n) {
                    x[j] = row[v];
                    if (FILTER) c[j] = comp[v];
                }
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int v = base + j * kWave;
                if (v < n) consider(x[j], v, FILTER ? c[j] : 0);
            }
        }
    }
    uint64_t* out = lists + (size_t)u * kK;
    for (int q = 0; q < kK; ++q) {
        const uint64_t m = wave_min_u64(top[0]);
        if (lane == 0) out[q] = m;
        if (m != kNone && top[0] == m) {  // entries are unique: exactly one lane pops
#pragma unroll
            for (int z = 0; z < kK - 1; ++z) top[z] = top[z + 1];
            top[kK - 1] = kNone;
        }
    }
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
    // order phase (run once, by the call that completes the tree)
    uint64_t* keyup;
    int32_t* link;
    int32_t* size;
    int32_t* gcount;
    int32_t* gstart;
    int32_t* gfill;
    int32_t* tstart;
    int32_t* grouped;
    int32_t* rank;
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

// One workgroup.  With LDS: component labels and parents as 16-bit values in
// LDS (n <= kMaxLdsN); otherwise the global arrays are used directly.
template <bool LDS, bool WIDEST>
__global__ __launch_bounds__(kRoundThreads) void tree_rounds_kernel(RoundArgs a) {
    extern __shared__ uint16_t s_mem[];  // [0,n): component, [n,2n): parent
    __shared__ int s_flag[4];
    __shared__ int s_scan[kRoundThreads];
    const int n = a.n;
    const int t = threadIdx.x;
    const int lane = t & (kWave - 1);
    int32_t* ctrl = a.ctrl;
    if (ctrl[C_ORDERED] || ctrl[C_FALLBACK]) return;
    constexpr uint16_t NIL = 0xffff;
    auto getc = [&](int v) -> int { return LDS ? (int)s_mem[v] : a.comp[v]; };
    auto setc = [&](int v, int c) {
        if (LDS) s_mem[v] = (uint16_t)c;
        else a.comp[v] = c;
    };
    auto getp = [&](int v) -> int {
        if (LDS) {
            const uint16_t x = s_mem[n + v];
            return x == NIL ? -1 : (int)x;
        }
        return a.par[v];
    };
    auto setp = [&](int v, int p) {
        if (LDS) s_mem[n + v] = p < 0 ? NIL : (uint16_t)p;
        else a.par[v] = p;
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
    __syncthreads();

    for (int guard = 0; guard < 64 && !ctrl[C_DONE]; ++guard) {
        if (t == 0) {
            s_flag[0] = 0;  // components that decided this round
            s_flag[2] = 0;  // components left
            ctrl[C_ROUNDS] += 1;
        }
        // 1. cheapest outgoing candidate (or lower bound) of every vertex; a wave
        //    whose vertices share one component sends one atomic per minimum.
        for (int base = 0; base < n; base += kRoundThreads) {
            const int u = base + t;
            const bool act = u < n;
            int cu = -1;
            uint64_t kc = kNone, kb = kNone;
            if (act) {
                cu = getc(u);
                int p = a.lptr[u];
                const uint64_t* L = a.lists + (size_t)u * kK;
                uint64_t ent = p < kK ? L[p] : kNone;
                while (p < kK && ent != kNone && getc((int)(uint32_t)ent) == cu) {
                    ++p;
                    ent = p < kK ? L[p] : kNone;
                }
                if (p < kK && ent == kNone) p = kK;  // short list: no vertex beyond it
                a.lptr[u] = p;
                if (p < kK) {
                    kc = edge_key_of(ent, u, n);
                } else {
                    const uint64_t last = L[kK - 1];
                    if (last != kNone) kb = edge_key_of(last, u, n);
                }
            }
            const int c0 = __shfl(cu, 0);
            const uint64_t same = __ballot(act && cu == c0);
            const uint64_t acts = __ballot(act);
            if (same == acts) {
                const uint64_t mc = wave_min_u64(kc), mb = wave_min_u64(kb);
                if (lane == 0) {
                    if (mc != kNone) atomicMin((unsigned long long*)&a.best[c0], mc);
                    if (mb != kNone) atomicMin((unsigned long long*)&a.lb[c0], mb);
                }
            } else if (act) {
                if (kc != kNone) atomicMin((unsigned long long*)&a.best[cu], kc);
                if (kb != kNone) atomicMin((unsigned long long*)&a.lb[cu], kb);
            }
        }
        __syncthreads();
        // 2. decide: a component hooks when its best exact candidate beats every bound
        for (int c = t; c < n; c += kRoundThreads) {
            if (getc(c) != c) continue;
            const uint64_t b = ld_l2(&a.best[c]);
            a.hook[c] = c;
            if (b != kNone && b < ld_l2(&a.lb[c])) {
                const uint32_t f = (uint32_t)b;
                const int x0 = (int)(f / (uint32_t)n), y0 = (int)(f % (uint32_t)n);
                const bool xin = getc(x0) == c;
                const int x = xin ? x0 : y0, y = xin ? y0 : x0;
                a.hx[c] = x;
                a.hy[c] = y;
                a.hook[c] = getc(y);
                atomicAdd(&s_flag[0], 1);
            }
        }
        __syncthreads();
        const int decided = s_flag[0];
        if (decided == 0) {
            // the minima gathered from these lists are stale once the lists are
            // refreshed: clear them for the next call
            for (int c = t; c < n; c += kRoundThreads) {
                a.best[c] = kNone;
                a.lb[c] = kNone;
            }
            if (t == 0) ctrl[C_NEED_PASS] = 1;
            break;
        }
        // 3. a mutual pair chose the same edge: the smaller id stays the root.
        //    Every other hooking component re-roots itself at its endpoint,
        //    whose parent becomes the endpoint outside.
        for (int c = t; c < n; c += kRoundThreads) {
            if (getc(c) != c) continue;
            const int h = a.hook[c];
            if (h == c) continue;
            if (a.hook[h] == c && ld_l2(&a.best[h]) == ld_l2(&a.best[c]) && c < h) {
                a.hook[c] = -1 - c;  // root of the pair, restored below
                continue;
            }
            int cur = a.hx[c], prev = a.hy[c];
            while (cur >= 0) {  // reverse the parent pointers on hx -> old root
                const int nxt = getp(cur);
                setp(cur, prev);
                prev = cur;
                cur = nxt;
            }
        }
        __syncthreads();
        for (int c = t; c < n; c += kRoundThreads)
            if (getc(c) == c && a.hook[c] < 0) a.hook[c] = c;
        __syncthreads();
        // 4. pointer jumping: every component id -> the root it now belongs to
        for (int it = 0; it < 64; ++it) {
            if (t == 0) s_flag[1] = 0;
            __syncthreads();
            for (int c = t; c < n; c += kRoundThreads) {
                if (getc(c) != c) continue;
                const int h = a.hook[c];
                const int hh = a.hook[h];
                if (hh != h) {
                    a.hook[c] = hh;
                    s_flag[1] = 1;
                }
            }
            __syncthreads();
            const int again = s_flag[1];
            __syncthreads();  // every thread has read the flag before it is reset
            if (!again) break;
        }
        // 5. relabel; reset the per-component minima; count the roots
        for (int u = t; u < n; u += kRoundThreads) setc(u, a.hook[getc(u)]);
        __syncthreads();
        for (int c = t; c < n; c += kRoundThreads) {
            a.best[c] = kNone;
            a.lb[c] = kNone;
            if (getc(c) == c) atomicAdd(&s_flag[2], 1);
        }
        __syncthreads();
        const int left = s_flag[2];
        if (t == 0) {
            ctrl[C_NCOMP] = left;
            if (left == 1) ctrl[C_DONE] = 1;
        }
        __syncthreads();
        if (left == 1) break;
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

    // ---- order phase, part 1 (this workgroup): edge keys, links, sizes, groups
    const float sg = WIDEST ? -1.0f : 1.0f;
    for (int v = t; v < n; v += kRoundThreads) {
        const int p = getp(v);
        uint64_t k = 0;
        if (p >= 0) k = make_key(sg * a.W[(size_t)v * n + p], flat_idx(v, p, n));
        a.keyup[v] = k;
        a.link[v] = p;
        a.size[v] = 1;
        a.gcount[v] = 0;
    }
    __syncthreads();
    // link(v): jump over ancestors whose edge is smaller than e(v).  Every link[]
    // entry is at all times an ancestor reached over smaller edges only, so the
    // jumps may read entries other threads are updating.
    for (int it = 0; it < 4096; ++it) {
        if (t == 0) s_flag[1] = 0;
        __syncthreads();
        for (int v = t + 1; v < n; v += kRoundThreads) {
            const int c = a.link[v];
            if (c > 0 && a.keyup[c] < a.keyup[v]) {
                a.link[v] = a.link[c];
                s_flag[1] = 1;
            }
        }
        __syncthreads();
        const int again = s_flag[1];
        __syncthreads();
        if (!again) break;
    }
    // link-subtree sizes and sibling-group sizes
    for (int v = t + 1; v < n; v += kRoundThreads) {
        const int g = a.link[v];
        atomicAdd(&a.gcount[g], 1);
        for (int x = g; x > 0; x = a.link[x]) atomicAdd(&a.size[x], 1);
    }
    __syncthreads();
    // group starts and rank-tile starts (exclusive scans over n)
    const int per = (n + kRoundThreads - 1) / kRoundThreads;
    const int b0 = min(n, t * per), b1 = min(n, b0 + per);
    int s = 0, ts = 0;
    for (int i = b0; i < b1; ++i) {
        const int m = ld_l2(&a.gcount[i]);
        const int nt = (m + kRankTile - 1) / kRankTile;
        s += m;
        ts += m > 1 ? nt * nt : 0;
    }
    int run = block_excl_scan(s, s_scan);
    int trun = block_excl_scan(ts, s_scan);
    for (int i = b0; i < b1; ++i) {
        const int m = ld_l2(&a.gcount[i]);
        const int nt = (m + kRankTile - 1) / kRankTile;
        a.gstart[i] = run;
        a.gfill[i] = 0;
        a.tstart[i] = trun;
        run += m;
        trun += m > 1 ? nt * nt : 0;
    }
    if (t == kRoundThreads - 1) ctrl[C_TILES] = trun;
    __syncthreads();
    for (int v = t + 1; v < n; v += kRoundThreads) {
        const int g = a.link[v];
        a.grouped[a.gstart[g] + atomicAdd(&a.gfill[g], 1)] = v;
        a.rank[v] = 0;
    }
    if (t == 0) ctrl[C_ORDERED] = 1;
}

// ---------------------------------------------------------------- order, part 2
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

// One workgroup: place each vertex's link-subtree size at (group start + rank),
// then a segmented exclusive scan gives the sizes of smaller siblings.
__global__ __launch_bounds__(kRoundThreads) void tree_presize_kernel(
    int n, const int32_t* link, const int32_t* gstart, const int32_t* rank, const int32_t* size,
    int32_t* sorted_size, int32_t* sorted_grp, int32_t* sorted_pre, const int32_t* ctrl) {
    __shared__ int s_val[kRoundThreads];
    __shared__ int s_head[kRoundThreads];
    if (!ctrl[C_ORDERED]) return;
    const int t = threadIdx.x;
    for (int v = t + 1; v < n; v += kRoundThreads) {
        const int slot = gstart[link[v]] + rank[v];
        sorted_size[slot] = size[v];
        sorted_grp[slot] = link[v];
    }
    __syncthreads();
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
        tree_fallback_kernel<C, WIDEST><<<1, 1024, 0, s>>>(W, n, out, ctrl);         \
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
        tree_pass_kernel<WIDEST, FILTER, true><<<blocks, kPassThreads, 0, s>>>(
            W, n, w.comp, w.lptr, w.lists, w.ctrl);
    else
        tree_pass_kernel<WIDEST, FILTER, false><<<blocks, kPassThreads, 0, s>>>(
            W, n, w.comp, w.lptr, w.lists, w.ctrl);
}

template <bool WIDEST>
static hipError_t run_tree_parallel_t(const float* W, int n, PrimOut out, void* tws,
                                      hipStream_t s) {
    TreeWs w = carve_tree(tws, n);
    const int nb = (n + 255) / 256;
    hipError_t e;
#define APPD_CHK()                                     \
    if ((e = hipGetLastError()) != hipSuccess) return e;
    tree_init_kernel<<<max(nb, 1), 256, 0, s>>>(n, w.comp, w.best, w.lb, w.ctrl);
    APPD_CHK();
    const bool lds = n <= kMaxLdsN;
    const size_t round_lds = lds ? 4 * (size_t)n : 0;
    if (round_lds > 64 * 1024) {
        e = hipFuncSetAttribute((const void*)tree_rounds_kernel<true, WIDEST>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)round_lds);
        if (e != hipSuccess) return e;
    }
    RoundArgs ra{W,      n,        w.comp,   w.best,  w.lb,     w.lptr,    w.lists,
                 w.hook, w.hx,     w.hy,     w.par,   w.ctrl,   w.keyup,   w.link,
                 w.size, w.gcount, w.gstart, w.gfill, w.tstart, w.grouped, w.rank};
    for (int p = 0; p < kPasses; ++p) {
        if (p == 0) launch_pass<WIDEST, false>(W, n, w, s);
        else launch_pass<WIDEST, true>(W, n, w, s);
        APPD_CHK();
        if (lds)
            tree_rounds_kernel<true, WIDEST><<<1, kRoundThreads, round_lds, s>>>(ra);
        else
            tree_rounds_kernel<false, WIDEST><<<1, kRoundThreads, 0, s>>>(ra);
        APPD_CHK();
    }
    e = launch_fallback<WIDEST>(W, n, out, w.ctrl, s);
    if (e != hipSuccess) return e;
    tree_rank_kernel<<<1024, kRankTile, 0, s>>>(n, w.gcount, w.gstart, w.tstart, w.grouped,
                                                w.keyup, w.rank, w.ctrl);
    APPD_CHK();
    tree_presize_kernel<<<1, kRoundThreads, 0, s>>>(n, w.link, w.gstart, w.rank, w.size,
                                                    w.sorted_size, w.sorted_grp, w.sorted_pre,
                                                    w.ctrl);
    APPD_CHK();
    tree_pos_kernel<<<nb, 256, 0, s>>>(n, w.link, w.gstart, w.rank, w.sorted_pre, w.keyup, w.par,
                                       out, w.ctrl);
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
