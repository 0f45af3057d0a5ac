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
// Tree.  A full pass over W keeps, for every row u, its K smallest keys towards
// vertices outside u's component (sorted).  Boruvka rounds then run on these
// lists in one workgroup: a vertex's first list entry outside its component is
// its exact cheapest outgoing edge; a vertex whose list is used up only bounds
// its outgoing edges from below by its K-th entry.  A component whose best exact
// candidate is below every such bound has found its cheapest outgoing edge,
// which is a tree edge (cut property), and hooks along it.  When no component can
// decide, rows whose lists are used up are refreshed by another pass.  Each
// hooking component is re-rooted at its endpoint (the parent pointers on the
// path to its old root are reversed), so the merged tree stays rooted; at the
// end it is re-rooted at vertex 0.
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

constexpr int kK = 16;              // list length
constexpr int kPassThreads = 256;   // 4 waves, one row per wave at a time
constexpr int kPassRowsPerWG = 16;
constexpr int kRoundThreads = 1024;
constexpr int kRankTile = 256;
constexpr uint64_t kNone = ~0ull;

// control block (int32 words)
enum { C_DONE = 0, C_NCOMP, C_NEDGES, C_NEED_PASS, C_FALLBACK, C_ROUNDS, C_PASSES, C_WORDS };

// List entries are ord32(w) << 32 | v: within one row the flat index of (u, v)
// grows with v, so this orders a row exactly like the global edge key.
__device__ __forceinline__ uint64_t edge_key_of(uint64_t entry, uint32_t u, uint32_t n) {
    const uint32_t v = (uint32_t)entry;
    return (entry & 0xffffffff00000000ull) | (uint64_t)flat_idx(u, v, n);
}

// Values updated by device-scope atomics (performed in L2) are read past L1.
__device__ __forceinline__ uint64_t load_l2(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- init
__global__ void tree_init_kernel(int n, int32_t* comp, uint64_t* best, uint64_t* lb,
                                 int32_t* lptr, int32_t* ctrl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        comp[i] = i;
        best[i] = kNone;
        lb[i] = kNone;
        lptr[i] = kK;  // every list "used up": the first pass fills all rows
    }
    if (i < C_WORDS) ctrl[i] = (i == C_NCOMP) ? n : 0;
    if (i == 0 && n == 1) ctrl[C_DONE] = 1;
}

// ---------------------------------------------------------------- pass
// Wave-wide top-K of a row: each lane keeps its K smallest in registers
// (insertion), then K rounds of wave-minimum extraction merge them.
template <bool WIDEST, bool FILTER>
__global__ __launch_bounds__(kPassThreads) void tree_pass_kernel(const float* __restrict__ W,
                                                                 int n,
                                                                 const int32_t* __restrict__ comp,
                                                                 int32_t* __restrict__ lptr,
                                                                 uint64_t* __restrict__ lists,
                                                                 const int32_t* __restrict__ ctrl) {
    extern __shared__ uint16_t s_comp[];  // n entries when FILTER
    if (ctrl[C_DONE]) return;
    if (FILTER) {
        for (int v = threadIdx.x; v < n; v += kPassThreads) s_comp[v] = (uint16_t)comp[v];
        __syncthreads();
    }
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int r0 = blockIdx.x * kPassRowsPerWG;
    const int r1 = min(n, r0 + kPassRowsPerWG);
    for (int u = r0 + wid; u < r1; u += kPassThreads / kWave) {
        if (lptr[u] < kK) continue;  // its list still reaches outside: keep it
        const float* row = W + (size_t)u * (size_t)n;
        const uint32_t cu = FILTER ? s_comp[u] : (uint32_t)u;
        uint64_t top[kK];
#pragma unroll
        for (int q = 0; q < kK; ++q) top[q] = kNone;
        for (int v = lane; v < n; v += kWave) {
            const float w = row[v];
            const bool skip = FILTER ? (s_comp[v] == cu) : (v == u);
            const uint64_t e = skip ? kNone
                                    : (((uint64_t)ord32(WIDEST ? -w : w) << 32) | (uint32_t)v);
            if (e < top[kK - 1]) {
                // insert, keeping top[] ascending
                uint64_t x = e;
#pragma unroll
                for (int q = 0; q < kK; ++q) {
                    const uint64_t t = top[q];
                    const bool sw = x < t;
                    top[q] = sw ? x : t;
                    x = sw ? t : x;
                }
            }
        }
        // merge the 64 lane lists: K rounds of wave minimum
        uint64_t* out = lists + (size_t)u * kK;
        for (int q = 0; q < kK; ++q) {
            const uint64_t m = wave_min_u64(top[0]);
            if (lane == 0) out[q] = m;
            if (m != kNone && top[0] == m) {  // unique entries: exactly one lane pops
#pragma unroll
                for (int z = 0; z < kK - 1; ++z) top[z] = top[z + 1];
                top[kK - 1] = kNone;
            }
        }
        if (lane == 0) lptr[u] = 0;
    }
}

// ---------------------------------------------------------------- rounds
// One workgroup.  par/upe: parent vertex and parent-edge id of every vertex,
// kept in LDS as 16-bit values while rounds run (n <= 32768), else in global.
struct RoundArgs {
    int n;
    int32_t* comp;
    uint64_t* best;
    uint64_t* lb;
    int32_t* lptr;
    const uint64_t* lists;
    int32_t* hook;
    int32_t* hx;  // hooking endpoint inside the component
    int32_t* hy;  // endpoint outside
    uint64_t* ekey;
    int32_t* par_g;
    int32_t* upe_g;
    int32_t* ctrl;
    int final_call;  // re-root at 0 when done
};

template <bool LDSPAR>
__global__ __launch_bounds__(kRoundThreads) void tree_rounds_kernel(RoundArgs a) {
    extern __shared__ uint16_t s_pu[];  // [0,n): parent, [n,2n): parent edge (LDSPAR)
    __shared__ int s_flag[4];
    const int n = a.n;
    const int t = threadIdx.x;
    int32_t* ctrl = a.ctrl;
    if (ctrl[C_DONE] && !a.final_call) return;
    const uint16_t NIL = 0xffff;
    auto getp = [&](int v) -> int {
        if (LDSPAR) { const uint16_t x = s_pu[v]; return x == NIL ? -1 : (int)x; }
        return a.par_g[v];
    };
    auto setp = [&](int v, int p) {
        if (LDSPAR) s_pu[v] = p < 0 ? NIL : (uint16_t)p;
        else a.par_g[v] = p;
    };
    auto gete = [&](int v) -> int {
        if (LDSPAR) { const uint16_t x = s_pu[n + v]; return x == NIL ? -1 : (int)x; }
        return a.upe_g[v];
    };
    auto sete = [&](int v, int e) {
        if (LDSPAR) s_pu[n + v] = e < 0 ? NIL : (uint16_t)e;
        else a.upe_g[v] = e;
    };
    // load the rooted forest built so far (first call: every vertex a root)
    const bool first = ctrl[C_ROUNDS] == 0;
    if (LDSPAR) {
        for (int v = t; v < n; v += kRoundThreads) {
            setp(v, first ? -1 : a.par_g[v]);
            sete(v, first ? -1 : a.upe_g[v]);
        }
    } else if (first) {
        for (int v = t; v < n; v += kRoundThreads) {
            a.par_g[v] = -1;
            a.upe_g[v] = -1;
        }
    }
    __syncthreads();

    for (int guard = 0; guard < 64 && !ctrl[C_DONE]; ++guard) {
        if (t == 0) {
            s_flag[0] = 0;  // resolved components this round
            s_flag[1] = 0;  // changed during pointer jumping
            s_flag[2] = 0;  // components left
            ctrl[C_ROUNDS] += 1;
        }
        // 1. cheapest outgoing candidate (or lower bound) of every vertex
        for (int u = t; u < n; u += kRoundThreads) {
            const int cu = a.comp[u];
            int p = a.lptr[u];
            const uint64_t* L = a.lists + (size_t)u * kK;
            while (p < kK && L[p] != kNone && a.comp[(uint32_t)L[p]] == cu) ++p;
            if (p < kK && L[p] == kNone) p = kK;  // short list (n - 1 < K): nothing beyond
            a.lptr[u] = p;
            if (p < kK) {
                atomicMin((unsigned long long*)&a.best[cu],
                          (unsigned long long)edge_key_of(L[p], u, n));
            } else if (L[kK - 1] != kNone) {
                atomicMin((unsigned long long*)&a.lb[cu],
                          (unsigned long long)edge_key_of(L[kK - 1], u, n));
            }
        }
        __syncthreads();
        // 2. decide: a component hooks when its best exact candidate beats every bound
        for (int c = t; c < n; c += kRoundThreads) {
            if (a.comp[c] != c) continue;
            const uint64_t b = load_l2(&a.best[c]);
            const bool res = b != kNone && b < load_l2(&a.lb[c]);
            a.hook[c] = c;
            if (res) {
                const uint32_t f = (uint32_t)b;
                const int x0 = (int)(f / (uint32_t)n), y0 = (int)(f % (uint32_t)n);
                const bool xin = a.comp[x0] == c;
                a.hx[c] = xin ? x0 : y0;
                a.hy[c] = xin ? y0 : x0;
                a.hook[c] = a.comp[a.hy[c]];
                atomicAdd(&s_flag[0], 1);
            }
        }
        __syncthreads();
        if (s_flag[0] == 0) {
            if (t == 0) ctrl[C_NEED_PASS] = 1;
            break;
        }
        // 3. a mutual pair chose the same edge: the smaller id stays the root.
        //    Every other hooking component records its edge and re-roots itself
        //    at its endpoint, whose parent becomes the endpoint outside.
        for (int c = t; c < n; c += kRoundThreads) {
            if (a.comp[c] != c) continue;
            const int h = a.hook[c];
            if (h == c) continue;
            if (a.hook[h] == c && load_l2(&a.best[h]) == load_l2(&a.best[c]) && c < h) {
                a.hook[c] = -1 - c;  // marker: root of the pair, resolved after the walks
                continue;
            }
            const int e = atomicAdd(&ctrl[C_NEDGES], 1);
            a.ekey[e] = load_l2(&a.best[c]);
            // reverse the parent pointers on the path hx -> old root
            int cur = a.hx[c], prev = a.hy[c], pe = e;
            while (cur >= 0) {
                const int nxt = getp(cur);
                const int ne = gete(cur);
                setp(cur, prev);
                sete(cur, pe);
                prev = cur;
                pe = ne;
                cur = nxt;
            }
        }
        __syncthreads();
        for (int c = t; c < n; c += kRoundThreads)
            if (a.comp[c] == c && a.hook[c] < 0) a.hook[c] = c;
        __syncthreads();
        // 4. pointer jumping: every component id -> its new root
        for (int it = 0; it < 32; ++it) {
            if (t == 0) s_flag[1] = 0;
            __syncthreads();
            for (int c = t; c < n; c += kRoundThreads) {
                if (a.comp[c] != c) continue;
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
        // 5. relabel; reset the per-component minima of the surviving roots
        for (int u = t; u < n; u += kRoundThreads) {
            const int cu = a.comp[u];
            a.comp[u] = a.hook[cu];
        }
        __syncthreads();
        for (int c = t; c < n; c += kRoundThreads) {
            a.best[c] = kNone;
            a.lb[c] = kNone;
            if (a.comp[c] == c) atomicAdd(&s_flag[2], 1);
        }
        __syncthreads();
        if (t == 0) {
            ctrl[C_NCOMP] = s_flag[2];
            if (s_flag[2] == 1) ctrl[C_DONE] = 1;
        }
        __syncthreads();
    }
    __syncthreads();
    // finished: re-root at vertex 0 (one thread walks the path 0 -> root)
    if (ctrl[C_DONE] && a.final_call && t == 0) {
        int cur = 0, prev = -1, pe = -1;
        while (cur >= 0) {
            const int nxt = getp(cur);
            const int ne = gete(cur);
            setp(cur, prev);
            sete(cur, pe);
            prev = cur;
            pe = ne;
            cur = nxt;
        }
    }
    __syncthreads();
    if (LDSPAR) {
        for (int v = t; v < n; v += kRoundThreads) {
            a.par_g[v] = getp(v);
            a.upe_g[v] = gete(v);
        }
    }
}

// ---------------------------------------------------------------- order
// Only when the rounds finished the tree (else the sequential fallback ran).
__global__ __launch_bounds__(256) void tree_keyup_kernel(int n, const int32_t* par,
                                                        const int32_t* upe, const uint64_t* ekey,
                                                        uint64_t* keyup, int32_t* link,
                                                        int32_t* gcount, int32_t* size,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    keyup[v] = v == 0 ? 0ull : ekey[upe[v]];
    link[v] = v == 0 ? -1 : par[v];
    gcount[v] = 0;
    size[v] = 1;
}

// link(v): jump over ancestors whose edge is smaller than e(v).  Every link[]
// value is at any time an ancestor reachable over smaller edges only, so the
// jumps may use partially updated entries.
__global__ __launch_bounds__(kRoundThreads) void tree_link_kernel(int n, const uint64_t* keyup,
                                                                 int32_t* link,
                                                                 const int32_t* ctrl) {
    __shared__ int s_changed;
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
    for (int it = 0; it < 4096; ++it) {
        if (threadIdx.x == 0) s_changed = 0;
        __syncthreads();
        for (int v = threadIdx.x + 1; v < n; v += kRoundThreads) {
            const int c = link[v];
            if (c > 0 && keyup[c] < keyup[v]) {
                link[v] = link[c];
                s_changed = 1;
            }
        }
        __syncthreads();
        if (!s_changed) break;
        __syncthreads();
    }
}

// Subtree sizes in the link tree and the group (sibling set) sizes.
__global__ __launch_bounds__(256) void tree_sizes_kernel(int n, const int32_t* link,
                                                        int32_t* size, int32_t* gcount,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    atomicAdd(&gcount[link[v]], 1);
    for (int a = link[v]; a > 0; a = link[a]) atomicAdd(&size[a], 1);
}

// Exclusive scans (one workgroup): group starts, and rank-tile starts of groups.
__global__ __launch_bounds__(kRoundThreads) void tree_scan_kernel(int n, const int32_t* gcount,
                                                                 int32_t* gstart, int32_t* gfill,
                                                                 int32_t* tstart,
                                                                 int32_t* ctrl_tiles,
                                                                 const int32_t* ctrl) {
    __shared__ int s_part[kRoundThreads];
    __shared__ int s_tpart[kRoundThreads];
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
    const int t = threadIdx.x;
    const int per = (n + kRoundThreads - 1) / kRoundThreads;
    const int b = t * per, e = min(n, b + per);
    int s = 0, ts = 0;
    for (int i = b; i < e; ++i) {
        const int m = gcount[i];
        s += m;
        const int nt = (m + kRankTile - 1) / kRankTile;
        ts += m > 1 ? nt * nt : 0;
    }
    s_part[t] = s;
    s_tpart[t] = ts;
    __syncthreads();
    for (int d = 1; d < kRoundThreads; d <<= 1) {
        const int x = t >= d ? s_part[t - d] : 0;
        const int y = t >= d ? s_tpart[t - d] : 0;
        __syncthreads();
        s_part[t] += x;
        s_tpart[t] += y;
        __syncthreads();
    }
    int run = t ? s_part[t - 1] : 0;
    int trun = t ? s_tpart[t - 1] : 0;
    for (int i = b; i < e; ++i) {
        const int m = gcount[i];
        gstart[i] = run;
        gfill[i] = 0;
        tstart[i] = trun;
        run += m;
        const int nt = (m + kRankTile - 1) / kRankTile;
        trun += m > 1 ? nt * nt : 0;
    }
    if (t == kRoundThreads - 1) ctrl_tiles[0] = trun;
}

__global__ __launch_bounds__(256) void tree_group_kernel(int n, const int32_t* link,
                                                        const int32_t* gstart, int32_t* gfill,
                                                        int32_t* grouped, int32_t* rank,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
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
                                                             const int32_t* ntiles,
                                                             const int32_t* grouped,
                                                             const uint64_t* keyup, int32_t* rank,
                                                             const int32_t* ctrl) {
    __shared__ uint64_t s_key[kRankTile];
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
    const int total = ntiles[0];
    for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
        // group owning this tile: last g with tstart[g] <= tile among groups with tiles
        int lo = 0, hi = n - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (tstart[mid] <= tile) lo = mid;
            else hi = mid - 1;
        }
        // groups without tiles share their tstart with the next group that has
        // tiles, so the last match is the owner
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
            const int v = mem[vi];
            const uint64_t kv = keyup[v];
            int cnt = 0;
            const int lim = min(kRankTile, m - mb * kRankTile);
            for (int j = 0; j < lim; ++j) cnt += s_key[j] < kv ? 1 : 0;
            if (cnt) atomicAdd(&rank[v], cnt);
        }
    }
}

// Sizes of smaller siblings: place sizes at (group start + rank), scan within
// groups (one workgroup), read back per vertex.
__global__ __launch_bounds__(256) void tree_place_kernel(int n, const int32_t* link,
                                                        const int32_t* gstart,
                                                        const int32_t* rank, const int32_t* size,
                                                        int32_t* sorted_size, int32_t* sorted_grp,
                                                        const int32_t* ctrl) {
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v == 0 || v >= n) return;
    const int slot = gstart[link[v]] + rank[v];
    sorted_size[slot] = size[v];
    sorted_grp[slot] = link[v];
}

__global__ __launch_bounds__(kRoundThreads) void tree_segscan_kernel(int n,
                                                                    const int32_t* sorted_size,
                                                                    const int32_t* sorted_grp,
                                                                    int32_t* sorted_pre,
                                                                    const int32_t* ctrl) {
    // segmented exclusive scan over m = n - 1 slots, segments = equal group ids
    __shared__ int s_val[kRoundThreads];
    __shared__ int s_head[kRoundThreads];  // 1 if a segment starts inside the chunk
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
    const int m = n - 1;
    const int t = threadIdx.x;
    const int per = (m + kRoundThreads - 1) / kRoundThreads;
    const int b = t * per, e = min(m, b + per);
    // chunk total after its last segment start
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
    // inclusive segmented scan of (val, head) pairs over chunks
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

__global__ __launch_bounds__(256) void tree_pos_kernel(int n, const int32_t* link,
                                                      const int32_t* gstart, const int32_t* rank,
                                                      const int32_t* sorted_pre,
                                                      const uint64_t* keyup, const int32_t* par,
                                                      PrimOut out, const int32_t* ctrl) {
    if (!ctrl[C_DONE] || ctrl[C_FALLBACK]) return;
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
    for (int a = v; a > 0; a = link[a]) p += 1 + sorted_pre[gstart[link[a]] + rank[a]];
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
size_t tree_workspace_bytes(int n) {
    size_t off = 0;
    auto take = [&](size_t b) { off = align_up(off + b); };
    take(8 * (size_t)n * kK);  // lists
    for (int i = 0; i < 12; ++i) take(4 * (size_t)n);  // int arrays
    for (int i = 0; i < 4; ++i) take(8 * (size_t)n);   // u64 arrays
    take(4 * 64);  // control
    return off;
}

struct TreeWs {
    uint64_t* lists;
    int32_t *comp, *lptr, *hook, *hx, *hy, *par, *upe, *link, *size, *gcount, *gstart, *gfill;
    int32_t *tstart, *grouped, *rank, *sorted_size, *sorted_grp, *sorted_pre;
    uint64_t *best, *lb, *ekey, *keyup;
    int32_t* ctrl;
};

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
    int32_t** ints[12] = {&w.comp, &w.lptr, &w.hook, &w.hx, &w.hy, &w.par,
                          &w.upe, &w.link, &w.size, &w.gcount, &w.gstart, &w.gfill};
    for (int i = 0; i < 12; ++i) *ints[i] = (int32_t*)take(4 * (size_t)n);
    uint64_t** longs[4] = {&w.best, &w.lb, &w.ekey, &w.keyup};
    for (int i = 0; i < 4; ++i) *longs[i] = (uint64_t*)take(8 * (size_t)n);
    w.ctrl = (int32_t*)take(4 * 64);
    // order-phase arrays reuse the list storage (lists are dead by then):
    // 6 int arrays of n fit in 8 * K * n bytes
    int32_t* r = (int32_t*)w.lists;
    w.tstart = r;
    w.grouped = r + n;
    w.rank = r + 2 * (size_t)n;
    w.sorted_size = r + 3 * (size_t)n;
    w.sorted_grp = r + 4 * (size_t)n;
    w.sorted_pre = r + 5 * (size_t)n;
    return w;
}

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

template <bool WIDEST>
static hipError_t run_tree_parallel_t(const float* W, int n, PrimOut out, void* tws,
                                      hipStream_t s) {
    TreeWs w = carve_tree(tws, n);
    const int nb = (n + 255) / 256;
    hipError_t e;
#define APPD_CHK()                                     \
    if ((e = hipGetLastError()) != hipSuccess) return e;
    tree_init_kernel<<<max(nb, 1), 256, 0, s>>>(n, w.comp, w.best, w.lb, w.lptr, w.ctrl);
    APPD_CHK();
    const bool ldspar = n <= 32768;
    const size_t pass_lds = 2 * (size_t)n;
    const size_t round_lds = ldspar ? 4 * (size_t)n : 0;
    if (pass_lds > 64 * 1024) {
        e = hipFuncSetAttribute((const void*)tree_pass_kernel<WIDEST, true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)pass_lds);
        if (e != hipSuccess) return e;
    }
    if (round_lds > 64 * 1024) {
        e = hipFuncSetAttribute((const void*)tree_rounds_kernel<true>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)round_lds);
        if (e != hipSuccess) return e;
    }
    RoundArgs ra{n, w.comp, w.best, w.lb, w.lptr, w.lists, w.hook, w.hx, w.hy, w.ekey,
                 w.par, w.upe, w.ctrl, 0};
    const int pass_blocks = (n + kPassRowsPerWG - 1) / kPassRowsPerWG;
    constexpr int kPasses = 3;
    for (int p = 0; p < kPasses; ++p) {
        if (p == 0)
            tree_pass_kernel<WIDEST, false><<<pass_blocks, kPassThreads, 0, s>>>(
                W, n, w.comp, w.lptr, w.lists, w.ctrl);
        else
            tree_pass_kernel<WIDEST, true><<<pass_blocks, kPassThreads, pass_lds, s>>>(
                W, n, w.comp, w.lptr, w.lists, w.ctrl);
        APPD_CHK();
        ra.final_call = p == kPasses - 1;
        if (ldspar)
            tree_rounds_kernel<true><<<1, kRoundThreads, round_lds, s>>>(ra);
        else
            tree_rounds_kernel<false><<<1, kRoundThreads, 0, s>>>(ra);
        APPD_CHK();
    }
    e = launch_fallback<WIDEST>(W, n, out, w.ctrl, s);
    if (e != hipSuccess) return e;
    tree_keyup_kernel<<<nb, 256, 0, s>>>(n, w.par, w.upe, w.ekey, w.keyup, w.link, w.gcount,
                                         w.size, w.ctrl);
    APPD_CHK();
    tree_link_kernel<<<1, kRoundThreads, 0, s>>>(n, w.keyup, w.link, w.ctrl);
    APPD_CHK();
    tree_sizes_kernel<<<nb, 256, 0, s>>>(n, w.link, w.size, w.gcount, w.ctrl);
    APPD_CHK();
    tree_scan_kernel<<<1, kRoundThreads, 0, s>>>(n, w.gcount, w.gstart, w.gfill, w.tstart,
                                                 w.ctrl + 32, w.ctrl);
    APPD_CHK();
    tree_group_kernel<<<nb, 256, 0, s>>>(n, w.link, w.gstart, w.gfill, w.grouped, w.rank,
                                         w.ctrl);
    APPD_CHK();
    tree_rank_kernel<<<1024, kRankTile, 0, s>>>(n, w.gcount, w.gstart, w.tstart, w.ctrl + 32,
                                                w.grouped, w.keyup, w.rank, w.ctrl);
    APPD_CHK();
    tree_place_kernel<<<nb, 256, 0, s>>>(n, w.link, w.gstart, w.rank, w.size, w.sorted_size,
                                         w.sorted_grp, w.ctrl);
    APPD_CHK();
    tree_segscan_kernel<<<1, kRoundThreads, 0, s>>>(n, w.sorted_size, w.sorted_grp,
                                                    w.sorted_pre, w.ctrl);
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
