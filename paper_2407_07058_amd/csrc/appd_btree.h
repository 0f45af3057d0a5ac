// Device pieces of the batched spanning tree (appd_btree.hip, and the
// persistent batched forward in appd_persist.hip): the candidate list of one
// row, and the per-graph tree, Prim order and fill rank tables of one
// workgroup.  See appd_btree.hip for the method.
#pragma once

#include "appd.h"
#include "appd_device.h"
#include "appd_internal.h"
#include "appd_prim.h"
#include "appd_topk.h"

namespace appd {

constexpr int kBtRefreshes = 8;      // refreshes of a stuck graph's lists before Prim
constexpr int kBtK = 16;             // candidate list length
constexpr int kBtPre = 4;            // list entries per vertex read ahead in a round
constexpr uint16_t kNil16 = 0xffff;

// Block-wide exclusive scan over NT threads; s: NT / 64 ints.
template <int NT>
__device__ __forceinline__ int bt_excl_scan(int x, int* s, int* total) {
    constexpr int NW = NT / kWave;
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
    for (int w = 0; w < NW; ++w) {
        const int v = s[w];
        before += w < wid ? v : 0;
        all += v;
    }
    __syncthreads();
    *total = all;
    return before + incl - x;
}

// LDS of one graph, nmax = the class's largest n (bytes: 39 * nmax, see
// btree_lds_bytes).  The rounds' per-component tables and the order phase's
// per-vertex arrays share the same regions.
struct BtLds {
    uint64_t* a8;   // rounds: best[c]   order: keyup[v]
    uint64_t* b8;   // rounds: lb[c]     order: packed (size << 12 | arrivals)[v], then S[v]
    int32_t* c4;    // rounds: hook[c]   order: link[v]
    int32_t* d4;    // rounds: hx[c]     order: gcount[v]
    int32_t* e4;    // rounds: hy[c]     order: gstart[v]
    int32_t* f4;    //                   order: group fill counters
    uint16_t* comp; // component of each vertex (dense ids)
    uint16_t* par;  // rooted forest (kNil16: root)
    uint16_t* mem;  // order: group members
    uint8_t* lptr;  // list pointer of each vertex
};

__host__ __device__ inline size_t btree_lds_bytes(int nmax) { return (size_t)39 * nmax + 64; }

__device__ __forceinline__ BtLds bt_carve(void* base, int nmax) {
    char* p = (char*)base;
    BtLds L;
    L.a8 = (uint64_t*)p;
    p += 8 * nmax;
    L.b8 = (uint64_t*)p;
    p += 8 * nmax;
    L.c4 = (int32_t*)p;
    p += 4 * nmax;
    L.d4 = (int32_t*)p;
    p += 4 * nmax;
    L.e4 = (int32_t*)p;
    p += 4 * nmax;
    L.f4 = (int32_t*)p;
    p += 4 * nmax;
    L.comp = (uint16_t*)p;
    p += 2 * nmax;
    L.par = (uint16_t*)p;
    p += 2 * nmax;
    L.mem = (uint16_t*)p;
    p += 2 * nmax;
    L.lptr = (uint8_t*)p;
    return L;
}

// The same sort with E = N / NT elements per thread held in registers:
// element t * E + r sits in register r of thread t, so the stages whose
// stride is below E run in registers, those below 64 E exchange with another
// lane of the wave (no barrier), and only strides of 64 E and above go
// through LDS with two barriers.  Equal keys (the padding) stay where they
// are, so the payloads remain a permutation.
template <int NT, int E, class K>
__device__ __forceinline__ void bt_bitonic_regs(K* key, uint16_t* pay, int N) {
    const int t = threadIdx.x, lane = t & (kWave - 1);
    const int base = t * E;
    __syncthreads();
    K k[E];
    uint32_t p[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
        k[r] = key[base + r];
        p[r] = pay[base + r];
    }
    for (int size = 2; size <= N; size <<= 1) {
        // strides across waves, through LDS
        for (int stride = size >> 1; stride >= kWave * E; stride >>= 1) {
#pragma unroll
            for (int r = 0; r < E; ++r) {
                key[base + r] = k[r];
                pay[base + r] = (uint16_t)p[r];
            }
            __syncthreads();
            const int pb = base ^ stride;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const K o = key[pb + r];
                const uint32_t po = pay[pb + r];
                const int idx = base + r;
                const bool up = (idx & size) == 0, lower = (idx & stride) == 0;
                if (lower == up ? o < k[r] : o > k[r]) {
                    k[r] = o;
                    p[r] = po;
                }
            }
            __syncthreads();
        }
        // strides across the lanes of a wave
        for (int stride = min(size >> 1, kWave * E / 2); stride >= E; stride >>= 1) {
            const int lm = stride / E;
            const bool lower = (lane & lm) == 0;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const K o = __shfl_xor(k[r], lm);
                const uint32_t po = (uint32_t)__shfl_xor((int)p[r], lm);
                const bool up = ((base + r) & size) == 0;
                if (lower == up ? o < k[r] : o > k[r]) {
                    k[r] = o;
                    p[r] = po;
                }
            }
        }
        // strides within a thread's registers
#pragma unroll
        for (int s = E / 2; s >= 1; s >>= 1) {
            if (s > (size >> 1)) continue;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                if (r & s) continue;
                const int q = r | s;
                const bool up = ((base + r) & size) == 0;
                if ((k[r] > k[q]) == up) {
                    const K kx = k[r];
                    k[r] = k[q];
                    k[q] = kx;
                    const uint32_t px = p[r];
                    p[r] = p[q];
                    p[q] = px;
                }
            }
        }
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
        key[base + r] = k[r];
        pay[base + r] = (uint16_t)p[r];
    }
    __syncthreads();
}

// Ascending bitonic sort of key[0 .. N) (N a power of two) with a 16-bit
// payload, by the NT threads of the workgroup.
template <int NT, class K>
__device__ __forceinline__ void bt_bitonic(K* key, uint16_t* pay, int N) {
    if (N == NT) return bt_bitonic_regs<NT, 1>(key, pay, N);
    if (N == 2 * NT) return bt_bitonic_regs<NT, 2>(key, pay, N);
    if (N == 4 * NT) return bt_bitonic_regs<NT, 4>(key, pay, N);
    if (N == 8 * NT) return bt_bitonic_regs<NT, 8>(key, pay, N);
    // fewer keys than threads: one compare-exchange per thread and stage
    for (int size = 2; size <= N; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            __syncthreads();
            for (int i = threadIdx.x; i < N / 2; i += NT) {
                const int a = 2 * i - (i & (stride - 1));
                const int b = a + stride;
                const bool up = (a & size) == 0;
                const K ka = key[a], kb = key[b];
                if ((ka > kb) == up) {
                    key[a] = kb;
                    key[b] = ka;
                    const uint16_t pa = pay[a];
                    pay[a] = pay[b];
                    pay[b] = pa;
                }
            }
        }
    }
    __syncthreads();
}

// The candidate list of row r (rows of the batch in perm order; rgraph gives
// each row's graph position) by the calling wave; wbuf: 128 entries of LDS
// owned by the wave.  Rows whose candidates overflow take row_topk.
template <bool WIDEST, int E>
__device__ __forceinline__ void bt_pass_row(const float* __restrict__ W,
                                            const int64_t* __restrict__ offsets,
                                            const int32_t* __restrict__ ns,
                                            const int32_t* __restrict__ perm,
                                            const int64_t* __restrict__ noff,
                                            const int32_t* __restrict__ rstart,
                                            const int32_t* __restrict__ rgraph, int r,
                                            uint64_t* __restrict__ lists, uint64_t* wbuf) {
    const int lane = threadIdx.x & (kWave - 1);
    const int i = rgraph[r];
    const int g = perm[i];
    const int n = ns[g];
    const int u = r - rstart[i];
    const float* row = W + offsets[g] + (size_t)u * n;
    float x[E];
    rank_row_load<E>(row, n, x);
    uint64_t mine;
    if (!row_topk_rank_vals<WIDEST, E, kBtK>(x, n, u, wbuf, &mine))
        mine = row_topk<WIDEST, false, false, E, kBtK>(
            row, n, u, [](int) { return 0; }, [](int) { return make_int4(0, 0, 0, 0); });
    if (lane < kBtK) lists[(size_t)(noff[g] + u) * kBtK + lane] = mine;
}

// Scratch of bt_finish_graph besides its BtLds region (LDS).
struct BtAux {
    int* segv;          // NT
    int* segh;          // NT
    uint64_t* red_key;  // 2 * NT / 64
    int32_t* red_v;     // 2 * NT / 64
    int* wsum;          // NT / 64
    int* flag;          // 4
    uint64_t* wbuf;     // 128 per wave: the refresh's candidate buffers
};

template <int NT>
__host__ __device__ constexpr size_t bt_aux_bytes() {
    return 8 * (128 * (NT / 64) + 2 * NT / 64) + 4 * (2 * NT + 2 * NT / 64 + NT / 64 + 4);
}

template <int NT>
__device__ __forceinline__ BtAux bt_aux_carve(char* p) {
    BtAux a;
    a.wbuf = (uint64_t*)p;
    p += 8 * 128 * (NT / 64);
    a.red_key = (uint64_t*)p;
    p += 8 * (2 * NT / 64);
    a.segv = (int*)p;
    p += 4 * NT;
    a.segh = (int*)p;
    p += 4 * NT;
    a.red_v = (int32_t*)p;
    p += 4 * (2 * NT / 64);
    a.wsum = (int*)p;
    p += 4 * (NT / 64);
    a.flag = (int*)p;
    return a;
}

// The tree, Prim order and fill rank tables of the graph at position gpos of
// perm, by the NT threads of the calling workgroup (every thread calls it).
// lds: btree_lds_bytes(nmax) bytes, 8-byte aligned; aux: bt_aux_carve<NT>.
// The caller synchronises the workgroup before reusing either.
template <int NT, int CH, bool WIDEST>
__device__ __forceinline__ void bt_finish_graph(
    const float* __restrict__ Wall, const int64_t* __restrict__ offsets,
    const int32_t* __restrict__ ns, const int32_t* __restrict__ perm,
    const int64_t* __restrict__ noff, int gpos, int nmax, uint64_t* __restrict__ lists_all,
    BatchTree tree, int32_t* __restrict__ tstats, BatchBlk blk, void* lds, const BtAux& aux) {
    constexpr int NW = NT / kWave;
    int* s_segv = aux.segv;
    int* s_segh = aux.segh;
    uint64_t* red_key = aux.red_key;
    int32_t* red_v = aux.red_v;
    int* s_wsum = aux.wsum;
    int* s_flag = aux.flag;
    const int t = threadIdx.x, lane = t & (kWave - 1), wid = t / kWave;
    const int g = perm[gpos];
    const int n = ns[g];
    const int64_t o = noff[g];
    const float* W = Wall + offsets[g];
    uint64_t* lists = lists_all + (size_t)o * kBtK;
    PrimOut out{tree.order + o, tree.ek + o, tree.pos + o, tree.parent + o};
    if (n == 1) {
        if (t == 0) {
            tstats[g] = 1 << 8;
            blk.slot[o] = 0;
            blk.dM[o] = 0.0f;
            blk.dI[o] = -1;
            out.order[0] = 0;
            out.ek[0] = 0;
            out.pos[0] = 0;
            out.parent[0] = -1;
        }
        return;
    }
    BtLds L = bt_carve(lds, nmax);
    const uint32_t un = (uint32_t)n;
    for (int v = t; v < n; v += NT) {
        L.comp[v] = (uint16_t)v;
        L.par[v] = kNil16;
        L.lptr[v] = 0;
    }
    int C = n;
    int nrounds = 0, nrefresh = 0;
    __syncthreads();
    for (int guard = 0; guard < 96 && C > 1; ++guard) {
        {
            ++nrounds;
            // 1. every vertex's first list entry outside its component, or its
            //    bound.  The entries from the list pointer on are read eight at
            //    a time (independent loads), then checked in order.
            for (int d = t; d < C; d += NT) L.a8[d] = L.b8[d] = kTopkNone;
            if (t == 0) s_flag[0] = 0;
            __syncthreads();
            // A vertex's scan from its list pointer: `pre` holds the entries
            // at p .. p + PRE - 1 (read before), further ones are read eight
            // at a time.  (Fewer read ahead in 1024-thread workgroups, whose
            // threads have 128 registers.)
            constexpr int PRE = NT >= 1024 ? 1 : kBtPre;
            auto scan = [&](int v, int p, const uint64_t (&pre)[PRE]) {
                const int cv = L.comp[v];
                const uint64_t* lv = lists + (size_t)v * kBtK;
                int state = 0;  // 0 searching, 1 external entry at p, 2 list ended, 3 used up
                uint64_t e = kTopkNone;
#pragma unroll
                for (int j = 0; j < PRE; ++j) {
                    if (state != 0) continue;
                    if (p + j >= kBtK) {
                        state = 3;
                        continue;
                    }
                    const uint64_t x = pre[j];
                    if ((uint32_t)x >= un) {  // end of the list (or not a vertex)
                        state = 2;
                        p += j;
                    } else if ((int)L.comp[(uint32_t)x] != cv) {
                        state = 1;
                        e = x;
                        p += j;
                    }
                }
                if (state == 0) p += PRE;
                if (state == 3) p = kBtK;
                while (state == 0) {
                    if (p >= kBtK) {
                        state = 3;
                        break;
                    }
                    uint64_t w[8];
#pragma unroll
                    for (int j = 0; j < 8; ++j) w[j] = lv[min(p + j, kBtK - 1)];
#pragma unroll
                    for (int j = 0; j < 8; ++j) {
                        if (state != 0) continue;
                        if (p + j >= kBtK) {
                            state = 3;
                            continue;
                        }
                        const uint64_t x = w[j];
                        if ((uint32_t)x >= un) {
                            state = 2;
                            p += j;
                        } else if ((int)L.comp[(uint32_t)x] != cv) {
                            state = 1;
                            e = x;
                            p += j;
                        }
                    }
                    if (state == 0) p += 8;
                    if (state == 3) p = kBtK;
                }
                L.lptr[v] = (uint8_t)p;
                if (state == 1) {
                    const uint64_t k = (e & 0xffffffff00000000ull) | flat_idx((uint32_t)v, (uint32_t)e, un);
                    atomicMin((unsigned long long*)&L.a8[cv], (unsigned long long)k);
                } else if (state == 3) {
                    // a full list, every entry inside the component: every
                    // outgoing edge of v is larger than its last entry
                    const uint64_t last = lv[kBtK - 1];  // a vertex (checked above)
                    const uint64_t k =
                        (last & 0xffffffff00000000ull) | flat_idx((uint32_t)v, (uint32_t)last, un);
                    atomicMin((unsigned long long*)&L.b8[cv], (unsigned long long)k);
                }
                // state 2: the list held every eligible entry of the row: no bound
            };
            // the first entries of all of this thread's vertices are read
            // before any is checked (one memory latency per round, not one per
            // vertex); 1024-thread workgroups take their vertices one by one
            constexpr int CHP = NT >= 1024 ? 0 : CH;  // vertices read ahead together
            if constexpr (CHP > 0) {
                uint64_t pre[CHP][PRE];
                int p0[CHP];
#pragma unroll
                for (int c = 0; c < CHP; ++c) {
                    const int v = min(t + c * NT, n - 1);
                    p0[c] = L.lptr[v];
                    const uint64_t* lv = lists + (size_t)v * kBtK;
#pragma unroll
                    for (int j = 0; j < PRE; ++j) pre[c][j] = lv[min(p0[c] + j, kBtK - 1)];
                }
#pragma unroll
                for (int c = 0; c < CHP; ++c)
                    if (t + c * NT < n) scan(t + c * NT, p0[c], pre[c]);
            }
            for (int v = t + CHP * NT; v < n; v += NT) {
                uint64_t pv[PRE];
                const int p = L.lptr[v];
#pragma unroll
                for (int j = 0; j < PRE; ++j) pv[j] = lists[(size_t)v * kBtK + min(p + j, kBtK - 1)];
                scan(v, p, pv);
            }
            __syncthreads();
            // 2. decide: hook when the best candidate beats every bound
            for (int d = t; d < C; d += NT) {
                const uint64_t b = L.a8[d];
                L.c4[d] = d;
                if (b != kTopkNone && b < L.b8[d]) {
                    const uint32_t f = (uint32_t)b;
                    const int x0 = (int)(f / un), y0 = (int)(f % un);
                    const bool xin = L.comp[x0] == d;
                    const int x = xin ? x0 : y0, y = xin ? y0 : x0;
                    L.d4[d] = x;
                    L.e4[d] = y;
                    L.c4[d] = L.comp[y];
                    atomicAdd(&s_flag[0], 1);
                }
            }
            __syncthreads();
            const int decided = s_flag[0];
            __syncthreads();
            if (decided == 0) {
                // No component can decide: the smallest component's vertices get
                // fresh lists of their entries outside it (exact candidates), so
                // that it decides in the next round.  After kBtRefreshes such
                // refreshes Prim's algorithm finishes the graph instead.
                if (nrefresh == kBtRefreshes) break;
                ++nrefresh;
                for (int d = t; d < C; d += NT) L.d4[d] = 0;
                if (t == 0) s_flag[2] = 0x7fffffff;
                __syncthreads();
                for (int v = t; v < n; v += NT) atomicAdd(&L.d4[L.comp[v]], 1);
                __syncthreads();
                for (int d = t; d < C; d += NT) atomicMin(&s_flag[2], (L.d4[d] << 16) | d);
                __syncthreads();
                const int sc = s_flag[2] & 0xffff;
                // Only its used-up vertices (every list entry inside the
                // component) need new lists: a vertex whose pointer stopped
                // earlier holds its cheapest outgoing edge (or has none).
                for (int u = wid; u < n; u += NW) {  // u wave-uniform
                    if ((int)L.comp[u] != sc || L.lptr[u] < kBtK) continue;
                    constexpr int kRefE = NT * CH / 64 < 4 ? 4 : (NT * CH / 64 > 32 ? 32 : NT * CH / 64);
                    // the row's entries inside the component become NaN (never
                    // a candidate), then its 16 smallest by rank; a row with
                    // too many candidates under the threshold (heavy ties), and
                    // every row in 1024-thread workgroups (128 registers),
                    // takes the insertion list instead
                    bool have = false;
                    uint64_t mine = kTopkNone;
                    if constexpr (NT < 1024) {
                        float xr[kRefE];
                        rank_row_load<kRefE>(W + (size_t)u * n, n, xr);
#pragma unroll
                        for (int e = 0; e < kRefE; ++e) {
                            const int col = e * kWave + lane;
                            if (col < n && (int)L.comp[col] == sc) xr[e] = __builtin_nanf("");
                        }
                        have = row_topk_rank_vals<WIDEST, kRefE, kBtK>(xr, n, u, aux.wbuf + wid * 128,
                                                                        &mine);
                    }
                    if (!have)
                        mine = row_topk<WIDEST, true, false, kRefE, kBtK>(
                            W + (size_t)u * n, n, u, [&](int c) { return (int)L.comp[c]; },
                            [](int) { return make_int4(0, 0, 0, 0); });
                    if (lane < kBtK) lists[(size_t)u * kBtK + lane] = mine;
                    if (lane == 0) L.lptr[u] = 0;
                }
                __syncthreads();
                continue;
            }
            // 3. a mutual pair chose the same edge: the smaller id stays the
            //    root; every other hooking component re-roots at its endpoint
            for (int d = t; d < C; d += NT) {
                const int h = L.c4[d];
                if (h == d) continue;
                if (d < h && L.c4[h] == d && L.a8[h] == L.a8[d]) {
                    L.c4[d] = d;
                    continue;
                }
                int cur = L.d4[d], prev = L.e4[d];
                while (cur != kNil16) {
                    const int nxt = L.par[cur];
                    L.par[cur] = (uint16_t)prev;
                    prev = cur;
                    cur = nxt;
                }
            }
            __syncthreads();
            // 4. pointer jumping: every component -> the root it now belongs to
            for (int it = 0; it < 32; ++it) {
                if (t == 0) s_flag[1] = 0;
                __syncthreads();
                for (int d = t; d < C; d += NT) {
                    const int h = L.c4[d];
                    const int hh = L.c4[h];
                    if (hh != h) {
                        L.c4[d] = hh;
                        s_flag[1] = 1;
                    }
                }
                __syncthreads();
                const int again = s_flag[1];
                __syncthreads();
                if (!again) break;
            }
            // 5. dense numbers of the roots (kept in d4 of each root)
            const int per = (C + NT - 1) / NT;
            const int d0 = min(C, t * per), d1 = min(C, d0 + per);
            int cnt = 0;
            for (int d = d0; d < d1; ++d) cnt += L.c4[d] == d ? 1 : 0;
            int total;
            int id = bt_excl_scan<NT>(cnt, s_wsum, &total);
            for (int d = d0; d < d1; ++d)
                if (L.c4[d] == d) L.d4[d] = id++;
            __syncthreads();
            // 6. relabel every vertex
            for (int v = t; v < n; v += NT) L.comp[v] = (uint16_t)L.d4[L.c4[L.comp[v]]];
            C = total;
            __syncthreads();
        }
    }
    const bool done = C == 1;
    if (t == 0) tstats[g] = min(nrounds, 255) | ((1 + nrefresh) << 8) | ((done ? 0 : 1) << 16);
    if (!done) {
        // the lists could not finish the tree: Prim's algorithm (same outputs)
        __syncthreads();
        prim_run<NT, CH, WIDEST>(W, n, out, red_key, red_v);
        __syncthreads();
        // the fill's rank tables from Prim's attachment keys
        uint64_t* skey = (uint64_t*)L.d4;
        for (int i = t; i < nmax; i += NT) {
            skey[i] = (i >= 1 && i < n) ? out.ek[i] : ~0ull;  // position i's key
            L.comp[i] = (uint16_t)i;
        }
        bt_bitonic<NT>(skey, L.comp, nmax);
        for (int r = t; r < n; r += NT) {
            if (r == 0) {
                blk.slot[o] = 0;
                blk.dM[o] = 0.0f;
                blk.dI[o] = -1;
                continue;
            }
            const int k = L.comp[r - 1];  // position of the key of rank r - 1
            const uint64_t key = skey[r - 1];
            blk.slot[o + k] = (uint16_t)r;
            blk.dM[o + r] = key_weight<WIDEST>(key);
            blk.dI[o + r] = (int32_t)(uint32_t)key;
        }
        return;
    }
    // re-root the tree at vertex 0
    if (t == 0) {
        int cur = 0, prev = kNil16;
        while (cur != kNil16) {
            const int nxt = L.par[cur];
            L.par[cur] = (uint16_t)prev;
            prev = cur;
            cur = nxt;
        }
    }
    __syncthreads();
    // ---- Prim's order from the tree
    uint64_t* keyup = L.a8;
    uint32_t* pk = (uint32_t*)L.b8;   // (size << 12) | arrivals
    uint32_t* S = pk + nmax;          // sizes of the smaller siblings
    int32_t* link = L.c4;
    int32_t* gcount = L.d4;
    for (int v = t; v < n; v += NT) {
        const int p = v ? (int)L.par[v] : -1;
        uint64_t k = 0;
        if (p >= 0) k = make_key((WIDEST ? -1.0f : 1.0f) * W[(size_t)v * n + p], flat_idx(v, p, un));
        keyup[v] = k;
        link[v] = p;
        gcount[v] = 0;
        pk[v] = 1u << 12;
    }
    __syncthreads();
    // link(v): jump over ancestors whose edge is smaller than e(v).  Any value
    // a link entry holds at any time is an ancestor reached over smaller edges
    // only, so a thread may follow entries other threads still update.
    volatile int32_t* vlink = link;
    for (int v = t; v < n; v += NT) {
        if (v == 0) continue;
        const uint64_t kv = keyup[v];
        int c = vlink[v];
        while (c > 0 && keyup[c] < kv) {
            c = vlink[c];
            vlink[v] = c;
        }
    }
    __syncthreads();
    for (int v = t; v < n; v += NT)
        if (v) atomicAdd(&gcount[link[v]], 1);
    __syncthreads();
    // link-subtree sizes bottom-up: a walk starts at every leaf; one packed
    // atomic adds a child's size and its arrival, and the child that arrives
    // last reads the parent's final size from the value it returns
    for (int v = t; v < n; v += NT) {
        if (v == 0 || gcount[v] != 0) continue;
        int x = v;
        uint32_t sx = 1;
        for (int guard = 0; guard < n; ++guard) {
            const int p = link[x];
            if (p <= 0) break;
            const uint32_t old = atomicAdd(&pk[p], (sx << 12) | 1u);
            if ((int)(old & 0xfffu) + 1 != gcount[p]) break;
            sx += old >> 12;
            x = p;
        }
    }
    __syncthreads();
    // S(v), the total link-subtree size of v's siblings with smaller keys:
    // (a) the vertices 1..n-1 sorted by edge key give each its key rank; (b)
    // sorted by (link parent, key rank) they come grouped by sibling set in
    // key order; (c) an exclusive scan of the sizes restarted at every group
    // gives S.  Keys are distinct, ranks are < 2048 and parents < 2048.
    uint64_t* skey = (uint64_t*)L.d4;  // d4 and e4: 8 bytes per entry
    uint32_t* skey2 = (uint32_t*)L.d4;
    int32_t* rankv = L.f4;
    for (int i = t; i < nmax; i += NT) {
        skey[i] = (i >= 1 && i < n) ? keyup[i] : ~0ull;
        L.comp[i] = (uint16_t)i;
    }
    bt_bitonic<NT>(skey, L.comp, nmax);
    for (int i = t; i < n - 1; i += NT) rankv[L.comp[i]] = i;
    __syncthreads();
    for (int i = t; i < nmax; i += NT) {
        skey2[i] = (i >= 1 && i < n) ? ((uint32_t)link[i] << 11) | (uint32_t)rankv[i] : ~0u;
        L.comp[i] = (uint16_t)i;
    }
    bt_bitonic<NT>(skey2, L.comp, nmax);
    {
        // segmented exclusive scan over positions 0 .. n-2: thread t takes a
        // run of consecutive positions; (sum since the last group start, seen a
        // start) per run, combined across threads
        const int m = n - 1;
        const int per = (m + NT - 1) / NT;
        const int i0 = min(m, t * per), i1 = min(m, i0 + per);
        int tot = 0, head = 0;
        for (int i = i0; i < i1; ++i) {
            if (i == 0 || (skey2[i] >> 11) != (skey2[i - 1] >> 11)) {
                tot = 0;
                head = 1;
            }
            tot += (int)(pk[L.comp[i]] >> 12);
        }
        s_segv[t] = tot;
        s_segh[t] = head;
        __syncthreads();
        // inclusive segmented scan of the runs: (v, h) + (v', h') = (h' ? v' : v + v', h | h')
        for (int d = 1; d < NT; d <<= 1) {
            int pv = 0, ph = 0;
            if (t >= d) {
                pv = s_segv[t - d];
                ph = s_segh[t - d];
            }
            __syncthreads();
            if (t >= d && !s_segh[t]) {
                s_segv[t] += pv;
                s_segh[t] |= ph;
            }
            __syncthreads();
        }
        int run = t == 0 ? 0 : s_segv[t - 1];
        for (int i = i0; i < i1; ++i) {
            if (i == 0 || (skey2[i] >> 11) != (skey2[i - 1] >> 11)) run = 0;
            const int v = L.comp[i];
            S[v] = (uint32_t)run;
            run += (int)(pk[v] >> 12);
        }
    }
    __syncthreads();
    // pos(v) = sum over v and its link ancestors below the root of 1 + S
    for (int v = t; v < n; v += NT) {
        int p = 0;
        for (int x = v; x > 0; x = link[x]) p += 1 + (int)S[x];
        p = min(p, n - 1);  // a position is always < n; never write outside the graph
        out.pos[v] = p;
        out.order[p] = v;
        out.ek[p] = keyup[v];
        out.parent[v] = v ? (int)L.par[v] : -1;
        // the fill's tables: rank code of each position (1 + the rank of its
        // key among the n - 1 keys; 0 at position 0), and each code's weight
        // and flat index (code 0: the diagonal)
        const int r = v ? rankv[v] + 1 : 0;
        blk.slot[o + p] = (uint16_t)r;
        blk.dM[o + r] = v ? key_weight<WIDEST>(keyup[v]) : 0.0f;
        blk.dI[o + r] = v ? (int32_t)(uint32_t)keyup[v] : -1;
    }
}

}  // namespace appd
