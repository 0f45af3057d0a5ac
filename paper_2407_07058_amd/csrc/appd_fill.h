// The calculation-and-copy fill (arXiv 2407.07058, Section 3 and the argument
// of Section 5), restated over Prim's attachment order.
//
// Prim attaches v_0 = 0, v_1, ..., v_{n-1}; ek[k] is the key of the edge that
// attached v_k.  For a < b the minimax key of the pair (v_a, v_b) is
//     max(ek[a+1], ..., ek[b]).
// (>=: when v_b is attached... more precisely, at step c = argmax the attached
// set {v_0..v_{c-1}} holds v_a but not v_b, and ek[c] is the smallest edge
// leaving it, so every a-b path pays at least ek[c].  <=: take the last step
// t <= a whose key exceeds that maximum; no edge of weight below it leaves
// {v_0..v_{t-1}}, so v_t..v_b all hang off one another through edges no larger
// than the maximum.)  This is the removal order of Algorithm 4 read the other
// way round: the removed edge that first separates two vertices is the largest
// key between their attachment positions.  A row of M is therefore a running
// maximum over ek, outward from the row's own position, gathered back into
// column order.
//
// Columns are processed in blocks of CB original indices.  A prep kernel sorts
// each block's columns by attachment position (slots sp[0..cnt)) and stores
// gap[k] = max ek over (sp[k-1], sp[k]].  For a row at position a, with k* the
// first slot whose position is >= a:
//   slot k >= k*:  max(ek over (a, sp[k*]],  gap[k*+1..k])      (running max up)
//   slot k <  k*:  max(gap[k+1..k*-1], ek over (sp[k*-1], a])    (running max down)
// The two partial ranges next to a are read from ek directly (a wave-wide max);
// when the row's own column lies in the block (sp[k*] == a) it is the diagonal
// and both boundaries are gap entries.  One wave owns a row of one block: a
// running max within each lane's S = CB/64 consecutive slots, a cross-lane
// inclusive scan, a write into the wave's LDS row buffer, then a gather through
// slot_of_col to coalesced stores of M and idx.
#pragma once

#include "appd_device.h"
#include "appd_wcount.h"

namespace appd {

// Block prep: one workgroup (CB threads) per column block.  The block's
// positions go into a bitmap over 0..n-1 with per-word prefix counts; the slot
// of a column is the rank of its position read off them (the columns in
// position order, without a sort).  The gap maxima are taken in one sweep over
// ek: position p (sp[k-1] < p <= sp[k]) belongs to slot k = the number of the
// block's positions below p, read off the same bitmap, and is folded into
// gap[k] with an LDS atomic max.  ek is read coalesced, once per block.
// Then the block's gap keys are sorted (bitonic, u64, one per thread) and every
// slot k >= 1 gets its code for the fill: (2 * (rank of gap[k] among the
// block's gaps + 1)) << 11 | k, an order-preserving 32-bit stand-in for the
// key, together with the decoded weight and flat index of gap[k] (decode
// tables indexed by k; entry 0 is the diagonal: 0.0, -1).  The sorted gaps are
// kept so that the fill can code the two boundary keys of a row the same way.
// LDS: keys CB words; bits and prefix (n + 31) / 32 words each; gap and srt CB
// keys each.
constexpr int kCodeShift = 11;  // slot codes below 2^11 (CB + boundary entries)
constexpr uint32_t kCodeMask = (1u << kCodeShift) - 1;

template <int CB, bool WIDEST>
__device__ __forceinline__ void fill_prep_block(const int32_t* __restrict__ pos,
                                                const uint64_t* __restrict__ ek, int n, int blk,
                                                uint16_t* __restrict__ blk_sp,
                                                uint16_t* __restrict__ blk_slot,
                                                uint32_t* __restrict__ blk_code,
                                                float* __restrict__ blk_dM,
                                                int32_t* __restrict__ blk_dI,
                                                uint64_t* __restrict__ blk_sorted, uint32_t* keys,
                                                uint32_t* bits, int32_t* wpre, uint64_t* gap,
                                                uint64_t* srt) {
    static_assert(CB + 16 <= (1 << kCodeShift), "slot codes must fit");
    static_assert(CB % kWave == 0 && CB / kWave <= kWave, "one wave scans the wave totals");
    const int t = threadIdx.x;  // blockDim.x == CB: one column (and one gap) per thread
    const int lane = t & (kWave - 1), wid = t / kWave;
    const int j0 = blk * CB;
    const int cnt = min(CB, n - j0);
    const int nw = (n + 31) / 32;
    const int pm = t < cnt ? pos[j0 + t] : -1;  // this thread's column's position
    gap[t] = 0;
    for (int w = t; w < nw; w += CB) bits[w] = 0;
    __syncthreads();
    // the block's positions as a bitmap over 0..n-1
    if (pm >= 0) atomicOr(&bits[pm >> 5], 1u << (pm & 31));
    __syncthreads();
    // exclusive prefix of the word counts: each thread counts a run of words,
    // then a block scan of the run counts (shuffles within each wave, one wave
    // over the wave totals)
    const int per = (nw + CB - 1) / CB;
    const int w0 = min(nw, t * per), w1 = min(nw, w0 + per);
    int c = 0;
    for (int w = w0; w < w1; ++w) c += __popc(bits[w]);
    __shared__ int s_tot[CB / kWave];
    int incl = c;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int y = __shfl_up(incl, d);
        if (lane >= d) incl += y;
    }
    if (lane == kWave - 1) s_tot[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const int v = lane < CB / kWave ? s_tot[lane] : 0;
        int x = v;
#pragma unroll
        for (int d = 1; d < CB / kWave; d <<= 1) {
            const int y = __shfl_up(x, d);
            if (lane >= d) x += y;
        }
        if (lane < CB / kWave) s_tot[lane] = x - v;
    }
    __syncthreads();
    int run = s_tot[wid] + incl - c;
    for (int w = w0; w < w1; ++w) {
        wpre[w] = run;
        run += __popc(bits[w]);
    }
    __syncthreads();
    // slot of column c = rank of its position among the block's positions
    if (pm >= 0) {
        const int k = wpre[pm >> 5] + __popc(bits[pm >> 5] & ((1u << (pm & 31)) - 1u));
        keys[k] = ((uint32_t)pm << 16) | (uint32_t)t;
        blk_sp[j0 + k] = (uint16_t)pm;
        blk_slot[j0 + t] = (uint16_t)k;
    }
    __syncthreads();
    // one sweep over ek: position p > sp[0] lies in slot k = #{sp < p}; the
    // loads of a batch are issued before its atomics
    const int lo = (int)(keys[0] >> 16) + 1, hi = (int)(keys[cnt - 1] >> 16);
    constexpr int kSweep = 8;
    for (int p0 = lo + t; p0 <= hi; p0 += kSweep * CB) {
        uint64_t e[kSweep];
#pragma unroll
        for (int i = 0; i < kSweep; ++i) {
            const int p = p0 + i * CB;
            e[i] = p <= hi ? ek[p] : 0;
        }
#pragma unroll
        for (int i = 0; i < kSweep; ++i) {
            const int p = p0 + i * CB;
            if (p <= hi) {
                const int k = wpre[p >> 5] + __popc(bits[p >> 5] & ((1u << (p & 31)) - 1u));
                atomicMax((unsigned long long*)&gap[k], (unsigned long long)e[i]);
            }
        }
    }
    __syncthreads();
    // sorted gaps (slots 1..cnt-1), padded with the largest key: bitonic sort
    // with one key per thread (blockDim.x == CB); exchanges at strides below
    // the wave width go through shuffles, the others through LDS
    {
        uint64_t x = (t + 1 < cnt) ? gap[t + 1] : ~0ull;
        for (int size = 2; size <= CB; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                uint64_t y;
                if (stride >= kWave) {
                    srt[t] = x;
                    __syncthreads();
                    y = srt[t ^ stride];
                    __syncthreads();
                } else {
                    y = shfl_xor_u64(x, stride);
                }
                const bool up = (t & size) == 0;
                const bool lower = (t & stride) == 0;
                x = (lower == up) ? umin64(x, y) : umax64(x, y);
            }
        }
        srt[t] = x;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
        uint32_t code = 0;
        float dm = 0.0f;
        int32_t di = -1;
        if (k > 0) {
            const uint64_t key = gap[k];
            int lo = 0, hi = cnt - 1;  // rank of key among srt[0 .. cnt-2]
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (srt[mid] < key) lo = mid + 1;
                else hi = mid;
            }
            code = ((uint32_t)(2 * (lo + 1)) << kCodeShift) | (uint32_t)k;
            dm = key_weight<WIDEST>(key);
            di = (int32_t)(uint32_t)key;
        }
        blk_code[j0 + k] = code;
        blk_dM[j0 + k] = dm;
        blk_dI[j0 + k] = di;
        blk_sorted[j0 + k] = srt[k];
    }
}

// One column block, rows [r0, r1), waves of the workgroup take rows in turn.
// s_R: this wave's row buffer of CB keys.  Each lane owns the S = CB/64
// consecutive slots k0..k0+S-1 and keeps their gap keys in registers for all
// rows of the block.  Per row: the lane's running maxima within its own slots
// (upward for slots at or above k*, downward below it), a cross-lane scan of the
// lane totals, then the combined values go to s_R and are gathered in column
// order.  VEC: rows are 16-byte aligned (n % 4 == 0), so each lane writes four
// consecutive columns of M and of idx with one 16-byte store each.
// 16-byte vectors for the non-temporal stores of M and idx
typedef float f4v __attribute__((ext_vector_type(4)));
typedef int i4v __attribute__((ext_vector_type(4)));
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

template <int CB, bool WIDEST, bool VEC>
__device__ __forceinline__ void fill_rows_block(const int32_t* __restrict__ pos,
                                                const uint64_t* __restrict__ ek, int n,
                                                int j0, int cnt, int r0, int r1,
                                                const uint16_t* s_sp, const uint16_t* s_slot,
                                                const uint64_t* s_gap, uint64_t* s_R,
                                                float* __restrict__ M, int32_t* __restrict__ idx,
                                                int nwaves) {
    constexpr int S = CB / kWave;
    static_assert(S >= 1 && S <= kWave, "CB must be in [64, 4096]");
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = threadIdx.x / kWave;
    const int k0 = lane * S;
    uint64_t g[S];  // gap[k0 + q]; padding slots hold 0
#pragma unroll
    for (int q = 0; q < S; ++q) g[q] = s_gap[k0 + q];
    uint64_t gnx = shfl_down_u64(g[0], 1);  // gap[k0 + S]
    if (lane == kWave - 1) gnx = 0;
    const int sp_last = s_sp[k0 + S - 1];   // padded slots hold 0xffff

    int i = r0 + wid;
    int a_next = i < r1 ? pos[i] : 0;
    for (; i < r1; i += nwaves) {
        const int a = a_next;
        if (i + nwaves < r1) a_next = pos[i + nwaves];
        // k* = number of slots whose position is below a
        const int nbl = __popcll(__ballot(sp_last < a));
        const int base = nbl * S;
        const bool part = (lane < S) && (base + lane < CB) && (s_sp[min(base + lane, CB - 1)] < a);
        const int ks = base + __popcll(__ballot(part));
        const bool diag = ks < cnt && (int)s_sp[ks] == a;

        // keys crossed next to the row's own position
        uint64_t bl = 0, br = 0;
        if (diag) {
            bl = ks > 0 ? s_gap[ks] : 0ull;
        } else {
            const int lo = ks > 0 ? (int)s_sp[ks - 1] + 1 : a + 1;
            const int hi = ks < cnt ? (int)s_sp[ks] : a;
            for (int x = lo + lane; x <= hi; x += kWave) {
                const uint64_t e = ek[x];
                if (x <= a) bl = umax64(bl, e);
                else br = umax64(br, e);
            }
            bl = wave_max_u64(bl);
            br = wave_max_u64(br);
        }
        const uint64_t brk = diag ? 0ull : br;

        // lane-local running maxima: upward over slots >= k*, downward below
        uint64_t loc[S];
        uint64_t run = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int k = k0 + q;
            const uint64_t e = k > ks ? g[q] : (k == ks ? brk : 0ull);
            run = umax64(run, e);
            loc[q] = run;
        }
        const uint64_t up_tot = run;
        run = 0;
#pragma unroll
        for (int q = S - 1; q >= 0; --q) {
            const int k = k0 + q;
            const uint64_t nxt = q + 1 < S ? g[q + 1] : gnx;
            const uint64_t e = k < ks - 1 ? nxt : (k == ks - 1 ? bl : 0ull);
            run = umax64(run, e);
            if (k < ks) loc[q] = run;
        }
        const uint64_t dn_tot = run;
        const uint64_t up_in = wave_excl_max_up(up_tot, lane);
        const uint64_t dn_in = wave_excl_max_down(dn_tot, lane);
#pragma unroll
        for (int q = 0; q < S; ++q) {
            const int k = k0 + q;
            s_R[k] = umax64(loc[q], k >= ks ? up_in : dn_in);
        }
        wave_lds_sync();

        float* mrow = M + (size_t)i * (size_t)n + j0;
        int32_t* irow = idx + (size_t)i * (size_t)n + j0;
        if (VEC) {
            for (int c = lane * 4; c < cnt; c += kWave * 4) {
                const uint64_t sl = *(const uint64_t*)(s_slot + c);  // 4 slots
                float4 mv;
                int4 iv;
                const uint64_t k0v = s_R[sl & 0xffff], k1v = s_R[(sl >> 16) & 0xffff];
                const uint64_t k2v = s_R[(sl >> 32) & 0xffff], k3v = s_R[sl >> 48];
                mv.x = k0v ? key_weight<WIDEST>(k0v) : 0.0f;
                mv.y = k1v ? key_weight<WIDEST>(k1v) : 0.0f;
                mv.z = k2v ? key_weight<WIDEST>(k2v) : 0.0f;
                mv.w = k3v ? key_weight<WIDEST>(k3v) : 0.0f;
                iv.x = k0v ? (int32_t)(uint32_t)k0v : -1;
                iv.y = k1v ? (int32_t)(uint32_t)k1v : -1;
                iv.z = k2v ? (int32_t)(uint32_t)k2v : -1;
                iv.w = k3v ? (int32_t)(uint32_t)k3v : -1;
                *(float4*)(mrow + c) = mv;
                *(int4*)(irow + c) = iv;
                count_writes(mrow + c, 4);
                count_writes(irow + c, 4);
            }
        } else {
            auto put1 = [&](int c) {
                const uint64_t key = s_R[s_slot[c]];
                mrow[c] = key ? key_weight<WIDEST>(key) : 0.0f;
                irow[c] = key ? (int32_t)(uint32_t)key : -1;
                count_writes(mrow + c, 1);
                count_writes(irow + c, 1);
            };
            // A row may start at any 4-byte boundary (graphs packed back to
            // back).  When the M and idx rows are aligned alike: the columns
            // up to the first 16-byte boundary and the last (cnt - h) % 4 one
            // lane each, the rest four columns per 16-byte non-temporal store
            // (the batch's outputs far exceed the last-level cache: ragged
            // batch 2.47 -> 2.42 ms per replay).
            const int mis = (int)(((uintptr_t)mrow >> 2) & 3u);
            if (mis == (int)(((uintptr_t)irow >> 2) & 3u)) {
                const int h = min(cnt, (4 - mis) & 3);
                const int nq = (cnt - h) >> 2;
                const int tail0 = h + 4 * nq;
                if (lane < h) put1(lane);
                if (lane < cnt - tail0) put1(tail0 + lane);
                for (int m = lane; m < nq; m += kWave) {
                    const int c = h + 4 * m;
                    const uint64_t k0v = s_R[s_slot[c]], k1v = s_R[s_slot[c + 1]];
                    const uint64_t k2v = s_R[s_slot[c + 2]], k3v = s_R[s_slot[c + 3]];
                    const f4v mv = {k0v ? key_weight<WIDEST>(k0v) : 0.0f,
                                    k1v ? key_weight<WIDEST>(k1v) : 0.0f,
                                    k2v ? key_weight<WIDEST>(k2v) : 0.0f,
                                    k3v ? key_weight<WIDEST>(k3v) : 0.0f};
                    const i4v iv = {k0v ? (int32_t)(uint32_t)k0v : -1,
                                    k1v ? (int32_t)(uint32_t)k1v : -1,
                                    k2v ? (int32_t)(uint32_t)k2v : -1,
                                    k3v ? (int32_t)(uint32_t)k3v : -1};
                    __builtin_nontemporal_store(mv, (f4v*)(mrow + c));
                    __builtin_nontemporal_store(iv, (i4v*)(irow + c));
                    count_writes(mrow + c, 4);
                    count_writes(irow + c, 4);
                }
            } else {
                for (int c = lane; c < cnt; c += kWave) put1(c);
            }
        }
        wave_lds_sync();
    }
}

// The same fill on 32-bit slot codes (fill_prep_block): the running maxima
// are taken over codes, which order like the keys, and each output is decoded
// through the block's tables in LDS.  The two boundary keys of a row (not gap
// values) are coded between the gaps by their rank among the sorted gaps
// (a two-step ballot search), with per-wave decode entries at CB + 2 * wave
// (left) and CB + 2 * wave + 1 (right).  A wave locates its next row and
// issues that row's ek loads before it fills the current one.  M and idx are
// written with non-temporal stores: n^2 outputs are far larger than the
// last-level cache, and lines left dirty there would be written back during
// whatever runs next (the following pass over W).  s_R: this wave's row
// buffer, the slot part (low kCodeShift bits) of each column's code, which is
// all the decode reads; s_dM / s_dI: CB + 2 * nwaves entries.
// EXACT (short blocks, the batched fill): the lanes past a short block's
// columns issue no stores; otherwise every lane issues CB / 256 of them (those
// past the block are dropped by the buffer range), so that the count of memory
// operations per row is fixed.
template <int CB, bool WIDEST, bool VEC, bool EXACT = false>
__device__ __forceinline__ void fill_rows_block_coded(
    const int32_t* __restrict__ pos, const uint64_t* __restrict__ ek, int n, int j0, int cnt,
    int r0, int r1, const uint16_t* s_sp, const uint16_t* s_slot,
    const uint32_t* __restrict__ code, const uint64_t* s_sorted, float* s_dM, int32_t* s_dI,
    uint16_t* s_R, float* __restrict__ M,
    int32_t* __restrict__ idx, int nwaves) {
    constexpr int S = CB / kWave;
    static_assert(S >= 1 && S <= kWave, "CB must be in [64, 4096]");
    const int lane = threadIdx.x & (kWave - 1);
    // wave-uniform, so the per-row position loads are scalar loads
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int k0 = lane * S;
    static_assert(S == 16, "the slots of one lane spread over one 16-lane DPP row");
    // Row-independent running maxima of this lane's slot codes (the block's
    // code[0 .. cnt), padding slots 0): pre[q] = max code[k0 .. k0+q] (going up
    // from below the lane), suf[q] = max code[k0+q+1 .. k0+S] (going down from
    // above it).
    uint32_t pre[S], suf[S];
    {
        uint32_t g[S];
#pragma unroll
        for (int q = 0; q < S; ++q) g[q] = k0 + q < cnt ? code[k0 + q] : 0u;
        uint32_t run = __shfl_down(g[0], 1);  // code of slot k0 + S
        if (lane == kWave - 1) run = 0;
#pragma unroll
        for (int q = S - 1; q >= 0; --q) {
            suf[q] = run;
            run = max(run, g[q]);
        }
        run = 0;
#pragma unroll
        for (int q = 0; q < S; ++q) {
            run = max(run, g[q]);
            pre[q] = run;
        }
    }
    const int sp_last = s_sp[k0 + S - 1];  // padded slots hold 0xffff
    const uint32_t cl = (uint32_t)(CB + 2 * wid), cr = cl + 1;
    // Where a row's position a sits among the block's slots, and this lane's
    // ek values of the positions between the two slots around it.
    struct RowAt {
        int a, ks, lo, hi, diag;
        uint64_t e0, e1;
        uint32_t c;  // lanes 0..15: code of slot S su + j; 16..31: of slot S sd + j + 1
    };
    // su = lane holding slot ks (kWave: none), sd = lane holding slot ks - 1 (-1: none)
    auto lanes_around = [&](int ks, int& su, int& sd) {
        su = ks / S;
        sd = (ks + S - 1) / S - 1;
    };
    // Every load and store of a row is issued unconditionally (indices
    // clamped), so the number of memory operations between a prefetch and its
    // use is fixed and the wait for it leaves the stores of the row before in
    // flight; loads for the next row are issued before the current one is
    // filled.
    auto locate = [&](int a) {
        RowAt r;
        r.a = a;
        // ks = number of slots whose position is below a
        const int nbl = __popcll(__ballot(sp_last < a));
        const int base = nbl * S;
        const bool part = (lane < S) && (base + lane < CB) && (s_sp[min(base + lane, CB - 1)] < a);
        r.ks = base + __popcll(__ballot(part));
        r.diag = r.ks < cnt && (int)s_sp[r.ks] == a;
        r.lo = r.ks > 0 ? (int)s_sp[r.ks - 1] + 1 : a + 1;
        r.hi = r.ks < cnt ? (int)s_sp[r.ks] : a;  // a valid position even when lo > hi
        r.e0 = ek[min(r.lo + lane, r.hi)];
        r.e1 = ek[min(r.lo + kWave + lane, r.hi)];
        int su, sd;
        lanes_around(r.ks, su, sd);
        const int j = lane & 15;
        const int ci = lane < 16 ? su * S + j : (lane < 32 ? sd * S + j + 1 : 0);
        r.c = code[min(max(ci, 0), cnt - 1)];  // used only where ci < cnt
        return r;
    };
    // Rank of a boundary key among the sorted gaps in two steps: lane l probes
    // gap S l + S - 1 (the last one of its S-run; entries from cnt - 1 on hold
    // ~0, above every key), so the keys below a probe count whole runs; then
    // one run of S entries is compared for each key at once (lanes 0..S-1 for
    // the left key, 32..32+S-1 for the right one).
    static_assert(S <= 32, "one run per half-wave");
    const uint64_t probe = s_sorted[k0 + S - 1];
    constexpr uint64_t kRunMask = S == 32 ? 0xffffffffull : ((1ull << S) - 1);

    auto fill_row = [&](const RowAt& cur, int i) {
        const int a = cur.a, ks = cur.ks;
        // codes of the keys crossed next to the row's own position
        uint32_t bl = 0, br = 0;
        if (cur.diag) {
            // the code of slot ks (< cnt), held by lane ks % S
            bl = ks > 0 ? (uint32_t)__builtin_amdgcn_readlane((int)cur.c, ks % S) : 0u;
        } else {
            uint64_t kl = 0, kr = 0;
            {
                const int x0 = cur.lo + lane, x1 = x0 + kWave;
                const uint64_t e0 = x0 <= cur.hi ? cur.e0 : 0ull;
                const uint64_t e1 = x1 <= cur.hi ? cur.e1 : 0ull;
                kl = umax64(x0 <= a ? e0 : 0ull, x1 <= a ? e1 : 0ull);
                kr = umax64(x0 > a ? e0 : 0ull, x1 > a ? e1 : 0ull);
            }
            for (int x = cur.lo + 2 * kWave + lane; x <= cur.hi; x += kWave) {  // long gaps
                const uint64_t e = ek[x];
                if (x <= a) kl = umax64(kl, e);
                else kr = umax64(kr, e);
            }
            kl = wave_max_u64(kl);
            kr = wave_max_u64(kr);
            const int bL = min(__popcll(__ballot(probe < kl)), CB / S - 1);
            const int bR = min(__popcll(__ballot(probe < kr)), CB / S - 1);
            const int j = lane & 31;
            const bool rgt = lane >= 32;
            const uint64_t sv = s_sorted[(rgt ? bR : bL) * S + (j < S ? j : 0)];
            const uint64_t m = __ballot(j < S && sv < (rgt ? kr : kl));
            const int loL = bL * S + __popcll(m & kRunMask);
            const int loR = bR * S + __popcll((m >> 32) & kRunMask);
            if (kl) bl = ((uint32_t)(2 * loL + 1) << kCodeShift) | cl;
            if (kr) br = ((uint32_t)(2 * loR + 1) << kCodeShift) | cr;
            if (lane == 0) {
                s_dM[cl] = kl ? key_weight<WIDEST>(kl) : 0.0f;
                s_dI[cl] = kl ? (int32_t)(uint32_t)kl : -1;
                s_dM[cr] = kr ? key_weight<WIDEST>(kr) : 0.0f;
                s_dI[cr] = kr ? (int32_t)(uint32_t)kr : -1;
            }
        }

        // R[k] = max code crossed from the row's position to slot k: upward
        // (k >= ks) br then code[ks+1 .. k], downward (k < ks) bl then
        // code[k+1 .. ks-1].  Lanes wholly above su or below sd take their
        // slots from pre / suf and the maxima of the lanes between them and
        // ks; the slots of su and sd go one per lane to lanes 0..15 and 16..31
        // and are scanned there (inclusive, up resp. down the 16-lane row).
        int su, sd;
        lanes_around(ks, su, sd);
        const int j = lane & 15;
        uint32_t e = 0;
        if (lane < 16) {
            const int k = su * S + j;
            e = k > ks ? (k < cnt ? cur.c : 0u) : (k == ks ? br : 0u);
        } else if (lane < 32) {
            const int k = sd * S + j;
            e = k < ks - 1 ? cur.c : (k == ks - 1 ? bl : 0u);
        }
        uint32_t xu = e, xd = e;
        xu = max(xu, dpp_u32<0x111>(xu, 0));  // row_shr:1
        xu = max(xu, dpp_u32<0x112>(xu, 0));
        xu = max(xu, dpp_u32<0x114>(xu, 0));
        xu = max(xu, dpp_u32<0x118>(xu, 0));
        xd = max(xd, dpp_u32<0x101>(xd, 0));  // row_shl:1
        xd = max(xd, dpp_u32<0x102>(xd, 0));
        xd = max(xd, dpp_u32<0x104>(xd, 0));
        xd = max(xd, dpp_u32<0x108>(xd, 0));
        const uint32_t up_s = (uint32_t)__builtin_amdgcn_readlane((int)xu, 15);
        const uint32_t dn_s = (uint32_t)__builtin_amdgcn_readlane((int)xd, 16);
        const uint32_t up_in =
            wave_excl_max_up_u32(lane > su ? pre[S - 1] : (lane == su ? up_s : 0u), lane);
        const uint32_t dn_in =
            wave_excl_max_down_u32(lane < sd ? suf[0] : (lane == sd ? dn_s : 0u), lane);
        const bool above = lane > su;
        if (above || lane < sd) {
            const uint32_t in = above ? up_in : dn_in;
#pragma unroll
            for (int q = 0; q < S; ++q)
                s_R[k0 + q] = (uint16_t)(max(above ? pre[q] : suf[q], in) & kCodeMask);
        }
        if (lane < 16 && su < kWave && su * S + j >= ks) s_R[su * S + j] = (uint16_t)(xu & kCodeMask);
        if (lane >= 16 && lane < 32 && sd >= 0 && sd * S + j < ks)
            s_R[sd * S + j] = (uint16_t)(xd & kCodeMask);
        wave_lds_sync();

        float* mrow = M + (size_t)i * (size_t)n + j0;
        int32_t* irow = idx + (size_t)i * (size_t)n + j0;
        if (VEC) {
            // cnt is a multiple of 4.  Buffer stores over the block's columns:
            // in a short block the lanes past cnt read the last four columns'
            // entries and their stores fall outside the range and are dropped,
            // so every lane issues the same stores and each column is written
            // once.
            const __amdgpu_buffer_rsrc_t rm =
                __builtin_amdgcn_make_buffer_rsrc(mrow, (short)0, cnt * 4, kBufferRsrcWord3);
            const __amdgpu_buffer_rsrc_t ri =
                __builtin_amdgcn_make_buffer_rsrc(irow, (short)0, cnt * 4, kBufferRsrcWord3);
#pragma unroll
            for (int it = 0; it < CB / (4 * kWave); ++it) {
                if (EXACT && lane * 4 + it * 4 * kWave >= cnt) break;
                const int cs = lane * 4 + it * 4 * kWave;  // the columns stored
                const int c = min(cs, cnt - 4);           // the entries read
                const uint64_t sl = *(const uint64_t*)(s_slot + c);  // 4 slots
                const uint32_t c0 = s_R[sl & 0xffff] & kCodeMask;
                const uint32_t c1 = s_R[(sl >> 16) & 0xffff] & kCodeMask;
                const uint32_t c2 = s_R[(sl >> 32) & 0xffff] & kCodeMask;
                const uint32_t c3 = s_R[sl >> 48] & kCodeMask;
                const f4v mv = {s_dM[c0], s_dM[c1], s_dM[c2], s_dM[c3]};
                const i4v iv = {s_dI[c0], s_dI[c1], s_dI[c2], s_dI[c3]};
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, mv), rm, cs * 4, 0,
                                                       kBufferNontemporal);
                __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4v, iv), ri, cs * 4, 0,
                                                       kBufferNontemporal);
                if (cs < cnt) {
                    count_writes(mrow + cs, 4);
                    count_writes(irow + cs, 4);
                }
            }
        } else {
            auto put1 = [&](int c) {
                const uint32_t cd = s_R[s_slot[c]] & kCodeMask;
                __builtin_nontemporal_store(s_dM[cd], mrow + c);
                __builtin_nontemporal_store(s_dI[cd], irow + c);
                count_writes(mrow + c, 1);
                count_writes(irow + c, 1);
            };
            // A row may start at any 4-byte boundary (n % 4 != 0, or graphs
            // packed back to back).  When the M and idx rows are misaligned
            // alike: the columns up to the first 16-byte boundary and the last
            // (cnt - h) % 4 one lane each, the rest four per 16-byte store.
            const int mis = (int)(((uintptr_t)mrow >> 2) & 3u);
            if (mis == (int)(((uintptr_t)irow >> 2) & 3u)) {
                const int h = min(cnt, (4 - mis) & 3);
                const int nq = (cnt - h) >> 2;
                const int tail0 = h + 4 * nq;
                if (lane < h) put1(lane);
                if (lane < cnt - tail0) put1(tail0 + lane);
                for (int m = lane; m < nq; m += kWave) {
                    const int c = h + 4 * m;
                    const uint32_t c0 = s_R[s_slot[c]] & kCodeMask;
                    const uint32_t c1 = s_R[s_slot[c + 1]] & kCodeMask;
                    const uint32_t c2 = s_R[s_slot[c + 2]] & kCodeMask;
                    const uint32_t c3 = s_R[s_slot[c + 3]] & kCodeMask;
                    const f4v mv = {s_dM[c0], s_dM[c1], s_dM[c2], s_dM[c3]};
                    const i4v iv = {s_dI[c0], s_dI[c1], s_dI[c2], s_dI[c3]};
                    __builtin_nontemporal_store(mv, (f4v*)(mrow + c));
                    __builtin_nontemporal_store(iv, (i4v*)(irow + c));
                    count_writes(mrow + c, 4);
                    count_writes(irow + c, 4);
                }
            } else {
                for (int c = lane; c < cnt; c += kWave) put1(c);
            }
        }
        wave_lds_sync();
    };

    // rows r0 + wid, + nwaves, ...: two row states in turn (no register holding
    // a load in flight is copied).  The first row is peeled so that every
    // path into the loop has issued the same loads and stores.
    int i = r0 + wid;
    if (i >= r1) return;
    const int last = r1 - 1;
    RowAt A = locate(pos[i]), B;
    int pa = pos[min(i + nwaves, last)], pb;
    pb = pos[min(i + 2 * nwaves, last)];
    B = locate(pa);
    asm volatile("" ::: "memory");  // issue the next row's loads before these stores
    fill_row(A, i);
    for (i += nwaves; i < r1;) {
        pa = pos[min(i + 2 * nwaves, last)];
        A = locate(pb);
        asm volatile("" ::: "memory");
        fill_row(B, i);
        i += nwaves;
        if (i >= r1) break;
        pb = pos[min(i + 2 * nwaves, last)];
        B = locate(pa);
        asm volatile("" ::: "memory");
        fill_row(A, i);
        i += nwaves;
    }
}

}  // namespace appd
