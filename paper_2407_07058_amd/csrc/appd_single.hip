// Single-graph APPD: persistent Prim kernel, column-block prep, row fill.
#include "appd_fill.h"
#include "appd_internal.h"
#include "appd_prim.h"
#include "appd.h"

namespace appd {

constexpr int kPrimThreads = 1024;
constexpr int kFillCB = 1024;
constexpr int kFillThreads = 256;
constexpr int kPrepThreads = 1024;  // one workgroup per column block: sorts and sweeps
constexpr int kFillRowsPerWG = 16;

template <int CH, bool WIDEST>
__global__ __launch_bounds__(kPrimThreads) void prim_single_kernel(const float* __restrict__ W,
                                                                   int n, PrimOut out) {
    __shared__ uint64_t red_key[2 * (kPrimThreads / kWave)];
    __shared__ int32_t red_v[2 * (kPrimThreads / kWave)];
    extern __shared__ uint16_t s_parents[];  // prim_parents_in_lds<CH>(): kPrimThreads * CH
    prim_run<kPrimThreads, CH, WIDEST>(W, n, out, red_key, red_v, s_parents);
}

template <int CB, bool WIDEST>
__global__ __launch_bounds__(kPrepThreads) void fill_prep_kernel(const int32_t* __restrict__ pos,
                                                                 const uint64_t* __restrict__ ek,
                                                                 int n, SingleWs w) {
    static_assert(kPrepThreads == CB, "the gap sort keeps one key per thread");
    __shared__ uint32_t keys[CB];
    __shared__ uint32_t bits[(APPD_MAX_N + 31) / 32];
    __shared__ int32_t wpre[(APPD_MAX_N + 31) / 32];
    __shared__ uint64_t gap[CB];
    __shared__ uint64_t srt[CB];
    fill_prep_block<CB, WIDEST>(pos, ek, n, blockIdx.x, w.blk_sp, w.blk_slot, w.blk_code, w.blk_dM,
                                w.blk_dI, w.blk_sorted, keys, bits, wpre, gap, srt);
}

template <int CB, bool WIDEST, bool VEC>
__global__ __launch_bounds__(kFillThreads) void fill_kernel(const int32_t* __restrict__ pos,
                                                            const uint64_t* __restrict__ ek, int n,
                                                            SingleWs w, float* __restrict__ M,
                                                            int32_t* __restrict__ idx,
                                                            int rows_per_wg) {
    constexpr int NWV = kFillThreads / kWave;
    __shared__ uint16_t s_sp[CB];
    __shared__ __align__(16) uint16_t s_slot[CB];
    __shared__ uint64_t s_sorted[CB];
    __shared__ float s_dM[CB + 2 * NWV];
    __shared__ int32_t s_dI[CB + 2 * NWV];
    __shared__ uint16_t s_R[NWV][CB];  // slot part of each column's code
    const int j0 = blockIdx.x * CB;
    const int cnt = min(CB, n - j0);
    for (int k = threadIdx.x; k < CB; k += kFillThreads) {
        const bool in = k < cnt;
        s_sp[k] = in ? w.blk_sp[j0 + k] : (uint16_t)0xffff;
        s_slot[k] = in ? w.blk_slot[j0 + k] : (uint16_t)0;
        s_sorted[k] = in ? w.blk_sorted[j0 + k] : ~0ull;
        s_dM[k] = in ? w.blk_dM[j0 + k] : 0.0f;
        s_dI[k] = in ? w.blk_dI[j0 + k] : -1;
    }
    __syncthreads();
    const int r0 = blockIdx.y * rows_per_wg;
    const int r1 = min(n, r0 + rows_per_wg);
    fill_rows_block_coded<CB, WIDEST, VEC>(pos, ek, n, j0, cnt, r0, r1, s_sp, s_slot,
                                           w.blk_code + j0, s_sorted, s_dM, s_dI,
                                           s_R[threadIdx.x / kWave], M, idx, NWV);
}

// ---------------------------------------------------------------- launchers
template <bool WIDEST>
static hipError_t launch_prim(const float* W, int n, PrimOut out, hipStream_t s) {
    const int ch = (n + kPrimThreads - 1) / kPrimThreads;
#define APPD_PRIM_CASE(C)                                                                    \
    if (ch <= C) {                                                                           \
        const size_t lds = prim_parents_in_lds<C>() ? (size_t)2 * kPrimThreads * C : 0;     \
        if (lds > 0) {                                                                       \
            const hipError_t e = hipFuncSetAttribute(                                        \
                (const void*)prim_single_kernel<C, WIDEST>,                                  \
                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                       \
            if (e != hipSuccess) return e;                                                   \
        }                                                                                    \
        APPD_LAUNCH("prim_single_kernel", s,                                                 \
                    prim_single_kernel<C, WIDEST><<<1, kPrimThreads, lds, s>>>(W, n, out));  \
        return hipGetLastError();                                                            \
    }
    APPD_PRIM_CASE(1)
    APPD_PRIM_CASE(2)
    APPD_PRIM_CASE(4)
    APPD_PRIM_CASE(8)
    APPD_PRIM_CASE(16)
    APPD_PRIM_CASE(24)
    APPD_PRIM_CASE(32)
    APPD_PRIM_CASE(46)
#undef APPD_PRIM_CASE
    return hipErrorInvalidValue;
}

int fill_blocks(int n) { return (n + kFillCB - 1) / kFillCB; }

size_t single_workspace_bytes(int n) {
    const size_t nb = (size_t)fill_blocks(n) * kFillCB;
    size_t off = 0;
    off = align_up(off + 4 * (size_t)n);  // order
    off = align_up(off + 4 * (size_t)n);  // parent
    off = align_up(off + 4 * (size_t)n);  // pos
    off = align_up(off + 8 * (size_t)n);  // ek
    off = align_up(off + 2 * nb);         // blk_sp
    off = align_up(off + 2 * nb);         // blk_slot
    off = align_up(off + 4 * nb);         // blk_code
    off = align_up(off + 4 * nb);         // blk_dM
    off = align_up(off + 4 * nb);         // blk_dI
    off = align_up(off + 8 * nb);         // blk_sorted
    off = align_up(off + tree_workspace_bytes(n));
    return off;
}

SingleWs carve_single(void* ws, int n) {
    const size_t nb = (size_t)fill_blocks(n) * kFillCB;
    const uintptr_t b = (uintptr_t)ws;  // null when only the size is wanted
    SingleWs w;
    size_t off = 0;
    w.order = (int32_t*)(b + off);
    off = align_up(off + 4 * (size_t)n);
    w.parent = (int32_t*)(b + off);
    off = align_up(off + 4 * (size_t)n);
    w.pos = (int32_t*)(b + off);
    off = align_up(off + 4 * (size_t)n);
    w.ek = (uint64_t*)(b + off);
    off = align_up(off + 8 * (size_t)n);
    w.blk_sp = (uint16_t*)(b + off);
    off = align_up(off + 2 * nb);
    w.blk_slot = (uint16_t*)(b + off);
    off = align_up(off + 2 * nb);
    w.blk_code = (uint32_t*)(b + off);
    off = align_up(off + 4 * nb);
    w.blk_dM = (float*)(b + off);
    off = align_up(off + 4 * nb);
    w.blk_dI = (int32_t*)(b + off);
    off = align_up(off + 4 * nb);
    w.blk_sorted = (uint64_t*)(b + off);
    off = align_up(off + 8 * nb);
    w.tree_ws = (void*)(b + off);
    return w;
}

// below this size Prim's sequential chain is short enough
constexpr int kParallelTreeMinN = 512;
int parallel_tree_min_n() { return kParallelTreeMinN; }

bool valid_mode(int mode) {
    if (mode & ~(0x31 | APPD_TREE_ONE_PASS)) return false;
    return (mode & 0x30) != 0x30;
}

template <bool WIDEST>
static hipError_t run_fill_t(int n, float* M, int32_t* idx, const SingleWs& w, hipStream_t s) {
    const int nb = fill_blocks(n);
    APPD_LAUNCH("fill_prep_kernel", s,
        fill_prep_kernel<kFillCB, WIDEST><<<nb, kPrepThreads, 0, s>>>(w.pos, w.ek, n, w));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid(nb, (n + kFillRowsPerWG - 1) / kFillRowsPerWG);
    const bool vec = (n % 4 == 0) && (((uintptr_t)M | (uintptr_t)idx) & 15u) == 0;
    if (vec)
        APPD_LAUNCH("fill_kernel", s,
            fill_kernel<kFillCB, WIDEST, true><<<grid, kFillThreads, 0, s>>>(w.pos, w.ek, n, w, M,
                idx, kFillRowsPerWG));
    else
        APPD_LAUNCH("fill_kernel", s,
            fill_kernel<kFillCB, WIDEST, false><<<grid, kFillThreads, 0, s>>>(w.pos, w.ek, n, w, M,
                idx, kFillRowsPerWG));
    return hipGetLastError();
}

hipError_t run_tree(const float* W, int n, int mode, const SingleWs& w, hipStream_t s) {
    PrimOut out{w.order, w.ek, w.pos, w.parent};
    const int algo = mode & 0x30;
    const bool parallel =
        algo == APPD_TREE_BORUVKA || (algo == APPD_TREE_AUTO && n >= kParallelTreeMinN);
    if (parallel) return run_tree_parallel(W, n, mode, out, w.tree_ws, s);
    return (mode & 1) ? launch_prim<true>(W, n, out, s) : launch_prim<false>(W, n, out, s);
}

hipError_t run_fill(int n, int mode, float* M, int32_t* idx, const SingleWs& w, hipStream_t s) {
    return (mode & 1) ? run_fill_t<true>(n, M, idx, w, s) : run_fill_t<false>(n, M, idx, w, s);
}

hipError_t run_single(const float* W, int n, int mode, float* M, int32_t* idx,
                      const SingleWs& w, hipStream_t s) {
    hipError_t e = run_tree(W, n, mode, w, s);
    if (e != hipSuccess) return e;
    return run_fill(n, mode, M, idx, w, s);
}

// This unit's copy of the write-count switch (appd_wcount.h).
hipError_t set_write_count_single(const WriteCount& wc, hipStream_t s) {
    return hipMemcpyToSymbolAsync(HIP_SYMBOL(c_write_count), &wc, sizeof wc, 0,
                                  hipMemcpyHostToDevice, s);
}

}  // namespace appd
