// Points -> complete graph, and the backward pass of the APPD selection.
//
// pairwise: W_ij = sqrt(sum_{t < d} (x_it - x_jt)^2), the sum taken in
//   increasing t with every subtraction, product, sum and the square root
//   rounded once (no contraction), so W is bit-symmetric and reproducible.
//   (Section 1: a dataset is turned into a complete graph; the paper does not
//   name the metric, Euclidean is the reading taken here.)  64 x 64 output tiles,
//   one workgroup each, the two point blocks staged in LDS.
//
// backward: with L = sum_{i != j} G_ij M_ij and M_ij the weight of the
//   bottleneck edge idx(i,j), dL/dw(e) = sum of G_ij over the pairs whose
//   bottleneck is e.  An edge (u,v) of the rooted spanning tree is stored at the
//   slot of its child endpoint (parent[child] == other end).  Each workgroup
//   accumulates a block of rows into an LDS histogram over the slots, then adds
//   its non-zero bins to the global per-edge sums.  The chain rule through
//   w = ||x_c - x_p|| then moves g * (x_c - x_p) / w to x_c and its negative to
//   x_p.  Float atomics make the summation order vary between runs.
#include "appd_device.h"
#include "appd_internal.h"

// Every product and sum below is rounded on its own (no fused multiply-add).
#pragma clang fp contract(off)

namespace appd {

constexpr int kTile = 64;
constexpr int kPairThreads = 256;
constexpr int kMaxD = 64;

// Locate work item b in a per-graph prefix table (last gi with start[gi] <= b).
__device__ __forceinline__ int find_item(const int32_t* __restrict__ start, int count, int b) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Correctly rounded float square root of x >= 0.  A hardware estimate s is
// moved to its neighbour while sqrt(x) lies beyond the midpoint between them:
// a midpoint of two adjacent floats has at most 25 significant bits, so its
// square is exact in double and the comparison with x is exact.  (No tie is
// possible: the square of such a midpoint needs more than 24 bits.)  Subnormal
// inputs are scaled by 2^24 first (exact), the root then by 2^-12 (exact).
__device__ __forceinline__ float sqrt_rn_exact(float x) {
    if (!(x > 0.0f) || x == __builtin_inff()) return x == 0.0f ? 0.0f : __builtin_sqrtf(x);
    const bool sub = x < 1.17549435e-38f;
    if (sub) x *= 16777216.0f;
    float s = __builtin_sqrtf(x);
    const double xd = (double)x;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const float up = __uint_as_float(__float_as_uint(s) + 1u);
        const double mu = ((double)s + (double)up) * 0.5;
        if (mu * mu < xd) {
            s = up;
            continue;
        }
        const float dn = __uint_as_float(__float_as_uint(s) - 1u);
        const double md = ((double)s + (double)dn) * 0.5;
        if (md * md > xd) s = dn;
    }
    return sub ? s * 2.44140625e-4f : s;
}

// Tile pair (bi, bj), bi <= bj, of the b-th upper-triangle tile in row-major
// order over an nt x nt tile grid (row bi holds nt - bi tiles).
__device__ __forceinline__ void upper_tile(int b, int nt, int* bi, int* bj) {
    const double tt = 2.0 * nt + 1.0;
    int i = (int)((tt - sqrt(tt * tt - 8.0 * (double)b)) * 0.5);
    i = i < 0 ? 0 : (i > nt - 1 ? nt - 1 : i);
    auto start = [&](int r) { return (int64_t)r * nt - (int64_t)r * (r - 1) / 2; };
    while (i > 0 && start(i) > b) --i;
    while (i < nt - 1 && start(i + 1) <= b) ++i;
    *bi = i;
    *bj = i + (int)(b - start(i));
}

// One workgroup per upper-triangle tile pair (ti <= tj): the 64 x 64 block of
// W at rows ti, columns tj is computed once and written there and, through an
// LDS transpose, at rows tj, columns ti (W is bit-symmetric: the differences of
// the mirrored pair are negations, their squares equal).  LDS (sized for d,
// pairwise_lds_bytes): the row block's points, 64 x (d + 1), later the 64 x 65
// transpose tile in the same place; then the column block's points
// transposed, d x 65.
constexpr int kPairTileWords = kTile * (kTile + 1);
static_assert(kMaxD <= kTile, "a 64 x (d + 1) point block fits the transpose tile");

inline size_t pairwise_lds_bytes(int d) { return 4 * ((size_t)kPairTileWords + (size_t)d * (kTile + 1)); }

__global__ __launch_bounds__(kPairThreads) void pairwise_kernel(
    const float* __restrict__ X, const int64_t* __restrict__ xoff,
    const int64_t* __restrict__ offsets, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ tile_start, int num_graphs, int d, float* __restrict__ W) {
    extern __shared__ float s_pair[];
    float* xs = s_pair;                    // xi[r][t] = xs[r * (d + 1) + t]; tile[r][c] = xs[r * 65 + c]
    float* xt = s_pair + kPairTileWords;   // xjT[t][c] = xt[t * 65 + c]
    const int dp = d + 1;
    const int g = find_item(tile_start, num_graphs, blockIdx.x);
    const int n = ns[g];
    const int nt = (n + kTile - 1) / kTile;
    const int tile = blockIdx.x - tile_start[g];
    int ti, tj;
    upper_tile(tile, nt, &ti, &tj);
    const float* Xg = X + xoff[g];
    float* Wg = W + offsets[g];
    const int i0 = ti * kTile, j0 = tj * kTile;
    for (int e = threadIdx.x; e < kTile * d; e += kPairThreads) {
        const int r = e / d, t = e % d;
        xs[r * dp + t] = (i0 + r < n) ? Xg[(size_t)(i0 + r) * d + t] : 0.0f;
        xt[t * (kTile + 1) + r] = (j0 + r < n) ? Xg[(size_t)(j0 + r) * d + t] : 0.0f;
    }
    __syncthreads();
    const int c = threadIdx.x & (kTile - 1);
    const int j = j0 + c;
    constexpr int RS = kPairThreads / kTile;  // row step
    float vals[kTile / RS];
#pragma unroll
    for (int k = 0; k < kTile / RS; ++k) {
        const int r = threadIdx.x / kTile + RS * k;
        const int i = i0 + r;
        vals[k] = 0.0f;
        if (i >= n || j >= n) continue;
        float acc = 0.0f;
        for (int t = 0; t < d; ++t) {
            const float df = __fsub_rn(xs[r * dp + t], xt[t * (kTile + 1) + c]);
            acc = __fadd_rn(acc, __fmul_rn(df, df));
        }
        vals[k] = (i == j) ? 0.0f : sqrt_rn_exact(acc);
        Wg[(size_t)i * n + j] = vals[k];
    }
    if (ti == tj) return;  // workgroup-uniform: a diagonal block is its own mirror
    __syncthreads();       // the point block is read no more: it becomes the transpose tile
#pragma unroll
    for (int k = 0; k < kTile / RS; ++k) xs[(threadIdx.x / kTile + RS * k) * (kTile + 1) + c] = vals[k];
    __syncthreads();
    const int ic = i0 + c;  // column of the mirrored block
#pragma unroll
    for (int k = 0; k < kTile / RS; ++k) {
        const int jr = threadIdx.x / kTile + RS * k;  // row of the mirrored block
        if (j0 + jr < n && ic < n) Wg[(size_t)(j0 + jr) * n + ic] = xs[c * (kTile + 1) + jr];
    }
}

// Columns per lane and block of a row in edge_grad_kernel, and the largest n
// whose parents are staged in LDS beside the histogram.
constexpr int kGradCols = 8;
constexpr int kGradParLds = 8192;

// Slot of the tree edge with flat index f = u*n + v (u < v, f < n*n): u and v
// by a float quotient, off by at most one for n < 2^22 (the product's
// relative error is below 2^-22 and f/n < n), then corrected.
__device__ __forceinline__ int edge_slot(uint32_t f, int n, float rcp_n,
                                         const int32_t* __restrict__ parent) {
    int u = (int)((float)f * rcp_n);
    int v = (int)f - u * n;
    if (v < 0) { --u; v += n; }
    else if (v >= n) { ++u; v -= n; }
    return parent[v] == u ? v : u;
}

// One workgroup: rows [r0, r1) of one graph, one wave per row at a time; LDS:
// the n-float histogram over the slots, then (PAR_LDS) the graph's parents.
// A wave reads a block of kGradCols * 64 columns of its row with every idx
// and G load issued before the first is used (buffer loads over the row: a
// row of a packed graph starts at any 4-byte boundary), then adds each entry
// to its slot's bin.
template <bool PAR_LDS>
__global__ __launch_bounds__(256) void edge_grad_kernel(
    const float* __restrict__ G, const int32_t* __restrict__ idx,
    const int64_t* __restrict__ offsets, const int64_t* __restrict__ noff,
    const int32_t* __restrict__ ns, const int32_t* __restrict__ parent,
    const int32_t* __restrict__ chunk_start, int num_graphs, int rows_per_wg,
    float* __restrict__ gedge) {
    extern __shared__ float hist[];
    const int g = find_item(chunk_start, num_graphs, blockIdx.x);
    const int n = ns[g];
    const int chunk = blockIdx.x - chunk_start[g];
    const float* Gg = G + offsets[g];
    const int32_t* Ig = idx + offsets[g];
    const int32_t* gpar = parent + noff[g];
    int32_t* spar = reinterpret_cast<int32_t*>(hist + n);
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        hist[k] = 0.0f;
        if (PAR_LDS) spar[k] = gpar[k];
    }
    __syncthreads();
    const int32_t* par = PAR_LDS ? spar : gpar;
    const float rcp_n = 1.0f / (float)n;
    const uint32_t nn = (uint32_t)n * (uint32_t)n;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int r0 = chunk * rows_per_wg, r1 = min(n, r0 + rows_per_wg);
    for (int r = r0 + wave; r < r1; r += blockDim.x / kWave) {
        // Most of a row's pairs share one bottleneck, nearly always the edge
        // of the row's own vertex, of its parent or of its grandparent (slots
        // r, parent[r], parent[parent[r]]): those three are summed in
        // registers, so that the bins' atomics see few lanes on one address.
        const int sa = r, sb = par[r], sc = sb >= 0 ? par[sb] : -1;
        float acc_a = 0.0f, acc_b = 0.0f, acc_c = 0.0f;
        const __amdgpu_buffer_rsrc_t ri = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<int32_t*>(Ig + (size_t)r * n), (short)0, n * 4, kBufferRsrcWord3);
        const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<float*>(Gg + (size_t)r * n), (short)0, n * 4, kBufferRsrcWord3);
        for (int c0 = 0; c0 < n; c0 += kGradCols * kWave) {
            uint32_t f[kGradCols];
            float gv[kGradCols];
#pragma unroll
            for (int e = 0; e < kGradCols; ++e) {
                const int off = (c0 + e * kWave + lane) * 4;
                f[e] = (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(ri, off, 0, 0);
                gv[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, off, 0, 0));
            }
#pragma unroll
            for (int e = 0; e < kGradCols; ++e) {
                // columns past the row, the diagonal (-1) and anything that is
                // not a flat index of this graph add nothing
                if (c0 + e * kWave + lane < n && f[e] < nn) {
                    const int sl = edge_slot(f[e], n, rcp_n, par);
                    if (sl == sa) acc_a += gv[e];
                    else if (sl == sb) acc_b += gv[e];
                    else if (sl == sc) acc_c += gv[e];
                    else atomicAdd(&hist[sl], gv[e]);
                }
            }
        }
#pragma unroll
        for (int m = kWave / 2; m >= 1; m >>= 1) {
            acc_a += __shfl_xor(acc_a, m);
            acc_b += __shfl_xor(acc_b, m);
            acc_c += __shfl_xor(acc_c, m);
        }
        if (lane == 0) {
            atomicAdd(&hist[sa], acc_a);
            if (sb >= 0) atomicAdd(&hist[sb], acc_b);
            if (sc >= 0) atomicAdd(&hist[sc], acc_c);
        }
    }
    __syncthreads();
    float* ge = gedge + noff[g];
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const float h = hist[k];
        if (h != 0.0f) atomicAdd(&ge[k], h);
    }
}

// The chain rule through w = ||x_c - x_p|| for every edge (c, parent c), in
// two launches.  The first writes every vertex's own term, dX[c] = f_c (x_c -
// x_p) with f_c = g_c / w_cp (0 at the root), with plain stores (each vertex
// is the child of one edge, so dX needs no clearing), and leaves f_c in
// gedge[c].  The second adds -f_c (x_c - x_p) to the parent's row, the only
// part several edges share (atomics).
__global__ __launch_bounds__(256) void chain_child_kernel(
    const float* __restrict__ X, const int64_t* __restrict__ xoff,
    const float* __restrict__ W, const int64_t* __restrict__ offsets,
    const int64_t* __restrict__ noff, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ parent, float* __restrict__ gedge,
    const int32_t* __restrict__ vstart, int num_graphs, int d, float* __restrict__ dX) {
    const int g = find_item(vstart, num_graphs, blockIdx.x);
    const int n = ns[g];
    const int c = (blockIdx.x - vstart[g]) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int p = parent[noff[g] + c];
    float f = 0.0f;
    if (p >= 0) {
        const float gv = gedge[noff[g] + c];
        const float w = W[offsets[g] + (size_t)c * n + p];
        if (gv != 0.0f && w > 0.0f) f = gv / w;
    }
    gedge[noff[g] + c] = f;
    const float* Xg = X + xoff[g];
    float* dXg = dX + xoff[g];
    for (int t = 0; t < d; ++t)
        dXg[(size_t)c * d + t] = f != 0.0f ? f * (Xg[(size_t)c * d + t] - Xg[(size_t)p * d + t]) : 0.0f;
}

__global__ __launch_bounds__(256) void chain_points_kernel(
    const float* __restrict__ X, const int64_t* __restrict__ xoff,
    const int64_t* __restrict__ noff, const int32_t* __restrict__ ns,
    const int32_t* __restrict__ parent, const float* __restrict__ gedge,
    const int32_t* __restrict__ vstart, int num_graphs, int d, float* __restrict__ dX) {
    const int g = find_item(vstart, num_graphs, blockIdx.x);
    const int n = ns[g];
    const int c = (blockIdx.x - vstart[g]) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int p = parent[noff[g] + c];
    const float f = gedge[noff[g] + c];
    if (p < 0 || f == 0.0f) return;
    const float* Xg = X + xoff[g];
    float* dXg = dX + xoff[g];
    for (int t = 0; t < d; ++t)
        atomicAdd(&dXg[(size_t)p * d + t], -f * (Xg[(size_t)c * d + t] - Xg[(size_t)p * d + t]));
}

hipError_t run_pairwise(const float* X, const int64_t* xoff, const int64_t* offsets,
                        const int32_t* ns, const int32_t* tile_start, int num_graphs,
                        int total_tiles, int d, float* W, hipStream_t s) {
    if (d < 1 || d > kMaxD) return hipErrorInvalidValue;
    if (total_tiles == 0) return hipSuccess;
    APPD_LAUNCH("pairwise_kernel", s,
        pairwise_kernel<<<total_tiles, kPairThreads, pairwise_lds_bytes(d), s>>>(
            X, xoff, offsets, ns, tile_start, num_graphs, d, W));
    return hipGetLastError();
}

hipError_t run_edge_grad(const float* G, const int32_t* idx, const int64_t* offsets,
                         const int64_t* noff, const int32_t* ns, const int32_t* parent,
                         const int32_t* chunk_start, int num_graphs, int total_chunks,
                         int rows_per_wg, int max_n, float* gedge, hipStream_t s) {
    if (total_chunks == 0) return hipSuccess;
    const bool par_lds = max_n <= kGradParLds;
    const size_t lds = (par_lds ? 8 : 4) * (size_t)max_n;
    const void* fn = par_lds ? (const void*)edge_grad_kernel<true> : (const void*)edge_grad_kernel<false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    if (par_lds)
        APPD_LAUNCH("edge_grad_kernel", s,
            edge_grad_kernel<true><<<total_chunks, 256, lds, s>>>(G, idx, offsets, noff, ns, parent,
                chunk_start, num_graphs, rows_per_wg, gedge));
    else
        APPD_LAUNCH("edge_grad_kernel", s,
            edge_grad_kernel<false><<<total_chunks, 256, lds, s>>>(G, idx, offsets, noff, ns,
                parent, chunk_start, num_graphs, rows_per_wg, gedge));
    return hipGetLastError();
}

hipError_t run_chain(const float* X, const int64_t* xoff, const float* W, const int64_t* offsets,
                     const int64_t* noff, const int32_t* ns, const int32_t* parent,
                     float* gedge, const int32_t* vstart, int num_graphs, int total_vblocks,
                     int d, float* dX, hipStream_t s) {
    if (total_vblocks == 0) return hipSuccess;
    APPD_LAUNCH("chain_child_kernel", s,
        chain_child_kernel<<<total_vblocks, 256, 0, s>>>(X, xoff, W, offsets, noff, ns, parent,
            gedge, vstart, num_graphs, d, dX));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    APPD_LAUNCH("chain_points_kernel", s,
        chain_points_kernel<<<total_vblocks, 256, 0, s>>>(X, xoff, noff, ns, parent, gedge,
            vstart, num_graphs, d, dX));
    return hipGetLastError();
}

// Capture-safe clear (a kernel, not a memset node).
__global__ void zero_kernel(uint32_t* __restrict__ p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t run_zero(void* p, size_t bytes, hipStream_t s) {
    const size_t words = bytes / 4;
    if (!words) return hipSuccess;
    const size_t blocks = (words + 255) / 256;
    APPD_LAUNCH("zero_kernel", s,
        zero_kernel<<<(unsigned)(blocks < 8192 ? blocks : 8192), 256, 0, s>>>((uint32_t*)p, words));
    return hipGetLastError();
}

__global__ void scale_offsets_kernel(const int64_t* __restrict__ noff, int num_graphs, int d,
                                     int64_t* __restrict__ xoff) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < num_graphs) xoff[g] = noff[g] * d;
}

hipError_t run_scale_offsets(const int64_t* noff, int num_graphs, int d, int64_t* xoff,
                             hipStream_t s) {
    APPD_LAUNCH("scale_offsets_kernel", s,
        scale_offsets_kernel<<<(num_graphs + 255) / 256, 256, 0, s>>>(noff, num_graphs, d, xoff));
    return hipGetLastError();
}

__global__ void single_table_kernel(int n, int32_t* ns, int64_t* offsets, int64_t* noff,
                                    int32_t* tile_start, int32_t* gchunk_start, int32_t* vstart) {
    if (threadIdx.x == 0) {
        ns[0] = n;
        offsets[0] = 0;
        noff[0] = 0;
        tile_start[0] = 0;
        gchunk_start[0] = 0;
        vstart[0] = 0;
    }
}

hipError_t run_single_table(int n, int32_t* ns, int64_t* offsets, int64_t* noff,
                            int32_t* tile_start, int32_t* gchunk_start, int32_t* vstart,
                            hipStream_t s) {
    APPD_LAUNCH("single_table_kernel", s,
        single_table_kernel<<<1, 64, 0, s>>>(n, ns, offsets, noff, tile_start, gchunk_start,
            vstart));
    return hipGetLastError();
}

// dW[min(c,p)*n + max(c,p)] = gedge[c] for each tree edge (c, parent c) of
// every graph (vertex blocks located through vstart, as in the chain kernel).
__global__ __launch_bounds__(256) void edge_to_w_kernel(
    const float* __restrict__ gedge, const int32_t* __restrict__ parent,
    const int64_t* __restrict__ offsets, const int64_t* __restrict__ noff,
    const int32_t* __restrict__ ns, const int32_t* __restrict__ vstart, int num_graphs,
    float* __restrict__ dW) {
    const int g = find_item(vstart, num_graphs, blockIdx.x);
    const int n = ns[g];
    const int c = (blockIdx.x - vstart[g]) * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int p = parent[noff[g] + c];
    if (p < 0 || p >= n) return;
    const int u = c < p ? c : p, v = c < p ? p : c;
    dW[offsets[g] + (size_t)u * n + v] = gedge[noff[g] + c];
}

hipError_t run_edge_to_w(const float* gedge, const int32_t* parent, const int64_t* offsets,
                         const int64_t* noff, const int32_t* ns, const int32_t* vstart,
                         int num_graphs, int total_vblocks, float* dW, hipStream_t s) {
    if (total_vblocks == 0) return hipSuccess;
    APPD_LAUNCH("edge_to_w_kernel", s,
        edge_to_w_kernel<<<total_vblocks, 256, 0, s>>>(gedge, parent, offsets, noff, ns, vstart,
            num_graphs, dW));
    return hipGetLastError();
}

int pairwise_tile() { return kTile; }
int pairwise_max_d() { return kMaxD; }

}  // namespace appd
