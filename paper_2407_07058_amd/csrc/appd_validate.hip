// Precondition check of a weight matrix (appd_validate, include/appd.h).
//
// The method takes an undirected graph with edge weights (Section 1), so W must
// be symmetric; the library also asks for a NaN-free W with a zero diagonal.
// One pass over W: workgroup (bi, bj), bi <= bj, loads the 64 x 64 tile at
// rows bi, columns bj and the mirrored tile at rows bj, columns bi (both
// coalesced, the second through LDS transposed), so every element is read
// once and compared with its mirror image.  Flags are or-ed per wave into one
// device word.
#include <mutex>

#include "appd.h"
#include "appd_device.h"
#include "appd_internal.h"

namespace appd {
namespace {

constexpr int kVT = 64;        // tile edge
constexpr int kVThreads = 256;  // 16 elements of each tile per thread

// Tile pair of workgroup b: the b-th (bi, bj), bi <= bj, in row-major order of
// the upper triangle of a T x T grid of tiles.
__device__ __forceinline__ void tile_pair(int b, int T, int* bi, int* bj) {
    // rows before bi hold bi*T - bi*(bi-1)/2 pairs; invert in double, then fix up
    const double tt = 2.0 * T + 1.0;
    int i = (int)((tt - sqrt(tt * tt - 8.0 * (double)b)) * 0.5);
    if (i < 0) i = 0;
    if (i > T - 1) i = T - 1;
    auto start = [&](int r) { return (int64_t)r * T - (int64_t)r * (r - 1) / 2; };
    while (i > 0 && start(i) > b) --i;
    while (i < T - 1 && start(i + 1) <= b) ++i;
    *bi = i;
    *bj = i + (int)(b - start(i));
}

__global__ __launch_bounds__(kVThreads) void validate_kernel(const float* __restrict__ W, int n,
                                                             int T, uint32_t* __restrict__ flags) {
    __shared__ float mirror[kVT][kVT + 1];
    int bi, bj;
    tile_pair(blockIdx.x, T, &bi, &bj);
    const int t = threadIdx.x;
    const int c = t & (kVT - 1), r0 = t / kVT;  // 4 rows per pass, 16 passes
    uint32_t f = 0;
    // mirrored tile: rows bj*64 + r, columns bi*64 + c, stored transposed
    for (int r = r0; r < kVT; r += kVThreads / kVT) {
        const int gr = bj * kVT + r, gc = bi * kVT + c;
        mirror[c][r] = (gr < n && gc < n) ? W[(size_t)gr * n + gc] : 0.0f;
    }
    __syncthreads();
    for (int r = r0; r < kVT; r += kVThreads / kVT) {
        const int gr = bi * kVT + r, gc = bj * kVT + c;
        if (gr >= n || gc >= n) continue;
        const float x = W[(size_t)gr * n + gc];
        const float y = mirror[r][c];  // W[gc][gr]
        if (x != x) f |= APPD_VALID_NAN;
        if (gr == gc) {
            if (x != 0.0f) f |= APPD_VALID_DIAG;
        } else if (bi != bj && y != y) {
            f |= APPD_VALID_NAN;  // the mirror tile is a different part of W
        }
        if (gr != gc && x == x && y == y && x != y) f |= APPD_VALID_ASYM;
    }
    // one atomic per wave
    uint32_t m = f;
    m |= __shfl_xor(m, 1);
    m |= __shfl_xor(m, 2);
    m |= __shfl_xor(m, 4);
    m |= __shfl_xor(m, 8);
    m |= __shfl_xor(m, 16);
    m |= __shfl_xor(m, 32);
    if ((t & (kWave - 1)) == 0 && m) atomicOr(flags, m);
}

__global__ void validate_clear_kernel(uint32_t* flags) {
    if (threadIdx.x == 0) *flags = 0u;
}

// Flags of the validated forwards since the last appd_sync on this GPU.
__device__ uint32_t pending_flags;

constexpr int kMaxDevices = 64;
std::mutex g_pending_mu;
uint32_t* g_pending_ptr[kMaxDevices];

// The current GPU's copy of pending_flags (null on a HIP error).
uint32_t* pending_for_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_pending_mu);
    if (!g_pending_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(pending_flags)) != hipSuccess || !p) return nullptr;
        g_pending_ptr[dev] = (uint32_t*)p;
    }
    return g_pending_ptr[dev];
}

}  // namespace

uint32_t* device_status_word() { return pending_for_current_device(); }

hipError_t enqueue_input_check(const float* W, int n, hipStream_t s) {
    uint32_t* pending = pending_for_current_device();
    if (!pending) return hipErrorUnknown;
    const int T = (n + kVT - 1) / kVT;
    APPD_LAUNCH("validate_kernel", s,
                validate_kernel<<<T * (T + 1) / 2, kVThreads, 0, s>>>(W, n, T, pending));
    return hipGetLastError();
}

}  // namespace appd

extern "C" int appd_sync(void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        appd::set_last_error(APPD_EHIP);
        return APPD_EHIP;
    }
    uint32_t* pending = appd::pending_for_current_device();
    uint32_t flags = 0;
    if (!pending || hipMemcpyAsync(&flags, pending, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        (void)hipGetLastError();
        appd::set_last_error(APPD_EHIP);
        return APPD_EHIP;
    }
    if (flags) {
        const uint32_t zero = 0;
        if (hipMemcpyAsync(pending, &zero, 4, hipMemcpyHostToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            (void)hipGetLastError();
            appd::set_last_error(APPD_EHIP);
            return APPD_EHIP;
        }
    }
    const int rc = (flags & appd::kStatusWaitTimeout) ? APPD_EHIP
                   : (flags & (APPD_VALID_NAN | APPD_VALID_ASYM)) ? APPD_EDATA
                                                                  : APPD_OK;
    appd::set_last_error(rc);
    return rc;
}

extern "C" int appd_validate(const float* W, int n, uint32_t* flags, void* stream) {
    if (!W || !flags || n < 1 || n > APPD_MAX_N) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const int T = (n + appd::kVT - 1) / appd::kVT;
    const int pairs = T * (T + 1) / 2;
    APPD_LAUNCH("validate_clear_kernel", s, appd::validate_clear_kernel<<<1, 64, 0, s>>>(flags));
    APPD_LAUNCH("validate_kernel", s,
                appd::validate_kernel<<<pairs, appd::kVThreads, 0, s>>>(W, n, T, flags));
    if (hipGetLastError() != hipSuccess) {
        appd::set_last_error(APPD_EHIP);
        return APPD_EHIP;
    }
    appd::set_last_error(APPD_OK);
    return APPD_OK;
}
