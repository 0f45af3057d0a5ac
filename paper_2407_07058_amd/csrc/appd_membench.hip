// Measurement aids: the reference points the kernels are compared with, taken
// on the same GPU.
//
//  - a streaming copy and a streaming store (16-byte vectors, grid-stride, a
//    launch wide enough for every CU): what plain HBM traffic reaches, beside
//    the published peak;
//  - a dependent-load chase: one lane follows next[] for `steps` loads, each
//    address known only when the previous load returns; the time per step is
//    the latency floor of a chain of dependent memory accesses (HBM when the
//    chain spans far more than the caches, L2 when it fits), against which the
//    sequential Prim step is compared.
#include "appd.h"
#include "appd_internal.h"

namespace appd {
namespace {

constexpr int kMbThreads = 256;
constexpr int kMbVec = 4;  // 16-byte vectors per thread: a workgroup covers 16 KiB
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// Workgroup b covers vectors [b * 1024, (b + 1) * 1024); thread t takes
// t, t + 256, t + 512, t + 768 of them (each instruction of a wave touches
// 1 KiB of contiguous memory), all loads issued before the stores.
__global__ __launch_bounds__(kMbThreads) void membench_copy_kernel(const u4v* __restrict__ src,
                                                                   u4v* __restrict__ dst,
                                                                   size_t n16) {
    const size_t base = (size_t)blockIdx.x * (kMbThreads * kMbVec) + threadIdx.x;
    u4v v[kMbVec];
#pragma unroll
    for (int k = 0; k < kMbVec; ++k) {
        const size_t i = base + (size_t)k * kMbThreads;
        if (i < n16) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < kMbVec; ++k) {
        const size_t i = base + (size_t)k * kMbThreads;
        if (i < n16) __builtin_nontemporal_store(v[k], dst + i);
    }
}

__global__ __launch_bounds__(kMbThreads) void membench_write_kernel(u4v* __restrict__ dst,
                                                                    size_t n16, uint32_t v) {
    const size_t base = (size_t)blockIdx.x * (kMbThreads * kMbVec) + threadIdx.x;
    const u4v x = {v, v, v, v};
#pragma unroll
    for (int k = 0; k < kMbVec; ++k) {
        const size_t i = base + (size_t)k * kMbThreads;
        if (i < n16) __builtin_nontemporal_store(x, dst + i);
    }
}

inline unsigned mb_blocks(size_t n16) {
    return (unsigned)((n16 + kMbThreads * kMbVec - 1) / (kMbThreads * kMbVec));
}

__global__ void membench_chase_kernel(const uint32_t* __restrict__ next, uint32_t length,
                                      uint32_t start, int steps, uint32_t* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint32_t p = start < length ? start : 0u;
    for (int s = 0; s < steps; ++s) {
        // keep the index in a vector register, so that the load is a vector
        // memory load (the path the kernels' dependent loads take), not a
        // scalar-cache load
        asm volatile("" : "+v"(p));
        p = __builtin_nontemporal_load(next + p);
        p = p < length ? p : 0u;  // any table stays in bounds
    }
    *out = p;
}

}  // namespace
}  // namespace appd

extern "C" {

int appd_membench_copy(const void* src, void* dst, size_t bytes, void* stream) {
    if (!src || !dst || (bytes & 15u) || (((uintptr_t)src | (uintptr_t)dst) & 15u) ||
        bytes / 16 / (appd::kMbThreads * appd::kMbVec) >= 0x7fffffffu) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    APPD_LAUNCH("membench_copy_kernel", s,
                appd::membench_copy_kernel<<<appd::mb_blocks(bytes / 16), appd::kMbThreads, 0, s>>>(
                    (const appd::u4v*)src, (appd::u4v*)dst, bytes / 16));
    if (hipGetLastError() != hipSuccess) {
        appd::set_last_error(APPD_EHIP);
        return APPD_EHIP;
    }
    appd::set_last_error(APPD_OK);
    return APPD_OK;
}

int appd_membench_write(void* dst, size_t bytes, uint32_t value, void* stream) {
    if (!dst || (bytes & 15u) || ((uintptr_t)dst & 15u) ||
        bytes / 16 / (appd::kMbThreads * appd::kMbVec) >= 0x7fffffffu) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    APPD_LAUNCH("membench_write_kernel", s,
                appd::membench_write_kernel<<<appd::mb_blocks(bytes / 16), appd::kMbThreads, 0, s>>>(
                    (appd::u4v*)dst, bytes / 16, value));
    if (hipGetLastError() != hipSuccess) {
        appd::set_last_error(APPD_EHIP);
        return APPD_EHIP;
    }
    appd::set_last_error(APPD_OK);
    return APPD_OK;
}

int appd_membench_chase(const uint32_t* next, uint32_t length, uint32_t start, int steps,
                        uint32_t* out, void* stream) {
    if (!next || !out || steps < 0 || length == 0) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    APPD_LAUNCH("membench_chase_kernel", s,
                appd::membench_chase_kernel<<<1, 64, 0, s>>>(next, length, start, steps, out));
    if (hipGetLastError() != hipSuccess) {
        appd::set_last_error(APPD_EHIP);
        return APPD_EHIP;
    }
    appd::set_last_error(APPD_OK);
    return APPD_OK;
}

}  // extern "C"
