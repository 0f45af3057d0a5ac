// appd_forward_noalloc: the single-graph forward with its workspace in a
// file-scope device array, for callers that cannot allocate device memory.
//
// The kernels are those of appd_forward_ws; only the workspace differs.  It is
// `scratch` below, APPD_NOALLOC_SCRATCH_BYTES per GPU, which every n up to
// APPD_MAX_N fits (about 240 bytes per vertex).  Each GPU the library runs on
// holds its own copy until the process ends.  In host code the array's name is
// only a stand-in, so the device address of each GPU's copy is looked up once
// per device (hipGetSymbolAddress, with that device current) and that address
// is what the kernels receive.
//
// Nothing in the workspace has to start at zero: appd_forward_ws accepts an
// uninitialised caller buffer, and every kernel writes what it later reads.
// Calls on one GPU share the array, so two calls that overlap on that GPU (on
// different streams, or from different host threads without ordering) race.
#include <mutex>

#include "appd.h"
#include "appd_internal.h"

namespace {

static_assert(APPD_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size in 256-byte units");
__device__ __align__(256) unsigned char scratch[APPD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of each GPU's copy (null: not looked up)

// The current device's copy of `scratch`, looked up on the first call on that
// device.  Returns null on a HIP error.
void* scratch_for_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

}  // namespace

extern "C" int appd_forward_noalloc(const float* W, int n, float* M, int32_t* idx, void* stream) {
    if (!W || !M || !idx || n < 1 || n > APPD_MAX_N) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    const size_t need = appd_forward_workspace_bytes(n);
    if (need == 0 || need > (size_t)APPD_NOALLOC_SCRATCH_BYTES) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    void* ws = scratch_for_current_device();
    if (!ws) {
        (void)hipGetLastError();
        appd::set_last_error(APPD_EHIP);
        return APPD_EHIP;
    }
    return appd_forward_ws(W, n, M, idx, ws, need, stream);
}
