// C ABI of libappd (declared in include/appd.h): argument checks, workspace,
// error reporting.  All compute is enqueued by the kernels' launchers.
#include "appd.h"
#include "appd_internal.h"
#include "appd_wcount.h"
#include "appd_prim.h"

namespace {

thread_local int g_last = APPD_OK;

int fail(int code) {
    g_last = code;
    return code;
}

int ok() {
    g_last = APPD_OK;
    return APPD_OK;
}

bool bad_n(int n) { return n < 1 || n > APPD_MAX_N; }

}  // namespace

namespace appd {
void set_last_error(int code) { g_last = code; }
}  // namespace appd

extern "C" {

const char* appd_error_string(int code) {
    switch (code) {
        case APPD_OK: return "APPD_OK: success";
        case APPD_EINVAL: return "APPD_EINVAL: invalid argument (null pointer, n out of range, workspace too small or bad mode)";
        case APPD_EHIP: return "APPD_EHIP: HIP runtime call or kernel launch failed";
        case APPD_ENOMEM: return "APPD_ENOMEM: device allocation failed";
        case APPD_EDATA: return "APPD_EDATA: a validated forward read a W with a NaN or an asymmetric pair";
        default: return "unknown appd status code";
    }
}

int appd_get_last_error(void) { return g_last; }

size_t appd_forward_workspace_bytes(int n) {
    if (bad_n(n)) return 0;
    return appd::single_workspace_bytes(n);
}

int appd_forward_ex(const float* W, int n, int mode, float* M, int32_t* idx, int32_t* order,
                    int32_t* parent, void* ws, size_t ws_bytes, void* stream) {
    if (bad_n(n) || !W || !M || !idx || !appd::valid_mode(mode))
        return fail(APPD_EINVAL);
    hipStream_t s = (hipStream_t)stream;
    const size_t need = appd::single_workspace_bytes(n);
    void* buf = ws;
    if (ws) {
        if (ws_bytes < need || ((uintptr_t)ws & 255u)) return fail(APPD_EINVAL);
    } else {
        if (hipMallocAsync(&buf, need, s) != hipSuccess) {
            (void)hipGetLastError();
            return fail(APPD_ENOMEM);
        }
    }
    appd::SingleWs w = appd::carve_single(buf, n);
    if (order) w.order = order;
    if (parent) w.parent = parent;
    hipError_t e = appd::validate_requested() ? appd::enqueue_input_check(W, n, s) : hipSuccess;
    if (e == hipSuccess) e = appd::run_single(W, n, mode, M, idx, w, s);
    if (!ws) {
        if (hipFreeAsync(buf, s) != hipSuccess && e == hipSuccess) e = hipErrorUnknown;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    return ok();
}

int appd_forward_ws(const float* W, int n, float* M, int32_t* idx, void* ws, size_t ws_bytes,
                    void* stream) {
    if (!ws) return fail(APPD_EINVAL);
    return appd_forward_ex(W, n, APPD_MINIMAX, M, idx, nullptr, nullptr, ws, ws_bytes, stream);
}

int appd_forward(const float* W, int n, float* M, int32_t* idx, void* stream) {
    return appd_forward_ex(W, n, APPD_MINIMAX, M, idx, nullptr, nullptr, nullptr, 0, stream);
}

int appd_tree(const float* W, int n, int mode, int32_t* order, int32_t* parent, void* ws,
              size_t ws_bytes, void* stream) {
    if (bad_n(n) || !W || !ws || !appd::valid_mode(mode)) return fail(APPD_EINVAL);
    if (ws_bytes < appd::single_workspace_bytes(n) || ((uintptr_t)ws & 255u)) return fail(APPD_EINVAL);
    appd::SingleWs w = appd::carve_single(ws, n);
    if (order) w.order = order;
    if (parent) w.parent = parent;
    if (appd::run_tree(W, n, mode, w, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    return ok();
}

int appd_fill(int n, int mode, const void* ws, size_t ws_bytes, float* M, int32_t* idx,
              void* stream) {
    if (bad_n(n) || !ws || !M || !idx || !appd::valid_mode(mode)) return fail(APPD_EINVAL);
    if (ws_bytes < appd::single_workspace_bytes(n) || ((uintptr_t)ws & 255u)) return fail(APPD_EINVAL);
    appd::SingleWs w = appd::carve_single(const_cast<void*>(ws), n);
    if (appd::run_fill(n, mode, M, idx, w, (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    return ok();
}

int appd_tree_stats(int n, int mode, const void* ws, size_t ws_bytes, int32_t* stats,
                    void* stream) {
    if (bad_n(n) || !ws || !stats || !appd::valid_mode(mode)) return fail(APPD_EINVAL);
    if (ws_bytes < appd::single_workspace_bytes(n) || ((uintptr_t)ws & 255u)) return fail(APPD_EINVAL);
    const int algo = mode & 0x30;
    const bool parallel =
        algo == APPD_TREE_BORUVKA || (algo == APPD_TREE_AUTO && n >= appd::parallel_tree_min_n());
    stats[0] = parallel ? 1 : 0;
    stats[1] = stats[2] = stats[3] = stats[4] = 0;
    if (!parallel || n < 2) return ok();
    appd::SingleWs w = appd::carve_single(const_cast<void*>(ws), n);
    if (appd::tree_stats(w.tree_ws, n, &stats[1], &stats[2], &stats[3], &stats[4],
                         (hipStream_t)stream) != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    return ok();
}

int appd_linkage(const float* W, int n, int mode, double* Z, void* ws, size_t ws_bytes,
                 void* stream) {
    if (bad_n(n) || !W || (!Z && n > 1) || !ws || !appd::valid_mode(mode))
        return fail(APPD_EINVAL);
    if (ws_bytes < appd::single_workspace_bytes(n) || ((uintptr_t)ws & 255u)) return fail(APPD_EINVAL);
    appd::SingleWs w = appd::carve_single(ws, n);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = appd::run_tree(W, n, mode, w, s);
    if (e == hipSuccess)
        e = appd::run_linkage(W, n, mode, appd::PrimOut{w.order, w.ek, w.pos, w.parent}, w.tree_ws,
                              Z, s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    return ok();
}

int appd_debug_write_counts(const float* W, int n, int mode, float* M, int32_t* idx,
                            uint32_t* counts, void* ws, size_t ws_bytes, void* stream) {
    if (bad_n(n) || !counts || !ws) return fail(APPD_EINVAL);
    hipStream_t s = (hipStream_t)stream;
    const appd::WriteCount on{counts, M, idx}, off{nullptr, nullptr, nullptr};
    hipError_t e = appd::run_zero(counts, (size_t)n * (size_t)n * 4, s);
    if (e == hipSuccess) e = appd::set_write_count_single(on, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    const int rc = appd_forward_ex(W, n, mode, M, idx, nullptr, nullptr, ws, ws_bytes, stream);
    e = hipStreamSynchronize(s);
    // the switch goes off whatever the forward returned
    const hipError_t e_off = appd::set_write_count_single(off, s);
    const hipError_t e_sync = hipStreamSynchronize(s);
    if (rc != APPD_OK) return rc;
    if (e != hipSuccess || e_off != hipSuccess || e_sync != hipSuccess) {
        (void)hipGetLastError();
        return fail(APPD_EHIP);
    }
    return ok();
}

}  // extern "C"
