// Launch timer (appd_timer_* in appd.h): HIP events recorded on the launch
// stream immediately before and after each launch of the selected kernel(s).
// The events are created by appd_timer_start, so a timed region records events
// only; nothing is allocated while it runs.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>
#include <vector>

#include "appd.h"
#include "appd_internal.h"

namespace appd {
namespace {

struct Record {
    const char* name;  // static string of the launch site
    hipEvent_t begin, end;
};

std::mutex g_mu;
std::atomic<bool> g_on{false};
bool g_all = false;
char g_name[128];
std::vector<hipEvent_t> g_pool;  // 2 * capacity events
std::vector<Record> g_rec;
size_t g_next = 0;
bool g_overflow = false;
thread_local int g_open = -1;  // record opened by timer_begin on this thread

void destroy_pool() {
    for (hipEvent_t e : g_pool) (void)hipEventDestroy(e);
    g_pool.clear();
    g_rec.clear();
    g_next = 0;
}

int env_flag(const char* name) {
    const char* v = getenv(name);
    return (v && *v && strcmp(v, "0") != 0) ? 1 : 0;
}

}  // namespace

bool log_on() {
    static const bool on = env_flag("APPD_LOG") != 0;
    return on;
}

void log_launch(const char* name, hipStream_t s) {
    fprintf(stderr, "appd: launch %s stream=%p\n", name, (void*)s);
}

bool validate_requested() { return env_flag("APPD_VALIDATE") != 0; }

namespace {
}  // namespace

bool timer_wants(const char* name) {
    if (!g_on.load(std::memory_order_relaxed)) return false;
    std::lock_guard<std::mutex> lk(g_mu);
    return g_on && (g_all || strcmp(g_name, name) == 0);
}

void timer_begin(const char* name, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_open = -1;
    if (g_next >= g_pool.size() / 2) {
        g_overflow = true;
        return;
    }
    Record r{name, g_pool[2 * g_next], g_pool[2 * g_next + 1]};
    if (hipEventRecord(r.begin, s) != hipSuccess) {
        (void)hipGetLastError();
        g_overflow = true;
        return;
    }
    g_rec.push_back(r);
    g_open = (int)g_next++;
}

void timer_end(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_open < 0) return;
    if (hipEventRecord(g_rec[g_open].end, s) != hipSuccess) {
        (void)hipGetLastError();
        g_overflow = true;
        g_rec.pop_back();
        --g_next;
    }
    g_open = -1;
}

}  // namespace appd

extern "C" {

int appd_timer_start(const char* kernel, int capacity) {
    std::lock_guard<std::mutex> lk(appd::g_mu);
    appd::g_on = false;
    appd::destroy_pool();
    appd::g_overflow = false;
    if (!kernel) {
        appd::set_last_error(APPD_OK);
        return APPD_OK;
    }
    if (capacity < 1 || capacity > (1 << 20) || strlen(kernel) >= sizeof(appd::g_name)) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    appd::g_pool.reserve(2 * (size_t)capacity);
    for (int i = 0; i < 2 * capacity; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            appd::destroy_pool();
            appd::set_last_error(APPD_EHIP);
            return APPD_EHIP;
        }
        appd::g_pool.push_back(e);
    }
    appd::g_rec.reserve(capacity);
    strcpy(appd::g_name, kernel);
    appd::g_all = strcmp(kernel, "*") == 0;
    appd::g_on = true;
    appd::set_last_error(APPD_OK);
    return APPD_OK;
}

int appd_timer_read(const char* kernel, int* launches, double* total_ms, int* overflow) {
    std::lock_guard<std::mutex> lk(appd::g_mu);
    if (!kernel || !launches || !total_ms) {
        appd::set_last_error(APPD_EINVAL);
        return APPD_EINVAL;
    }
    int cnt = 0;
    double tot = 0.0;
    for (const appd::Record& r : appd::g_rec) {
        if (strcmp(r.name, kernel) != 0) continue;
        float ms = 0.f;
        if (hipEventSynchronize(r.end) != hipSuccess ||
            hipEventElapsedTime(&ms, r.begin, r.end) != hipSuccess) {
            (void)hipGetLastError();
            appd::set_last_error(APPD_EHIP);
            return APPD_EHIP;
        }
        ++cnt;
        tot += ms;
    }
    *launches = cnt;
    *total_ms = tot;
    if (overflow) *overflow = appd::g_overflow ? 1 : 0;
    appd::set_last_error(APPD_OK);
    return APPD_OK;
}

int appd_timer_names(const char** names, int capacity) {
    std::lock_guard<std::mutex> lk(appd::g_mu);
    std::vector<const char*> uniq;
    for (const appd::Record& r : appd::g_rec) {
        bool seen = false;
        for (const char* u : uniq) seen |= strcmp(u, r.name) == 0;
        if (!seen) uniq.push_back(r.name);
    }
    for (int i = 0; names && i < capacity && i < (int)uniq.size(); ++i) names[i] = uniq[i];
    appd::set_last_error(APPD_OK);
    return (int)uniq.size();
}

}  // extern "C"
