// ttm_api.hip -- status strings, version, per-kernel timing registry.
#include <atomic>
#include <mutex>
#include <string>
#include <vector>
#include <string.h>

#include "ttm_host.hpp"

namespace ttm {

namespace {
struct TimedLaunch {
    std::string name;
    hipEvent_t start, stop;
};
std::mutex g_mu;
bool g_timing = false;
std::vector<TimedLaunch> g_launches;
std::vector<hipEvent_t> g_pool;
thread_local const char *t_pending_name = nullptr;
thread_local hipEvent_t t_pending_start = nullptr;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

bool timing_on() { return g_timing; }

void launch_begin(const char *name, hipStream_t s) {
    if (!g_timing) return;
    std::lock_guard<std::mutex> lk(g_mu);
    t_pending_name = name;
    t_pending_start = take_event();
    if (t_pending_start) (void)hipEventRecord(t_pending_start, s);
}

void launch_end(hipStream_t s) {
    if (!g_timing || !t_pending_start) return;
    std::lock_guard<std::mutex> lk(g_mu);
    hipEvent_t stop = take_event();
    if (!stop) return;
    (void)hipEventRecord(stop, s);
    g_launches.push_back({t_pending_name ? t_pending_name : "?", t_pending_start, stop});
    t_pending_start = nullptr;
}

namespace {
std::atomic<int> g_slab_mode{0};
}
int slab_kernel_mode() { return g_slab_mode.load(std::memory_order_relaxed); }

int device_cu_count() {
    static std::atomic<int> cached[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cached[dev].load(std::memory_order_relaxed);
    if (!n) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cached[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

}  // namespace ttm

extern "C" {

const char *ttm_status_string(int status) {
    switch (status) {
        case TTM_OK: return "ok";
        case TTM_ERR_INVALID_ARG: return "invalid argument";
        case TTM_ERR_UNSUPPORTED: return "unsupported dtype/math combination or size";
        case TTM_ERR_WORKSPACE: return "workspace missing or too small";
        case TTM_ERR_ALIAS: return "output overlaps an input";
        case TTM_ERR_HIP: return "HIP runtime error";
        default: return "unknown status";
    }
}

int ttm_version(void) { return 1 * 10000 + 0 * 100 + 0; }

int ttm_set_slab_kernel(int mode) {
    if (mode < 0 || mode > 3) return TTM_ERR_INVALID_ARG;
    ttm::g_slab_mode.store(mode, std::memory_order_relaxed);
    return TTM_OK;
}

int ttm_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(ttm::g_mu);
    ttm::g_timing = on != 0;
    return TTM_OK;
}

int ttm_timing_collect(char *names, int64_t *counts, double *total_ms, int max) {
    if (max < 0 || (max > 0 && (!names || !counts || !total_ms))) return TTM_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(ttm::g_mu);
    std::vector<std::string> keys;
    std::vector<int64_t> cnt;
    std::vector<double> ms;
    int rc = 0;
    for (auto &l : ttm::g_launches) {
        if (hipEventSynchronize(l.stop) != hipSuccess) rc = TTM_ERR_HIP;
        float t = 0.f;
        if (hipEventElapsedTime(&t, l.start, l.stop) != hipSuccess) rc = TTM_ERR_HIP;
        size_t k = 0;
        for (; k < keys.size(); ++k)
            if (keys[k] == l.name) break;
        if (k == keys.size()) {
            keys.push_back(l.name);
            cnt.push_back(0);
            ms.push_back(0.0);
        }
        cnt[k] += 1;
        ms[k] += t;
        ttm::g_pool.push_back(l.start);
        ttm::g_pool.push_back(l.stop);
    }
    ttm::g_launches.clear();
    if (rc) return rc;
    int n = 0;
    for (size_t k = 0; k < keys.size() && n < max; ++k, ++n) {
        strncpy(names + 64 * n, keys[k].c_str(), 63);
        names[64 * n + 63] = 0;
        counts[n] = cnt[k];
        total_ms[n] = ms[k];
    }
    return n;
}

}  // extern "C"
