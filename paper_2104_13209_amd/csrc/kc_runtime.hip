// Process-wide runtime helpers of libkc: device properties, the pools of side
// streams and profiling events (released by kc_shutdown or at process exit,
// while the HIP runtime is still alive), and status text.
#include <atomic>
#include <cstdlib>
#include <map>
#include <mutex>
#include <vector>

#include "kc_internal.h"

namespace kc {

namespace {
constexpr int kMaxDevices = 64;
std::atomic<int> g_cus[kMaxDevices];   // 0 = not read yet (zero-initialised: static storage)
}  // namespace

int device_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev < 0 || dev >= kMaxDevices) return 256;
    int cus = g_cus[dev].load(std::memory_order_relaxed);
    if (cus == 0) {
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        g_cus[dev].store(cus, std::memory_order_relaxed);   // every thread computes the same value
    }
    return cus;
}

namespace {
std::mutex g_side_mu;                                    // guards both pools
std::map<int, std::vector<SideStream>> g_side_free;       // per device
std::map<int, std::vector<ProfileEvents>> g_prof_free;    // per device
std::once_flag g_exit_once;

void release_pools() {
    std::lock_guard<std::mutex> lk(g_side_mu);
    bool any = false;
    for (auto& kv : g_side_free) any |= !kv.second.empty();
    for (auto& kv : g_prof_free) any |= !kv.second.empty();
    if (!any) return;   // nothing to release: no HIP call (also at exit)
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto& kv : g_side_free) {
        (void)hipSetDevice(kv.first);
        for (auto& s : kv.second) {
            (void)hipEventDestroy(s.fork);
            (void)hipEventDestroy(s.join);
            (void)hipStreamDestroy(s.stream);
        }
        kv.second.clear();
    }
    for (auto& kv : g_prof_free) {
        (void)hipSetDevice(kv.first);
        for (auto& e : kv.second) {
            for (auto ev : e.ev) (void)hipEventDestroy(ev);
            for (auto ev : e.wl) (void)hipEventDestroy(ev);
        }
        kv.second.clear();
    }
    if (cur >= 0) (void)hipSetDevice(cur);
}

// The pools are created after the HIP runtime has initialised, so a handler
// registered then runs before the runtime's own teardown at exit.
void register_exit_release() {
    std::call_once(g_exit_once, [] { std::atexit(release_pools); });
}
}  // namespace

int profile_acquire(ProfileEvents* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KC_EDEVICE;
    register_exit_release();
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        auto& v = g_prof_free[dev];
        if (!v.empty()) {
            *out = v.back();
            v.pop_back();
            return KC_OK;
        }
    }
    ProfileEvents e;
    e.device = dev;
    for (auto& ev : e.ev)
        if (hipEventCreate(&ev) != hipSuccess) return KC_EDEVICE;
    for (auto& ev : e.wl)
        if (hipEventCreate(&ev) != hipSuccess) return KC_EDEVICE;
    *out = e;
    return KC_OK;
}

void profile_release(const ProfileEvents& e) {
    std::lock_guard<std::mutex> lk(g_side_mu);
    g_prof_free[e.device].push_back(e);
}

int side_acquire(SideStream* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KC_EDEVICE;
    register_exit_release();
    {
        std::lock_guard<std::mutex> lk(g_side_mu);
        auto& v = g_side_free[dev];
        if (!v.empty()) {
            *out = v.back();
            v.pop_back();
            return KC_OK;
        }
    }
    SideStream s;
    s.device = dev;
    if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) return KC_EDEVICE;
    if (hipEventCreateWithFlags(&s.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&s.join, hipEventDisableTiming) != hipSuccess) {
        if (s.fork) (void)hipEventDestroy(s.fork);
        (void)hipStreamDestroy(s.stream);
        return KC_EDEVICE;
    }
    *out = s;
    return KC_OK;
}

void side_release(const SideStream& s) {
    std::lock_guard<std::mutex> lk(g_side_mu);
    g_side_free[s.device].push_back(s);
}

}  // namespace kc

extern "C" KC_API void kc_shutdown(void) { kc::release_pools(); }

extern "C" KC_API const char* kc_strerror(int32_t s) {
    switch (s) {
        case KC_OK: return "ok";
        case KC_EINVAL: return "invalid argument or malformed graph";
        case KC_ENOMEM: return "workspace too small";
        case KC_EOVERFLOW: return "count exceeds the result width";
        case KC_EDEVICE: return "HIP runtime error";
        case KC_ECANCELED: return "canceled";
        case KC_EUNSUPPORTED: return "graph exceeds a limit of this build";
        default: return "unknown status";
    }
}
