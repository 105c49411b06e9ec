// Process-wide runtime helpers of libkc: device properties, the side-stream
// pool and status text.
#include <atomic>
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
std::mutex g_side_mu;
std::map<int, std::vector<SideStream>> g_side_free;   // per device
}  // namespace

int side_acquire(SideStream* out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KC_EDEVICE;
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
