// Process-wide runtime helpers of libkc: device properties and status text.
#include "kc_internal.h"

namespace kc {

int device_cus() {
    static int cached_dev = -1, cached_cus = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (dev != cached_dev) {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        cached_cus = cus;
        cached_dev = dev;
    }
    return cached_cus;
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
