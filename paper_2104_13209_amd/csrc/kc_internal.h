// Internal helpers shared by the HIP sources of libkc (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kc.h"

#define KC_CHECK(call)                                   \
    do {                                                 \
        hipError_t kc_err_ = (call);                     \
        if (kc_err_ != hipSuccess) return KC_EDEVICE;    \
    } while (0)

namespace kc {

constexpr int kWave = 64;

// Workspace carving: consecutive 256-byte aligned slices of one caller buffer.
struct Carver {
    char* base;
    size_t off;
    explicit Carver(void* b) : base(static_cast<char*>(b)), off(0) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
        off += count * sizeof(T);
        return p;
    }
    size_t bytes() const { return (off + 255) & ~size_t(255); }
};

inline int div_up(long long a, long long b) { return static_cast<int>((a + b - 1) / b); }

// Number of compute units of the current device (cached per process).
int device_cus();

// An auxiliary stream (default priority) with two timing-free events, taken
// from a per-device pool for the length of one call, so that one launch of the
// call can run beside the others (fork: record on the caller's stream, wait on
// the side stream; join: the reverse).  Entries are created on first use and
// kept for the life of the process.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    int device = -1;
};
int side_acquire(SideStream* out);      // KC_OK or KC_EDEVICE
void side_release(const SideStream& s);

// Returns a held side stream to the pool at scope exit.
struct SideGuard {
    SideStream s;
    bool held = false;
    ~SideGuard() {
        if (held) side_release(s);
    }
};

// Timing events of one profiled call (kc_profile), from a per-device pool.
struct ProfileEvents {
    hipEvent_t ev[4] = {};
    hipEvent_t wl[12] = {};   // start / end of each width-list launch
    int device = -1;
};
int profile_acquire(ProfileEvents* out);   // KC_OK or KC_EDEVICE
void profile_release(const ProfileEvents& e);

struct ProfileGuard {
    ProfileEvents e;
    bool held = false;
    ~ProfileGuard() {
        if (held) profile_release(e);
    }
};

// ------------------------------------------------------------- device side

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Coherent (L2) load of a value other workgroups update with atomics.
template <class T>
__device__ __forceinline__ T ld_acquire(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Cooperative cancellation: the caller's flag (device memory or mapped host
// memory) holds a non-zero value once the count should stop.  Read at system
// scope so that a write by the host or another device queue is seen.
__device__ __forceinline__ bool cancel_requested(const int* flag) {
    return flag != nullptr && __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
}

// Exact unsigned 128-bit accumulation into device memory: lo receives x and a
// carry out of lo goes to hi (both 64-bit atomics, so the sum is exact).
// Returns true when the 128-bit total wrapped past 2^128.
__device__ __forceinline__ bool atomic_add_u128(unsigned long long* lo, unsigned long long* hi,
                                                unsigned long long x_lo, unsigned long long x_hi) {
    bool carry_in = false;
    if (x_lo) {
        unsigned long long old = atomicAdd(lo, x_lo);
        if (old + x_lo < old) {
            carry_in = true;
        }
    }
    unsigned long long add_hi = x_hi + (carry_in ? 1ull : 0ull);
    bool wrap = carry_in && add_hi == 0ull;   // x_hi was all ones
    if (add_hi) {
        unsigned long long old = atomicAdd(hi, add_hi);
        wrap |= old + add_hi < old;
    }
    return wrap;
}

// 128-bit value as four 32-bit limbs, little endian.
struct U4 { unsigned int l[4]; };

// x * m / d exactly, where d divides x * m; false when the result needs more
// than 128 bits.  The product is formed in five limbs so that no intermediate
// overflow is mistaken for an oversized result.
__device__ inline bool muldiv(U4& x, unsigned int m, unsigned int d) {
    unsigned int p[5];
    unsigned long long carry = 0;
    for (int i = 0; i < 4; i++) {
        unsigned long long t = static_cast<unsigned long long>(x.l[i]) * m + carry;
        p[i] = static_cast<unsigned int>(t);
        carry = t >> 32;
    }
    p[4] = static_cast<unsigned int>(carry);
    unsigned long long r = 0;
    for (int i = 4; i >= 0; i--) {
        unsigned long long cur = (r << 32) | p[i];
        p[i] = static_cast<unsigned int>(cur / d);
        r = cur % d;
    }
    for (int i = 0; i < 4; i++) x.l[i] = p[i];
    return p[4] == 0;
}

// Wave-wide sum of a per-lane u64 into (lo, hi): exact, with carry detection.
__device__ __forceinline__ void wave_sum_u128(unsigned long long v, unsigned long long& lo,
                                              unsigned long long& hi) {
    unsigned long long carry = 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        unsigned long long o = __shfl_xor(v, off, kWave);
        unsigned long long oc = __shfl_xor(carry, off, kWave);
        unsigned long long s = v + o;
        carry += oc + (s < v ? 1ull : 0ull);
        v = s;
    }
    lo = v;
    hi = carry;
}

}  // namespace kc

namespace kc {

// Make this wave's LDS writes visible to its other lanes before they read.
__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ unsigned long long lanemask_lt() {
    unsigned l = __lane_id();
    return l == 0 ? 0ull : (~0ull >> (64 - l));
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o > v ? o : v;
    }
    return v;
}

// Wave-wide maximum of an unsigned 32-bit value with DPP lane moves instead of
// LDS permutes: swap neighbours and pairs inside each quad, mirror the half rows
// and rows (every lane then holds its row of 16's maximum), broadcast lane 15
// into rows 1 and 3 and lane 31 into rows 2 and 3; lane 63 ends with the
// maximum of all 64 lanes.  Every lane must be active.
__device__ __forceinline__ unsigned int wave_max_dpp(unsigned int x) {
    int v = static_cast<int>(x);
#define KC_DPP_MAX(ctrl, rows)                                                                    \
    {                                                                                             \
        const unsigned int t = static_cast<unsigned int>(__builtin_amdgcn_update_dpp(v, v, ctrl, rows, 0xf, false)); \
        v = static_cast<int>(t > static_cast<unsigned int>(v) ? t : static_cast<unsigned int>(v)); \
    }
    KC_DPP_MAX(0xB1, 0xf)    // quad_perm [1, 0, 3, 2]
    KC_DPP_MAX(0x4E, 0xf)    // quad_perm [2, 3, 0, 1]
    KC_DPP_MAX(0x141, 0xf)   // row_half_mirror
    KC_DPP_MAX(0x140, 0xf)   // row_mirror
    KC_DPP_MAX(0x142, 0xa)   // row_bcast:15 into rows 1 and 3
    KC_DPP_MAX(0x143, 0xc)   // row_bcast:31 into rows 2 and 3
#undef KC_DPP_MAX
    return static_cast<unsigned int>(__builtin_amdgcn_readlane(v, 63));
}

template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        T o = __shfl_xor(v, off, kWave);
        v = o < v ? o : v;
    }
    return v;
}

}  // namespace kc
