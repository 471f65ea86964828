// Host-side helpers shared by the C-ABI translation units: thread-local
// error messages, HIP error mapping, argument checks, pinned staging.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/ising.h"
#include "ising_common.hpp"

namespace ising {

// The device-side moment sums are handed out as ising_moments unchanged.
static_assert(sizeof(Moments) == sizeof(ising_moments), "Moments layout");
static_assert(offsetof(Moments, sum_E2) == offsetof(ising_moments, sum_E2), "Moments layout");
static_assert(offsetof(Moments, sum_absM) == offsetof(ising_moments, sum_absM), "Moments layout");
static_assert(offsetof(Moments, sum_M4) == offsetof(ising_moments, sum_M4), "Moments layout");

std::string& last_error_ref();

inline int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    last_error_ref() = buf;
    return code;
}

inline int hip_fail(hipError_t e, const char* what) {
    return fail(ISING_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

#define ISING_HIP(call)                                      \
    do {                                                     \
        hipError_t ising_e_ = (call);                        \
        if (ising_e_ != hipSuccess) return ::ising::hip_fail(ising_e_, #call); \
    } while (0)

inline bool valid_L(int32_t L) { return L >= 4 && L <= kMaxL && (L % 2) == 0; }
inline bool valid_T(double T) { return std::isfinite(T) && T > 0.0; }

// floor(exp(x) 2^32) clamped to [0, 2^32 - 1], in IEEE double with the C
// library exp (the acceptance probability exp(-dE/kT) of Section 2, step 3,
// as an integer threshold for 32-bit uniforms).
inline uint32_t threshold_from_exponent(double x) {
    const double v = std::floor(std::exp(x) * 4294967296.0);
    if (v >= 4294967295.0) return 4294967295u;
    if (v <= 0.0) return 0u;
    return (uint32_t)v;
}

inline void thresholds_of(double T, uint32_t* t4, uint32_t* t8) {
    *t4 = threshold_from_exponent(-4.0 / T);
    *t8 = threshold_from_exponent(-8.0 / T);
}

inline bool valid_block(int b, int max_block) { return b >= 64 && b <= max_block && b % 64 == 0; }

}  // namespace ising
