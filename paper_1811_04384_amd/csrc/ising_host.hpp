// Host-side helpers shared by the C-ABI translation units: thread-local
// error messages, HIP error mapping, argument checks, pinned staging.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
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

// Spin input/output goes through a byte staging buffer in device memory that
// a handle allocates once, at creation: the whole L x L lattice when it is
// small, else 16 MiB, moved in pieces of whole rows.  No call that reads or
// writes spins allocates or frees device memory.
constexpr size_t kSpinStageMax = size_t(16) << 20;
inline size_t spin_stage_bytes(int32_t L) { return std::min((size_t)L * (size_t)L, kSpinStageMax); }

// The nrows x ncols window with top-left site (r0, c0), indices mod L, into
// host bytes (row major, 1 = up), staged through `stage` (cap bytes >= ncols);
// synchronises the stream.
int read_spin_window(const uint64_t* W, const Geometry& g, int32_t r0, int32_t c0, int32_t nrows, int32_t ncols,
                     uint8_t* host, uint8_t* stage, size_t cap, hipStream_t s);
// Replace every spin by the host bytes (L x L, nonzero = up), staged through
// `stage` (cap bytes >= L); synchronises the stream.
int write_spins(uint64_t* W, const Geometry& g, const uint8_t* host, uint8_t* stage, size_t cap, hipStream_t s);

}  // namespace ising
