// Exact moment sums of sampled (E, M), shared by the kernels that take
// samples.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_common.hpp"

namespace ising {

// Adds the sample (E, M) to exact moment sums.  For L <= 2^18, |E| <= 2 L^2
// <= 2^37 and |M| <= L^2 = 2^36, so E^2 and M^2 fit 128 bits; M^4 < 2^144 is
// formed in three limbs from q = M^2 = qh 2^64 + ql (qh < 2^8):
// q^2 = ql^2 + 2 ql qh 2^64 + qh^2 2^128.
__device__ inline void add128(uint64_t* s, unsigned __int128 x) {
    unsigned __int128 v = ((unsigned __int128)s[1] << 64) | s[0];
    v += x;
    s[0] = (uint64_t)v;
    s[1] = (uint64_t)(v >> 64);
}

__device__ inline void add_sample(Moments& m, int64_t E, int64_t M) {
    typedef unsigned __int128 u128;
    const uint64_t aE = E < 0 ? 0ull - (uint64_t)E : (uint64_t)E;
    const uint64_t aM = M < 0 ? 0ull - (uint64_t)M : (uint64_t)M;
    m.n += 1;
    m.sum_E += E;
    m.sum_absM += (int64_t)aM;
    add128(m.sum_E2, (u128)aE * aE);
    const u128 q = (u128)aM * aM;
    add128(m.sum_M2, q);
    const uint64_t ql = (uint64_t)q, qh = (uint64_t)(q >> 64);
    const u128 p0 = (u128)ql * ql;
    const u128 p1 = ((u128)ql * qh) << 1;
    const u128 mid = (p0 >> 64) + (uint64_t)p1;
    const uint64_t l0 = (uint64_t)p0, l1 = (uint64_t)mid;
    const uint64_t l2 = (uint64_t)(mid >> 64) + (uint64_t)(p1 >> 64) + qh * qh;
    const u128 a = (u128)m.sum_M4[0] + l0;
    const u128 b = (u128)m.sum_M4[1] + l1 + (uint64_t)(a >> 64);
    m.sum_M4[0] = (uint64_t)a;
    m.sum_M4[1] = (uint64_t)b;
    m.sum_M4[2] += l2 + (uint64_t)(b >> 64);
}

// a += b, exactly (limb sums with carries; the sums are integers, so the
// order in which samples are merged does not matter).
__device__ inline void merge_moments(Moments& a, const Moments& b) {
    typedef unsigned __int128 u128;
    a.n += b.n;
    a.sum_E += b.sum_E;
    a.sum_absM += b.sum_absM;
    add128(a.sum_E2, ((u128)b.sum_E2[1] << 64) | b.sum_E2[0]);
    add128(a.sum_M2, ((u128)b.sum_M2[1] << 64) | b.sum_M2[0]);
    const u128 x = (u128)a.sum_M4[0] + b.sum_M4[0];
    const u128 y = (u128)a.sum_M4[1] + b.sum_M4[1] + (uint64_t)(x >> 64);
    a.sum_M4[0] = (uint64_t)x;
    a.sum_M4[1] = (uint64_t)y;
    a.sum_M4[2] += b.sum_M4[2] + (uint64_t)(y >> 64);
}

// Every lane of a full wavefront ends with the merge of all 64 lanes' sums.
__device__ inline void wave_merge_moments(Moments& m) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        Moments o;
        o.n = __shfl_xor(m.n, off, 64);
        o.sum_E = __shfl_xor(m.sum_E, off, 64);
        o.sum_absM = __shfl_xor(m.sum_absM, off, 64);
        o.sum_E2[0] = __shfl_xor(m.sum_E2[0], off, 64);
        o.sum_E2[1] = __shfl_xor(m.sum_E2[1], off, 64);
        o.sum_M2[0] = __shfl_xor(m.sum_M2[0], off, 64);
        o.sum_M2[1] = __shfl_xor(m.sum_M2[1], off, 64);
        o.sum_M4[0] = __shfl_xor(m.sum_M4[0], off, 64);
        o.sum_M4[1] = __shfl_xor(m.sum_M4[1], off, 64);
        o.sum_M4[2] = __shfl_xor(m.sum_M4[2], off, 64);
        merge_moments(m, o);
    }
}

}  // namespace ising
