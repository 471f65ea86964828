// Replica multi-spin coding: 21 independent lattices packed field by field
// into one word lattice (kernels in ising_replicas.hip, C ABI in
// ising_replicas.cpp).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_common.hpp"

namespace ising {

constexpr int kReplicas = 21;
constexpr int32_t kMaxReplicaL = 1 << 16;  // keeps the counter word r L + c below 2^32

// Everything a half-sweep of the replicas needs; wave-uniform.
struct ReplicaArgs {
    int32_t L;
    uint32_t t_lo, t_hi;  // absolute sweep index
    uint32_t k0, k1;      // Philox key = seed
    uint32_t t4[kReplicas], t8[kReplicas];  // thresholds of replica k
};

hipError_t launch_replica_init(uint64_t* W, int L, uint64_t seed, int hot, hipStream_t s);
hipError_t launch_replica_halfsweep(int wpt, uint64_t* W, const ReplicaArgs& a, int colour, hipStream_t s);
// Per-replica E, M of the current words: series slot idx (21 entries each),
// moment sums mom[21], out_EM[0..41] (E then M), each optional.  `totals` is
// 42 zeroed unsigned 64-bit counters, left zeroed.
hipError_t launch_replica_observe(const uint64_t* W, int L, unsigned long long* totals, int64_t* series_E,
                                  int64_t* series_M, int64_t idx, Moments* mom, int64_t* out_EM, hipStream_t s);
// Spins of replica k in rows r0 .. r0 + nrows - 1 as bytes (row major).
hipError_t launch_replica_unpack(const uint64_t* W, int L, int k, int r0, int nrows, uint8_t* out, hipStream_t s);

}  // namespace ising
