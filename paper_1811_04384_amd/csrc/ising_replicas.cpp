// C ABI of replica multi-spin coding: 21 independent L x L lattices in one
// word lattice, replica k at its own temperature (see ising_replicas.hip).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>

#include "ising_host.hpp"
#include "ising_replicas.hpp"

using namespace ising;

struct ising_replicas {
    int32_t L = 0;
    uint64_t seed = 0;
    uint64_t t = 0;  // absolute index of the next sweep
    uint64_t* W = nullptr;
    hipStream_t stream = nullptr;
    int wpt = 2;
    unsigned long long* d_totals = nullptr;  // 42 counters of the observables reduction
    int64_t* d_EM = nullptr;                 // E[21], M[21] of ising_replicas_observables
    uint8_t* d_stage = nullptr;              // spin output staging, spin_stage_bytes(L)
};

namespace {

void release(ising_replicas* h) {
    if (!h) return;
    if (h->W) (void)hipFree(h->W);
    if (h->d_totals) (void)hipFree(h->d_totals);
    if (h->d_EM) (void)hipFree(h->d_EM);
    if (h->d_stage) (void)hipFree(h->d_stage);
    delete h;
}

bool valid_replica_L(int32_t L) { return L >= 4 && L <= kMaxReplicaL && L % 2 == 0; }

int fill_args(ising_replicas* h, const double* T, ReplicaArgs* a, const char* who) {
    if (!h) return fail(ISING_EINVAL, "%s: null handle", who);
    if (!T) return fail(ISING_EINVAL, "%s: null temperatures", who);
    for (int k = 0; k < kReplicas; ++k) {
        if (!valid_T(T[k])) return fail(ISING_EINVAL, "%s: T[%d] = %g is not finite and > 0", who, k, T[k]);
        thresholds_of(T[k], &a->t4[k], &a->t8[k]);
    }
    a->L = h->L;
    a->k0 = (uint32_t)h->seed;
    a->k1 = (uint32_t)(h->seed >> 32);
    return ISING_OK;
}

int sweep_impl(ising_replicas* h, const double* T, int64_t n, int32_t every, int64_t* dev_E, int64_t* dev_M,
               ising_moments* dev_acc, const char* who) {
    ReplicaArgs a;
    int rc = fill_args(h, T, &a, who);
    if (rc != ISING_OK) return rc;
    if (n < 0 || every < 0) return fail(ISING_EINVAL, "%s: negative count", who);
    if ((dev_E || dev_M || dev_acc) && every == 0) return fail(ISING_EINVAL, "%s: outputs need every >= 1", who);
    for (int64_t k = 1; k <= n; ++k) {
        const uint64_t t = h->t + (uint64_t)(k - 1);
        a.t_lo = (uint32_t)t;
        a.t_hi = (uint32_t)(t >> 32);
        ISING_HIP(launch_replica_halfsweep(h->wpt, h->W, a, 0, h->stream));
        ISING_HIP(launch_replica_halfsweep(h->wpt, h->W, a, 1, h->stream));
        if (every > 0 && k % every == 0)
            ISING_HIP(launch_replica_observe(h->W, h->L, h->d_totals, dev_E, dev_M, k / every - 1,
                                             reinterpret_cast<Moments*>(dev_acc), nullptr, h->stream));
    }
    h->t += (uint64_t)n;
    return ISING_OK;
}

}  // namespace

extern "C" {

int ising_replicas_create(int32_t L, uint64_t seed, int32_t init, void* stream, ising_replicas** out) {
    if (!out) return fail(ISING_EINVAL, "ising_replicas_create: null output handle");
    *out = nullptr;
    if (!valid_replica_L(L))
        return fail(ISING_EINVAL, "ising_replicas_create: L = %d must be even with 4 <= L <= %d", L, kMaxReplicaL);
    if (init != ISING_COLD && init != ISING_HOT) return fail(ISING_EINVAL, "ising_replicas_create: bad init %d", init);
    ising_replicas* h = new (std::nothrow) ising_replicas;
    if (!h) return fail(ISING_ENOMEM, "ising_replicas_create: out of host memory");
    h->L = L;
    h->seed = seed;
    h->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipMalloc(&h->W, sizeof(uint64_t) * (size_t)L * (size_t)L);
    if (e == hipSuccess) e = hipMalloc(&h->d_totals, sizeof(unsigned long long) * 2 * kReplicas);
    if (e == hipSuccess) e = hipMalloc(&h->d_EM, sizeof(int64_t) * 2 * kReplicas);
    if (e == hipSuccess) e = hipMalloc(&h->d_stage, spin_stage_bytes(L));
    if (e == hipSuccess) e = hipMemsetAsync(h->d_totals, 0, sizeof(unsigned long long) * 2 * kReplicas, h->stream);
    if (e == hipSuccess) e = launch_replica_init(h->W, L, seed, init == ISING_HOT, h->stream);
    if (e != hipSuccess) {
        release(h);
        return e == hipErrorOutOfMemory ? fail(ISING_ENOMEM, "ising_replicas_create: device memory")
                                        : hip_fail(e, "ising_replicas_create");
    }
    *out = h;
    return ISING_OK;
}

int ising_replicas_destroy(ising_replicas* h) {
    if (!h) return ISING_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    release(h);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ISING_OK;
}

int ising_replicas_sweep(ising_replicas* h, const double* T, int64_t n_sweeps) {
    return sweep_impl(h, T, n_sweeps, 0, nullptr, nullptr, nullptr, "ising_replicas_sweep");
}

int ising_replicas_sweep_measure(ising_replicas* h, const double* T, int64_t n_sweeps, int32_t every, int64_t* dev_E,
                                 int64_t* dev_M) {
    if (every < 1) return fail(ISING_EINVAL, "ising_replicas_sweep_measure: every must be >= 1");
    if (!dev_E || !dev_M) return fail(ISING_EINVAL, "ising_replicas_sweep_measure: null series pointer");
    return sweep_impl(h, T, n_sweeps, every, dev_E, dev_M, nullptr, "ising_replicas_sweep_measure");
}

int ising_replicas_sweep_moments(ising_replicas* h, const double* T, int64_t n_sweeps, int32_t every,
                                 ising_moments* dev_acc) {
    if (every < 1) return fail(ISING_EINVAL, "ising_replicas_sweep_moments: every must be >= 1");
    if (!dev_acc) return fail(ISING_EINVAL, "ising_replicas_sweep_moments: null accumulator");
    return sweep_impl(h, T, n_sweeps, every, nullptr, nullptr, dev_acc, "ising_replicas_sweep_moments");
}

int ising_replicas_observables(ising_replicas* h, int64_t* E, int64_t* M) {
    if (!h || !E || !M) return fail(ISING_EINVAL, "ising_replicas_observables: null argument");
    ISING_HIP(launch_replica_observe(h->W, h->L, h->d_totals, nullptr, nullptr, 0, nullptr, h->d_EM, h->stream));
    int64_t em[2 * kReplicas];
    ISING_HIP(hipMemcpyAsync(em, h->d_EM, sizeof em, hipMemcpyDeviceToHost, h->stream));
    ISING_HIP(hipStreamSynchronize(h->stream));
    for (int k = 0; k < kReplicas; ++k) {
        E[k] = em[k];
        M[k] = em[kReplicas + k];
    }
    return ISING_OK;
}

int ising_replicas_get_spins(ising_replicas* h, int32_t k, uint8_t* host) {
    if (!h || !host) return fail(ISING_EINVAL, "ising_replicas_get_spins: null argument");
    if (k < 0 || k >= kReplicas) return fail(ISING_EINVAL, "ising_replicas_get_spins: replica %d out of range", k);
    const int32_t L = h->L;
    const int32_t chunk = (int32_t)std::max<size_t>(1, spin_stage_bytes(L) / (size_t)L);
    for (int32_t r0 = 0; r0 < L; r0 += chunk) {
        const int32_t nr = std::min(chunk, L - r0);
        ISING_HIP(launch_replica_unpack(h->W, L, k, r0, nr, h->d_stage, h->stream));
        ISING_HIP(hipMemcpyAsync(host + (size_t)r0 * (size_t)L, h->d_stage, (size_t)nr * (size_t)L,
                                 hipMemcpyDeviceToHost, h->stream));
    }
    ISING_HIP(hipStreamSynchronize(h->stream));
    return ISING_OK;
}

int ising_replicas_get_sweep_count(ising_replicas* h, uint64_t* t) {
    if (!h || !t) return fail(ISING_EINVAL, "ising_replicas_get_sweep_count: null argument");
    *t = h->t;
    return ISING_OK;
}

int ising_replicas_set_plan(ising_replicas* h, int32_t words_per_thread) {
    if (!h) return fail(ISING_EINVAL, "ising_replicas_set_plan: null handle");
    if (words_per_thread != 1 && words_per_thread != 2 && words_per_thread != 4)
        return fail(ISING_EINVAL, "ising_replicas_set_plan: words_per_thread must be 1, 2 or 4");
    h->wpt = words_per_thread;
    return ISING_OK;
}

}  // extern "C"
