// ising_sweep_measure_static: the sweep with fused E/M samples of
// ising_sweep_measure on a caller's word buffer, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops).
// Its scratch -- the per-wavefront partial sums of a sampled half-sweep and
// the state of their reduction -- is a file-scope device array of fixed
// size, which every call on a device shares.  Its device address is looked
// up once per device (hipGetSymbolAddress) and used from then on; the
// array's name in host code is only a stand-in for the symbol.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "ising_host.hpp"
#include "ising_launch.hpp"

using namespace ising;

namespace {

// 2 MiB of partial sums (262,144 wavefronts: every lattice up to L = 32768 in
// the default launch shape) and the reduction's block sums and ticket.
constexpr size_t kStaticPartials = size_t(1) << 18;
constexpr size_t kStaticScratchBytes = kStaticPartials * sizeof(Partial) + 8192;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up once).
int scratch_on_device(int device, unsigned char** out) {
    if (device < 0 || device >= kMaxDevices) return fail(ISING_EINVAL, "ising_sweep_measure_static: device %d", device);
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[device]);
    return ISING_OK;
}

}  // namespace

extern "C" {

int ising_sweep_measure_static(void* dev_words, size_t bytes, int32_t L, uint64_t seed, uint64_t t0, double T,
                               int64_t n_sweeps, int32_t every, int64_t* dev_E, int64_t* dev_M, void* stream) {
    if (!valid_L(L)) return fail(ISING_EINVAL, "ising_sweep_measure_static: L must be even and in [4, %d]", kMaxL);
    if (!dev_words || !dev_E || !dev_M) return fail(ISING_EINVAL, "ising_sweep_measure_static: null pointer");
    const Geometry g = make_geometry(L);
    const size_t need = (size_t)g.N * (size_t)g.L * sizeof(uint64_t);
    if (bytes < need)
        return fail(ISING_EINVAL, "ising_sweep_measure_static: buffer of %zu bytes < %zu needed", bytes, need);
    if (reinterpret_cast<uintptr_t>(dev_words) % 8)
        return fail(ISING_EINVAL, "ising_sweep_measure_static: buffer not 8-byte aligned");
    if (!valid_T(T)) return fail(ISING_EINVAL, "ising_sweep_measure_static: T must be finite and > 0 (got %g)", T);
    if (n_sweeps < 0 || every < 1)
        return fail(ISING_EINVAL, "ising_sweep_measure_static: need n_sweeps >= 0 and every >= 1");
    // the launch shape of ising_create's default plan (one launch per
    // half-sweep); its sampled half-sweeps must fit the partial sums
    const int64_t words = units_per_colour(g, 1);
    const int wpt = words < ((int64_t)1 << 20) ? 1 : 2;
    const int block = (words >= ((int64_t)1 << 16) && words < ((int64_t)1 << 20)) ? 64 : 256;
    const int64_t waves = halfsweep_single_waves(g, wpt, block);
    if (waves > (int64_t)kStaticPartials)
        return fail(ISING_EINVAL,
                    "ising_sweep_measure_static: L = %d needs %lld partial sums, more than the %zu of the static "
                    "scratch (L up to 32768 fits)", L, (long long)waves, kStaticPartials);
    int device = 0;
    ISING_HIP(hipGetDevice(&device));
    unsigned char* base = nullptr;
    int rc = scratch_on_device(device, &base);
    if (rc != ISING_OK) return rc;
    Partial* partials = reinterpret_cast<Partial*>(base);
    void* fin = base + kStaticPartials * sizeof(Partial);
    hipStream_t s = (hipStream_t)stream;
    // the reduction's ticket must start at zero; a kernel clears it (this
    // entry point may be captured into a graph)
    ISING_HIP(launch_zero_words(reinterpret_cast<uint64_t*>(fin), finalize_scratch_bytes() / 8, s));
    uint32_t t4, t8;
    thresholds_of(T, &t4, &t8);
    SweepArgs a;
    a.L = g.L;
    a.N = g.N;
    a.istar = g.istar;
    a.sh_star = g.sh_star;
    a.k0 = (uint32_t)seed;
    a.k1 = (uint32_t)(seed >> 32);
    a.t4 = t4;
    a.t8 = t8;
    uint64_t* W = static_cast<uint64_t*>(dev_words);
    for (int64_t k = 1; k <= n_sweeps; ++k) {
        const uint64_t t = t0 + (uint64_t)(k - 1);
        a.t_lo = (uint32_t)t;
        a.t_hi = (uint32_t)(t >> 32);
        ISING_HIP(launch_halfsweep_single(wpt, block, W, a, 0, nullptr, nullptr, s));
        const bool meas = k % every == 0;
        int64_t nw = 0;
        ISING_HIP(launch_halfsweep_single(wpt, block, W, a, 1, meas ? partials : nullptr, &nw, s));
        if (meas)
            ISING_HIP(launch_finalize_single(partials, nw, g.L, dev_E, dev_M, k / every - 1, nullptr, nullptr, fin, s));
    }
    return ISING_OK;
}

}  // extern "C"
