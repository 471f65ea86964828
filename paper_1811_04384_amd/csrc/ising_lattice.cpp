// C ABI of the single-lattice path: one lattice, two half-sweep launches per
// sweep on the caller's stream (the plain one-lattice-per-launch form).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <limits>
#include <new>
#include <vector>

#include "ising_host.hpp"
#include "ising_launch.hpp"

using namespace ising;

struct ising_lattice {
    Geometry g;
    uint64_t seed = 0;
    uint64_t t = 0;  // absolute index of the next sweep
    uint64_t* W = nullptr;
    bool owns_W = false;
    hipStream_t stream = nullptr;
    int device = 0;
    int wpt = 4;
    int block = 256;
    Partial* partials = nullptr;  // per-wavefront bond/spin counts
    int64_t partial_cap = 0;
    int64_t* d_EM = nullptr;  // device scratch: E, M of ising_observables
    void* d_fin = nullptr;    // device scratch of the partial-sum reduction
    uint32_t* strip_pos = nullptr;    // drawn picks of the strip dynamics (allocated on first use)
    uint64_t* strip_codes = nullptr;  // their acceptance codes
    uint8_t* d_stage = nullptr;       // spin input/output staging, spin_stage_bytes(L)
    Moments* d_scan = nullptr;        // moment sums of up to kScanBlock temperatures of a scan
    // multi-sweep LDS tiles (tile_k = 0: one launch per half-sweep)
    int tile_k = 0, tile_cols = 0, tile_block = 256;
    int32_t n_tiles = 0;
    TileWork* d_tiles = nullptr;
    LatticeDesc* d_desc = nullptr;  // words and geometry of this lattice for the tile kernel
    Partial* d_tpart = nullptr;     // kTileMaxSweeps x n_tiles partial sums
    uint64_t* d_halo = nullptr;     // n_tiles x halo_stride: the tiles' halo copies (null: one tile)
    int64_t halo_stride = 0;
    // resident tiles with boundary exchange (res_cols = 0: off)
    int res_cols = 0, res_block = 256, res_sweeps = 0;
    int32_t n_res = 0;
    size_t res_lds = 0;
    PersistTile* d_res = nullptr;
    uint64_t* d_exch = nullptr;
    uint64_t* d_flags = nullptr;
    uint32_t* d_err = nullptr;      // 8 bytes: the error word and padding, cleared by a kernel
    uint32_t* h_err = nullptr;      // pinned copy of d_err, refreshed after every launch
    uint64_t res_wait = 0;          // bound of each wait, 100 MHz clock ticks
    Partial* d_rpart = nullptr;     // res_sweeps x n_res partial sums
    int64_t* d_rEM = nullptr;       // 2 x res_sweeps sample scratch (moments without a series)
};

// Temperatures of a scan whose moment sums are read back together.
constexpr int32_t kScanBlock = 256;

static int ensure_desc(ising_lattice* h);
static void free_resident(ising_lattice* h);

namespace ising {
std::string& last_error_ref() {
    thread_local std::string s;
    return s;
}

int read_spin_window(const uint64_t* W, const Geometry& g, int32_t r0, int32_t c0, int32_t nrows, int32_t ncols,
                     uint8_t* host, uint8_t* stage, size_t cap, hipStream_t s) {
    const int32_t chunk = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)nrows, cap / (size_t)ncols));
    for (int32_t i0 = 0; i0 < nrows; i0 += chunk) {
        const int32_t nr = std::min(chunk, nrows - i0);
        const int32_t r = (int32_t)(((int64_t)r0 + i0) % g.L);
        ISING_HIP(launch_unpack(W, g, r, c0, nr, ncols, stage, s));
        ISING_HIP(hipMemcpyAsync(host + (size_t)i0 * (size_t)ncols, stage, (size_t)nr * (size_t)ncols,
                                 hipMemcpyDeviceToHost, s));
    }
    ISING_HIP(hipStreamSynchronize(s));
    return ISING_OK;
}

int write_spins(uint64_t* W, const Geometry& g, const uint8_t* host, uint8_t* stage, size_t cap, hipStream_t s) {
    // at most N rows per piece, so that no word is written by two rows of one launch
    const int32_t chunk = (int32_t)std::max<size_t>(1, std::min<size_t>((size_t)g.N, cap / (size_t)g.L));
    for (int32_t r0 = 0; r0 < g.L; r0 += chunk) {
        const int32_t nr = std::min(chunk, g.L - r0);
        ISING_HIP(hipMemcpyAsync(stage, host + (size_t)r0 * (size_t)g.L, (size_t)nr * (size_t)g.L,
                                 hipMemcpyHostToDevice, s));
        ISING_HIP(launch_pack_rows(stage, g, r0, nr, W, s));
    }
    ISING_HIP(hipStreamSynchronize(s));
    return ISING_OK;
}
}  // namespace ising

extern "C" {

const char* ising_last_error(void) { return last_error_ref().c_str(); }

#ifndef ISING_SOURCE_HASH
#define ISING_SOURCE_HASH "unknown"
#endif
const char* ising_version(void) { return "ising-msc 1.0 (gfx950) src " ISING_SOURCE_HASH; }

int32_t ising_word_rows(int32_t L) { return valid_L(L) ? make_geometry(L).N : 0; }

size_t ising_required_bytes(int32_t L) {
    if (!valid_L(L)) return 0;
    const Geometry g = make_geometry(L);
    return (size_t)g.N * (size_t)g.L * sizeof(uint64_t);
}

int ising_thresholds(double T, uint32_t* t4, uint32_t* t8) {
    if (!valid_T(T)) return fail(ISING_EINVAL, "ising_thresholds: T must be finite and > 0 (got %g)", T);
    if (!t4 || !t8) return fail(ISING_EINVAL, "ising_thresholds: null output");
    thresholds_of(T, t4, t8);
    return ISING_OK;
}

static int64_t partials_needed(const Geometry& g) {
    // largest number of wavefronts any allowed plan launches
    int64_t m = observe_single_waves(g);
    for (int wpt : {1, 2, 4})
        for (int block = 64; block <= 256; block += 64) m = std::max(m, halfsweep_single_waves(g, wpt, block));
    return m;
}

static void release(ising_lattice* h) {
    if (!h) return;
    if (h->owns_W && h->W) (void)hipFree(h->W);
    if (h->partials) (void)hipFree(h->partials);
    if (h->d_EM) (void)hipFree(h->d_EM);
    if (h->d_fin) (void)hipFree(h->d_fin);
    if (h->strip_pos) (void)hipFree(h->strip_pos);
    if (h->strip_codes) (void)hipFree(h->strip_codes);
    if (h->d_stage) (void)hipFree(h->d_stage);
    if (h->d_scan) (void)hipFree(h->d_scan);
    if (h->d_tiles) (void)hipFree(h->d_tiles);
    if (h->d_desc) (void)hipFree(h->d_desc);
    if (h->d_tpart) (void)hipFree(h->d_tpart);
    if (h->d_halo) (void)hipFree(h->d_halo);
    if (h->d_res) (void)hipFree(h->d_res);
    if (h->d_exch) (void)hipFree(h->d_exch);
    if (h->d_flags) (void)hipFree(h->d_flags);
    if (h->d_err) (void)hipFree(h->d_err);
    if (h->h_err) (void)hipHostFree(h->h_err);
    if (h->d_rpart) (void)hipFree(h->d_rpart);
    if (h->d_rEM) (void)hipFree(h->d_rEM);
    delete h;
}

static int create_impl(int32_t L, uint64_t seed, int32_t init, void* dev_words, size_t bytes, void* stream,
                       ising_lattice** out) {
    if (!out) return fail(ISING_EINVAL, "ising_create: null output handle");
    *out = nullptr;
    if (!valid_L(L)) return fail(ISING_EINVAL, "ising_create: L must be even and in [4, %d] (got %d)", kMaxL, L);
    if (init != ISING_COLD && init != ISING_HOT) return fail(ISING_EINVAL, "ising_create: init must be 0 or 1");
    const size_t need = ising_required_bytes(L);
    if (dev_words) {
        if (bytes < need) return fail(ISING_EINVAL, "ising_create_in: buffer of %zu bytes < %zu needed", bytes, need);
        if (reinterpret_cast<uintptr_t>(dev_words) % 8) return fail(ISING_EINVAL, "ising_create_in: buffer not 8-byte aligned");
    }
    ising_lattice* h = new (std::nothrow) ising_lattice();
    if (!h) return fail(ISING_ENOMEM, "ising_create: host allocation failed");
    h->g = make_geometry(L);
    h->seed = seed;
    h->stream = (hipStream_t)stream;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        release(h);
        return hip_fail(e, "hipGetDevice");
    }
    if (dev_words) {
        h->W = (uint64_t*)dev_words;
    } else {
        e = hipMalloc(&h->W, need);
        if (e != hipSuccess) {
            h->W = nullptr;
            release(h);
            return fail(ISING_ENOMEM, "ising_create: hipMalloc of %zu bytes failed: %s", need, hipGetErrorString(e));
        }
        h->owns_W = true;
    }
    h->partial_cap = partials_needed(h->g);
    e = hipMalloc(&h->partials, (size_t)h->partial_cap * sizeof(Partial));
    if (e == hipSuccess) e = hipMalloc(&h->d_EM, 2 * sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&h->d_fin, finalize_scratch_bytes());
    if (e == hipSuccess) e = hipMalloc(&h->d_stage, spin_stage_bytes(L));
    if (e == hipSuccess) e = hipMalloc(&h->d_scan, sizeof(Moments) * kScanBlock);
    if (e == hipSuccess) e = hipMemsetAsync(h->d_fin, 0, finalize_scratch_bytes(), h->stream);
    if (e != hipSuccess) {
        release(h);
        return fail(ISING_ENOMEM, "ising_create: scratch allocation failed: %s", hipGetErrorString(e));
    }
    // default plan (measured on gfx950): from 64 Ki to 1 Mi words per colour
    // (L from about 1200 to 4600) one word per thread in 64-thread
    // workgroups is fastest (L = 4096: 1112 against 827 attempts/ns for two
    // words in 256-thread workgroups); above it the plans are within a few
    // per cent and two words per thread in 256-thread workgroups is kept;
    // below it (a handful of workgroups) 256-thread workgroups with one word
    // per thread
    const int64_t words = units_per_colour(h->g, 1);
    h->wpt = words < ((int64_t)1 << 20) ? 1 : 2;
    h->block = (words >= ((int64_t)1 << 16) && words < ((int64_t)1 << 20)) ? 64 : 256;
    e = launch_init(h->W, h->g, seed, init, h->stream);
    if (e != hipSuccess) {
        release(h);
        return hip_fail(e, "init kernel launch");
    }
    // Up to 7680 columns resident tiles are faster than one launch per
    // half-sweep at every size measured (attempts/ns, resident against
    // half-sweep launches, E/M every 10 sweeps: L = 64 1.7 / 0.7, 128
    // 5.2 / 2.9, 256 11.6 / 10.2, 512 47.6 / 45.0, 1024 190 / 152, 2048
    // 743 / 525, 4096 2182 / 1120, 5120 1687 / 1311, 7680 1815 / 1611).
    // Shapes: up to L = 192 the whole lattice in one workgroup, a thread per
    // word of a colour (a power of two, 64 to 1024); below L = 1024 bands
    // of 8 columns, 512 threads; from there bands of 2 ceil(L / 512)
    // columns (at most 256, one per compute unit), 1024 threads.  Above
    // 7680 a band no longer fits in LDS; where the tiles do not fit the
    // lattice keeps the half-sweep launches.
    if (L <= 7680) {
        int32_t w = 2 * ((L + 511) / 512), block = 1024;
        if (L <= 192) {
            const int64_t items = (int64_t)h->g.N * L / 2;
            w = L;
            block = 64;
            while (block < 1024 && block < items) block *= 2;
        } else if (L < 1024) {
            w = 8;
            block = 512;
        }
        if (ising_set_resident_tiles(h, w, block, 1000) != ISING_OK) last_error_ref().clear();
    }
    *out = h;
    return ISING_OK;
}

int ising_create(int32_t L, uint64_t seed, int32_t init, void* stream, ising_lattice** out) {
    return create_impl(L, seed, init, nullptr, 0, stream, out);
}

int ising_create_in(int32_t L, uint64_t seed, int32_t init, void* dev_words, size_t bytes, void* stream,
                    ising_lattice** out) {
    if (!dev_words) return fail(ISING_EINVAL, "ising_create_in: null device buffer");
    return create_impl(L, seed, init, dev_words, bytes, stream, out);
}

// Resident-tile flags follow the sweep counter: zero them when it goes back.
static int counter_set_back(ising_lattice* h) {
    if (h->d_flags) ISING_HIP(hipMemsetAsync(h->d_flags, 0, sizeof(uint64_t) * h->n_res, h->stream));
    return ISING_OK;
}

int ising_reset(ising_lattice* h, uint64_t seed, int32_t init) {
    if (!h) return fail(ISING_EINVAL, "ising_reset: null handle");
    if (init != ISING_COLD && init != ISING_HOT) return fail(ISING_EINVAL, "ising_reset: init must be 0 or 1");
    const int rc = counter_set_back(h);
    if (rc != ISING_OK) return rc;
    h->seed = seed;
    h->t = 0;
    ISING_HIP(launch_init(h->W, h->g, seed, init, h->stream));
    return ISING_OK;
}

int ising_destroy(ising_lattice* h) {
    if (!h) return ISING_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    release(h);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    return ISING_OK;
}

static SweepArgs sweep_args(const ising_lattice* h, uint64_t t, uint32_t t4, uint32_t t8) {
    SweepArgs a;
    a.L = h->g.L;
    a.N = h->g.N;
    a.istar = h->g.istar;
    a.sh_star = h->g.sh_star;
    a.t_lo = (uint32_t)t;
    a.t_hi = (uint32_t)(t >> 32);
    a.k0 = (uint32_t)h->seed;
    a.k1 = (uint32_t)(h->seed >> 32);
    a.t4 = t4;
    a.t8 = t8;
    return a;
}

// Enqueue n sweeps in multi-sweep tile launches of up to h->tile_k sweeps
// (the handle's words), starting at absolute sweep t0; the samples a launch
// takes are finalized right after it, in order.
static int enqueue_tile_sweeps(const ising_lattice* h, uint64_t t0, double T, int64_t n, int32_t every, int64_t* dev_E,
                               int64_t* dev_M, Moments* mom) {
    TileLaunch a = {};
    a.tiles = h->d_tiles;
    a.descs = h->d_desc;
    a.states = nullptr;
    a.k0 = (uint32_t)h->seed;
    a.k1 = (uint32_t)(h->seed >> 32);
    thresholds_of(T, &a.t4, &a.t8);
    a.sweep_off = 0;
    a.n_tiles = h->n_tiles;
    a.partials = h->d_tpart;
    for (int64_t done = 0; done < n;) {
        const int32_t kb = (int32_t)std::min<int64_t>(h->tile_k, n - done);
        uint32_t mask = 0;
        int32_t n_samples = 0;
        int64_t first = -1;
        for (int32_t j = 0; j < kb; ++j) {
            if (every > 0 && (done + j + 1) % every == 0) {
                mask |= 1u << j;
                if (first < 0) first = (done + j + 1) / every - 1;
                n_samples += 1;
            }
        }
        a.t0 = t0 + (uint64_t)done;
        a.K = kb;
        a.sample_mask = mask;
        ISING_HIP(launch_tiles(a, h->n_tiles, h->tile_block, tile_lds_bytes(h->g.L, h->g.N, h->tile_cols, kb),
                               h->d_halo, h->halo_stride, h->stream));
        if (n_samples)
            ISING_HIP(launch_finalize_samples(h->d_tpart, h->n_tiles, n_samples, h->g.L, dev_E, dev_M, first, mom,
                                              nullptr, h->stream));
        done += kb;
    }
    return ISING_OK;
}

// A wait of resident tiles longer than this (100 MHz clock ticks: one
// second) abandons the launch.
constexpr uint64_t kResidentWaitTicks = 100000000ull;

// Error left by an earlier resident-tile launch (its copy lands in pinned
// memory behind the launch); cleared once reported, the device word by a
// kernel on the handle's stream (ahead of any later launch, and valid under
// graph capture).
static int resident_error(ising_lattice* h) {
    if (h->h_err && *(volatile uint32_t*)h->h_err) {
        *(volatile uint32_t*)h->h_err = 0;
        ISING_HIP(launch_zero_words(reinterpret_cast<uint64_t*>(h->d_err), 1, h->stream));
        return fail(ISING_EHIP, "resident tiles: a launch waited too long for its neighbour tiles and was abandoned; "
                                "the lattice state is undefined");
    }
    return ISING_OK;
}

// Enqueue n sweeps as launches of resident tiles of up to h->res_sweeps
// sweeps each; each launch's samples are reduced right behind it.
static int enqueue_resident_sweeps(ising_lattice* h, uint64_t t0, double T, int64_t n, int32_t every, int64_t* dev_E,
                                   int64_t* dev_M, Moments* mom) {
    PersistLaunch a = {};
    a.tiles = h->d_res;
    a.descs = h->d_desc;
    a.k0 = (uint32_t)h->seed;
    a.k1 = (uint32_t)(h->seed >> 32);
    thresholds_of(T, &a.t4, &a.t8);
    a.every = every;
    a.n_tiles = h->n_res;
    a.partials = h->d_rpart;
    a.exch = h->d_exch;
    a.exch_tile_words = 4 * (int64_t)h->g.N;
    a.flags = h->d_flags;
    a.error = h->d_err;
    a.wait_ticks = h->res_wait ? h->res_wait : kResidentWaitTicks;
    for (int64_t done = 0; done < n;) {
        const int32_t kb = (int32_t)std::min<int64_t>(h->res_sweeps, n - done);
        a.t0 = t0 + (uint64_t)done;
        a.K = kb;
        a.sample_base = done;
        ISING_HIP(resident_gate(h->device, h->stream,
                                [&] { return launch_persist(a, h->n_res, h->res_block, h->res_lds, h->stream); }));
        const int64_t n_samples = every > 0 ? (done + kb) / every - done / every : 0;
        if (n_samples > 0) {
            const int64_t idx0 = done / every;  // series index of the launch's first sample
            int64_t* E = dev_E ? dev_E + idx0 : h->d_rEM;
            int64_t* M = dev_M ? dev_M + idx0 : h->d_rEM + h->res_sweeps;
            ISING_HIP(launch_samples(h->d_rpart, h->n_res, (int32_t)n_samples, h->g.L, E, M, mom, h->stream));
        }
        ISING_HIP(hipMemcpyAsync(h->h_err, h->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
        done += kb;
    }
    return ISING_OK;
}

// Enqueue n sweeps of lattice words W (the handle's or a scratch copy)
// starting at absolute sweep t0.
static int enqueue_sweeps(const ising_lattice* h, uint64_t* W, uint64_t t0, double T, int64_t n, int32_t every,
                          int64_t* dev_E, int64_t* dev_M, Moments* mom, int wpt, int block) {
    if (h->res_cols > 0 && W == h->W)
        return enqueue_resident_sweeps(const_cast<ising_lattice*>(h), t0, T, n, every, dev_E, dev_M, mom);
    if (h->tile_k > 0 && W == h->W) return enqueue_tile_sweeps(h, t0, T, n, every, dev_E, dev_M, mom);
    uint32_t t4, t8;
    thresholds_of(T, &t4, &t8);
    for (int64_t k = 1; k <= n; ++k) {
        const SweepArgs a = sweep_args(h, t0 + (uint64_t)(k - 1), t4, t8);
        ISING_HIP(launch_halfsweep_single(wpt, block, W, a, 0, nullptr, nullptr, h->stream));
        const bool meas = every > 0 && k % every == 0;
        int64_t nw = 0;
        ISING_HIP(launch_halfsweep_single(wpt, block, W, a, 1, meas ? h->partials : nullptr, &nw, h->stream));
        if (meas)
            ISING_HIP(launch_finalize_single(h->partials, nw, h->g.L, dev_E, dev_M, k / every - 1, nullptr, mom,
                                             h->d_fin, h->stream));
    }
    return ISING_OK;
}

static int sweep_impl(ising_lattice* h, double T, int64_t n, int32_t every, int64_t* dev_E, int64_t* dev_M,
                      Moments* mom = nullptr) {
    if (!h) return fail(ISING_EINVAL, "ising_sweep: null handle");
    if (!valid_T(T)) return fail(ISING_EINVAL, "ising_sweep: T must be finite and > 0 (got %g)", T);
    if (n < 0) return fail(ISING_EINVAL, "ising_sweep: n_sweeps must be >= 0");
    int rc = resident_error(h);
    if (rc != ISING_OK) return rc;
    rc = enqueue_sweeps(h, h->W, h->t, T, n, every, dev_E, dev_M, mom, h->wpt, h->block);
    if (rc != ISING_OK) return rc;
    h->t += (uint64_t)n;
    return ISING_OK;
}

int ising_sweep(ising_lattice* h, double T, int64_t n_sweeps) { return sweep_impl(h, T, n_sweeps, 0, nullptr, nullptr); }

int ising_sweep_measure(ising_lattice* h, double T, int64_t n_sweeps, int32_t every, int64_t* dev_E,
                        int64_t* dev_M) {
    if (every < 1) return fail(ISING_EINVAL, "ising_sweep_measure: every must be >= 1");
    if (!dev_E || !dev_M) return fail(ISING_EINVAL, "ising_sweep_measure: null series pointer");
    return sweep_impl(h, T, n_sweeps, every, dev_E, dev_M);
}

int ising_sweep_moments(ising_lattice* h, double T, int64_t n_sweeps, int32_t every, ising_moments* dev_acc) {
    if (every < 1) return fail(ISING_EINVAL, "ising_sweep_moments: every must be >= 1");
    if (!dev_acc) return fail(ISING_EINVAL, "ising_sweep_moments: null accumulator");
    return sweep_impl(h, T, n_sweeps, every, nullptr, nullptr, reinterpret_cast<Moments*>(dev_acc));
}

int ising_scan(ising_lattice* h, int32_t n_T, const double* T, int64_t therm, int64_t meas, int32_t every,
               ising_moments* out) {
    if (!h) return fail(ISING_EINVAL, "ising_scan: null handle");
    if (n_T < 0 || therm < 0 || meas < 0 || every < 1)
        return fail(ISING_EINVAL, "ising_scan: need n_T, therm, meas >= 0 and every >= 1");
    if (n_T == 0) return ISING_OK;
    if (!T || !out) return fail(ISING_EINVAL, "ising_scan: null array");
    for (int32_t i = 0; i < n_T; ++i)
        if (!valid_T(T[i])) return fail(ISING_EINVAL, "ising_scan: T[%d] = %g is not finite and > 0", i, T[i]);
    // blocks of up to kScanBlock temperatures accumulate into the handle's
    // moment array and are read back together
    for (int32_t j0 = 0; j0 < n_T; j0 += kScanBlock) {
        const int32_t nb = std::min(kScanBlock, n_T - j0);
        ISING_HIP(hipMemsetAsync(h->d_scan, 0, sizeof(Moments) * (size_t)nb, h->stream));
        for (int32_t i = 0; i < nb; ++i) {
            int rc = sweep_impl(h, T[j0 + i], therm, 0, nullptr, nullptr);
            if (rc == ISING_OK) rc = sweep_impl(h, T[j0 + i], meas, every, nullptr, nullptr, h->d_scan + i);
            if (rc != ISING_OK) {
                (void)hipStreamSynchronize(h->stream);
                return rc;
            }
        }
        ISING_HIP(hipMemcpyAsync(out + j0, h->d_scan, sizeof(Moments) * (size_t)nb, hipMemcpyDeviceToHost, h->stream));
        ISING_HIP(hipStreamSynchronize(h->stream));
    }
    return ISING_OK;
}

// Largest number of picks one strip may apply in one phase (bounds the run
// time of one thread).
constexpr int64_t kStripPickLimit = int64_t(1) << 22;
// Picks drawn ahead per launch pair of the two-step strip path (all strips
// together; 12 bytes each), and the largest LDS footprint of one strip for
// which that path is used.
constexpr int64_t kStripBufEntries = int64_t(1) << 22;
constexpr size_t kStripChainLdsMax = 16 * 1024;

static int strip_phase(ising_lattice* h, const StripArgs& a) {
    if (strip_chain_lds_bytes(a) > kStripChainLdsMax || strip_apply_lds_bytes(a, 1) > kStripLdsBytes) {
        ISING_HIP(launch_strip_phase(h->W, a, h->stream));
        return ISING_OK;
    }
    if (!h->strip_pos) {
        ISING_HIP(hipMalloc(&h->strip_pos, sizeof(uint32_t) * kStripBufEntries));
        hipError_t e = hipMalloc(&h->strip_codes, sizeof(uint64_t) * kStripBufEntries);
        if (e != hipSuccess) {
            (void)hipFree(h->strip_pos);
            h->strip_pos = nullptr;
            return hip_fail(e, "hipMalloc");
        }
    }
    const uint32_t chunk = (uint32_t)std::max<int64_t>(1, kStripBufEntries / a.strips);
    for (uint32_t k0 = 0; k0 < a.picks; k0 += chunk) {
        const uint32_t n_k = std::min(chunk, a.picks - k0);
        ISING_HIP(launch_strip_draws(a, k0, n_k, h->strip_pos, h->strip_codes, h->stream));
        ISING_HIP(launch_strip_apply(h->W, a, n_k, h->strip_pos, h->strip_codes, h->stream));
    }
    return ISING_OK;
}

int ising_random_iterations(ising_lattice* h, double T, int32_t strip_cols, int64_t n_iterations, int32_t every,
                            int64_t* dev_E, int64_t* dev_M, ising_moments* dev_acc) {
    if (!h) return fail(ISING_EINVAL, "ising_random_iterations: null handle");
    if (!valid_T(T)) return fail(ISING_EINVAL, "ising_random_iterations: T must be finite and > 0 (got %g)", T);
    const int32_t L = h->g.L, N = h->g.N;
    if (strip_cols < 2 || strip_cols > L || L % strip_cols != 0)
        return fail(ISING_EINVAL, "ising_random_iterations: strip_cols %d must be >= 2 and divide L = %d",
                    strip_cols, L);
    const int64_t picks1 = 10 * (int64_t)N * (strip_cols - strip_cols / 2);
    if (picks1 > kStripPickLimit)
        return fail(ISING_EINVAL, "ising_random_iterations: %lld picks per strip and phase exceed %lld",
                    (long long)picks1, (long long)kStripPickLimit);
    if (n_iterations < 0 || every < 0) return fail(ISING_EINVAL, "ising_random_iterations: negative count");
    if ((dev_E || dev_M || dev_acc) && every == 0)
        return fail(ISING_EINVAL, "ising_random_iterations: outputs need every >= 1");
    if ((h->t + (uint64_t)n_iterations) >> 56)
        return fail(ISING_EINVAL, "ising_random_iterations: iteration index beyond 2^56");
    uint32_t t4, t8;
    thresholds_of(T, &t4, &t8);
    StripArgs a;
    a.L = L;
    a.N = N;
    a.istar = h->g.istar;
    a.sh_star = h->g.sh_star;
    a.S = strip_cols;
    a.strips = L / strip_cols;
    a.k0 = (uint32_t)h->seed;
    a.k1 = (uint32_t)(h->seed >> 32);
    a.t4 = t4;
    a.t8 = t8;
    for (int64_t k = 1; k <= n_iterations; ++k) {
        const uint64_t t = h->t + (uint64_t)(k - 1);
        a.t_lo = (uint32_t)t;
        a.t_hi = (uint32_t)(t >> 32);
        for (uint32_t ph = 0; ph < 2; ++ph) {
            a.phase = ph;
            a.off = ph == 0 ? 0 : strip_cols / 2;
            a.width = ph == 0 ? strip_cols / 2 : strip_cols - strip_cols / 2;
            a.picks = (uint32_t)(10 * (int64_t)N * a.width);
            const int rc = strip_phase(h, a);
            if (rc != ISING_OK) return rc;
        }
        if (every > 0 && k % every == 0) {
            int64_t nw = 0;
            ISING_HIP(launch_observe_single(h->W, h->g, h->partials, &nw, h->stream));
            ISING_HIP(launch_finalize_single(h->partials, nw, L, dev_E, dev_M, k / every - 1, nullptr,
                                             reinterpret_cast<Moments*>(dev_acc), h->d_fin, h->stream));
        }
    }
    h->t += (uint64_t)n_iterations;
    return ISING_OK;
}

int ising_thermodynamics(const ising_moments* m, int32_t L, double T, ising_thermo* out) {
    if (!m || !out) return fail(ISING_EINVAL, "ising_thermodynamics: null argument");
    if (!valid_L(L)) return fail(ISING_EINVAL, "ising_thermodynamics: invalid L %d", L);
    if (!valid_T(T)) return fail(ISING_EINVAL, "ising_thermodynamics: T must be finite and > 0 (got %g)", T);
    if (m->n_samples < 1) return fail(ISING_EINVAL, "ising_thermodynamics: no samples");
    typedef long double ld;
    const ld two64 = 18446744073709551616.0L;
    const ld n = (ld)m->n_samples, spins = (ld)L * (ld)L;
    const ld E1 = (ld)m->sum_E / n;
    const ld E2 = ((ld)m->sum_E2[0] + (ld)m->sum_E2[1] * two64) / n;
    const ld A1 = (ld)m->sum_absM / n;
    const ld M2 = ((ld)m->sum_M2[0] + (ld)m->sum_M2[1] * two64) / n;
    const ld M4 = ((ld)m->sum_M4[0] + ((ld)m->sum_M4[1] + (ld)m->sum_M4[2] * two64) * two64) / n;
    const ld t = (ld)T;
    out->e = (double)(E1 / spins);
    out->c = (double)((E2 - E1 * E1) / (t * t * spins));
    out->abs_m = (double)(A1 / spins);
    out->chi = (double)((M2 - A1 * A1) / (t * spins));
    out->binder = M2 > 0 ? (double)(1.0L - M4 / (3.0L * M2 * M2)) : std::numeric_limits<double>::quiet_NaN();
    return ISING_OK;
}

int ising_observables(ising_lattice* h, int64_t* E, int64_t* M) {
    if (!h || !E || !M) return fail(ISING_EINVAL, "ising_observables: null argument");
    int64_t nw = 0;
    ISING_HIP(launch_observe_single(h->W, h->g, h->partials, &nw, h->stream));
    ISING_HIP(launch_finalize_single(h->partials, nw, h->g.L, nullptr, nullptr, 0, h->d_EM, nullptr, h->d_fin,
                                     h->stream));
    int64_t em[2];
    ISING_HIP(hipMemcpyAsync(em, h->d_EM, sizeof em, hipMemcpyDeviceToHost, h->stream));
    ISING_HIP(hipStreamSynchronize(h->stream));
    int rc = resident_error(h);
    if (rc != ISING_OK) return rc;
    *E = em[0];
    *M = em[1];
    return ISING_OK;
}

int ising_get_spins_region(ising_lattice* h, int32_t r0, int32_t c0, int32_t nrows, int32_t ncols, uint8_t* host) {
    if (!h || !host) return fail(ISING_EINVAL, "ising_get_spins_region: null argument");
    const int32_t L = h->g.L;
    if (nrows < 1 || ncols < 1 || nrows > L || ncols > L)
        return fail(ISING_EINVAL, "ising_get_spins_region: window %dx%d outside 1..L=%d", nrows, ncols, L);
    const int32_t rr = (int32_t)(((int64_t)r0 % L + L) % L), cc = (int32_t)(((int64_t)c0 % L + L) % L);
    return read_spin_window(h->W, h->g, rr, cc, nrows, ncols, host, h->d_stage, spin_stage_bytes(L), h->stream);
}

int ising_get_spins(ising_lattice* h, uint8_t* host) {
    if (!h) return fail(ISING_EINVAL, "ising_get_spins: null handle");
    return ising_get_spins_region(h, 0, 0, h->g.L, h->g.L, host);
}

int ising_set_spins(ising_lattice* h, const uint8_t* host) {
    if (!h || !host) return fail(ISING_EINVAL, "ising_set_spins: null argument");
    return write_spins(h->W, h->g, host, h->d_stage, spin_stage_bytes(h->g.L), h->stream);
}

int ising_get_sweep_count(ising_lattice* h, uint64_t* t) {
    if (!h || !t) return fail(ISING_EINVAL, "ising_get_sweep_count: null argument");
    *t = h->t;
    return ISING_OK;
}

int ising_set_sweep_count(ising_lattice* h, uint64_t t) {
    if (!h) return fail(ISING_EINVAL, "ising_set_sweep_count: null handle");
    if (t < h->t) {
        const int rc = counter_set_back(h);
        if (rc != ISING_OK) return rc;
    }
    h->t = t;
    return ISING_OK;
}

int ising_words(ising_lattice* h, void** dev_words, size_t* bytes) {
    if (!h || !dev_words || !bytes) return fail(ISING_EINVAL, "ising_words: null argument");
    *dev_words = h->W;
    *bytes = ising_required_bytes(h->g.L);
    return ISING_OK;
}

int ising_set_plan(ising_lattice* h, int32_t wpt, int32_t block) {
    if (!h) return fail(ISING_EINVAL, "ising_set_plan: null handle");
    if (wpt != 1 && wpt != 2 && wpt != 4) return fail(ISING_EINVAL, "ising_set_plan: words_per_thread must be 1, 2 or 4");
    if (!valid_block(block, 256)) return fail(ISING_EINVAL, "ising_set_plan: block must be 64, 128, 192 or 256");
    h->wpt = wpt;
    h->block = block;
    return ISING_OK;
}

int ising_get_plan(ising_lattice* h, int32_t* wpt, int32_t* block) {
    if (!h || !wpt || !block) return fail(ISING_EINVAL, "ising_get_plan: null argument");
    *wpt = h->wpt;
    *block = h->block;
    return ISING_OK;
}

int ising_set_tiling(ising_lattice* h, int32_t sweeps_per_launch, int32_t tile_cols, int32_t block) {
    if (!h) return fail(ISING_EINVAL, "ising_set_tiling: null handle");
    const int32_t L = h->g.L, N = h->g.N, K = sweeps_per_launch;
    if (K == 0) {
        h->tile_k = 0;
        return ISING_OK;
    }
    if (K < 0 || K > kTileMaxSweeps)
        return fail(ISING_EINVAL, "ising_set_tiling: sweeps_per_launch must be in [0, %d]", kTileMaxSweeps);
    if (tile_cols < 2 || tile_cols % 2) return fail(ISING_EINVAL, "ising_set_tiling: tile_cols must be even and >= 2");
    if (!valid_block(block, 1024)) return fail(ISING_EINVAL, "ising_set_tiling: block must be a multiple of 64 in [64, 1024]");
    const bool whole = tile_cols >= L;
    if (!whole && tile_cols + 4 * K > L)
        return fail(ISING_EINVAL, "ising_set_tiling: a tile of %d columns with halos of %d exceeds L = %d (use tile_cols >= L)",
                    tile_cols, 2 * K, L);
    const size_t need = tile_lds_bytes(L, N, whole ? L : tile_cols, K);
    const size_t have = tile_lds_limit(h->device);
    if (need > have)
        return fail(ISING_EINVAL, "ising_set_tiling: a tile needs %zu bytes of LDS, %zu available", need, have);
    std::vector<TileWork> tiles;
    const int32_t w = whole ? L : tile_cols;
    for (int32_t c0 = 0; c0 < L; c0 += w) tiles.push_back({0, c0, std::min(w, L - c0), (int32_t)tiles.size()});
    ISING_HIP(hipStreamSynchronize(h->stream));  // earlier launches may still read the old tables
    if (h->d_tiles) (void)hipFree(h->d_tiles);
    if (h->d_tpart) (void)hipFree(h->d_tpart);
    if (h->d_halo) (void)hipFree(h->d_halo);
    h->d_tiles = nullptr;
    h->d_tpart = nullptr;
    h->d_halo = nullptr;
    h->halo_stride = 0;
    h->tile_k = 0;
    ISING_HIP(allow_tile_lds(h->device));
    free_resident(h);  // resident tiles off
    const int rc = ensure_desc(h);
    if (rc != ISING_OK) return rc;
    ISING_HIP(hipMalloc(&h->d_tiles, sizeof(TileWork) * tiles.size()));
    ISING_HIP(hipMemcpy(h->d_tiles, tiles.data(), sizeof(TileWork) * tiles.size(), hipMemcpyHostToDevice));
    ISING_HIP(hipMalloc(&h->d_tpart, sizeof(Partial) * tiles.size() * kTileMaxSweeps));
    if (!whole) {
        const int64_t stride = tile_halo_stride(N, K);
        ISING_HIP(hipMalloc(&h->d_halo, sizeof(uint64_t) * tiles.size() * (size_t)stride));
        h->halo_stride = stride;
    }
    h->n_tiles = (int32_t)tiles.size();
    h->tile_k = K;
    h->tile_cols = w;
    h->tile_block = block;
    return ISING_OK;
}

static int ensure_desc(ising_lattice* h) {
    if (h->d_desc) return ISING_OK;
    LatticeDesc d = {};
    d.W = h->W;
    d.L = h->g.L;
    d.N = h->g.N;
    d.istar = h->g.istar;
    d.sh_star = h->g.sh_star;
    d.sweep_limit = 0x7FFFFFFF;
    ISING_HIP(hipMalloc(&h->d_desc, sizeof(LatticeDesc)));
    ISING_HIP(hipMemcpy(h->d_desc, &d, sizeof d, hipMemcpyHostToDevice));
    return ISING_OK;
}

static void free_resident(ising_lattice* h) {
    if (h->d_res) (void)hipFree(h->d_res);
    if (h->d_exch) (void)hipFree(h->d_exch);
    if (h->d_flags) (void)hipFree(h->d_flags);
    if (h->d_rpart) (void)hipFree(h->d_rpart);
    if (h->d_rEM) (void)hipFree(h->d_rEM);
    h->d_res = nullptr;
    h->d_exch = nullptr;
    h->d_flags = nullptr;
    h->d_rpart = nullptr;
    h->d_rEM = nullptr;
    h->res_cols = 0;
    h->n_res = 0;
}

// The resident tiles of one lattice (interior width w, the last one
// narrower), indexed by workgroup: consecutive workgroups are dealt to the
// 8 XCDs in turn, so when the tile count is a multiple of 8 tile t goes to
// workgroup 8 (t mod m) + t div m (m = count / 8) and every XCD holds a run
// of neighbouring tiles, which then trade their boundary words inside one
// XCD except at the ends of the runs.  part_base offsets the partial slots.
static std::vector<PersistTile> resident_tile_table(int32_t lattice, int32_t L, int32_t w, int32_t part_base) {
    int32_t n = 0;
    for (int32_t c0 = 0; c0 < L; c0 += w) ++n;
    const bool spread = n % 8 == 0;
    const int32_t m = n / 8;
    auto block_of = [&](int32_t t) { return spread ? 8 * (t % m) + t / m : t; };
    std::vector<PersistTile> tiles(n);
    for (int32_t t = 0; t < n; ++t) {
        const int32_t c0 = t * w;
        tiles[block_of(t)] = {lattice, c0, std::min(w, L - c0), block_of((t + n - 1) % n), block_of((t + 1) % n),
                              part_base + t};
    }
    return tiles;
}

// Largest number of sweeps of one resident-tile launch.
constexpr int32_t kResidentMaxSweeps = 4096;

int ising_set_resident_tiles(ising_lattice* h, int32_t tile_cols, int32_t block, int32_t max_sweeps) {
    if (!h) return fail(ISING_EINVAL, "ising_set_resident_tiles: null handle");
    ISING_HIP(hipStreamSynchronize(h->stream));  // earlier launches may still read the old tables
    int rc = resident_error(h);
    if (rc != ISING_OK) return rc;
    if (tile_cols == 0) {
        free_resident(h);
        return ISING_OK;
    }
    const int32_t L = h->g.L, N = h->g.N;
    if (tile_cols < 2 || tile_cols % 2) return fail(ISING_EINVAL, "ising_set_resident_tiles: tile_cols must be even and >= 2");
    if (!valid_block(block, 1024))
        return fail(ISING_EINVAL, "ising_set_resident_tiles: block must be a multiple of 64 in [64, 1024]");
    if (max_sweeps < 1 || max_sweeps > kResidentMaxSweeps)
        return fail(ISING_EINVAL, "ising_set_resident_tiles: max_sweeps must be in [1, %d]", kResidentMaxSweeps);
    const int32_t w = tile_cols >= L ? L : tile_cols;
    const size_t lds = persist_lds_bytes(L, N, w, block);
    if (lds > persist_lds_limit(h->device))
        return fail(ISING_EINVAL, "ising_set_resident_tiles: a tile needs %zu bytes of LDS, %zu available", lds,
                    persist_lds_limit(h->device));
    ISING_HIP(allow_persist_lds(h->device));
    std::vector<PersistTile> tiles = resident_tile_table(0, L, w, 0);
    const int32_t n = (int32_t)tiles.size();
    int64_t capacity = 0;
    ISING_HIP(persist_capacity(block, lds, h->device, &capacity));
    if (n > capacity)
        return fail(ISING_EINVAL, "ising_set_resident_tiles: %d tiles of %d threads and %zu bytes of LDS exceed the %lld "
                    "the device holds at once", n, block, lds, (long long)capacity);
    free_resident(h);
    h->tile_k = 0;  // multi-sweep halo tiles off
    rc = ensure_desc(h);
    if (rc != ISING_OK) return rc;
    hipError_t e = hipMalloc(&h->d_res, sizeof(PersistTile) * n);
    if (e == hipSuccess) e = hipMemcpy(h->d_res, tiles.data(), sizeof(PersistTile) * n, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&h->d_exch, sizeof(uint64_t) * 4 * (size_t)N * n);
    if (e == hipSuccess) e = hipMalloc(&h->d_flags, sizeof(uint64_t) * n);
    if (e == hipSuccess) e = hipMemset(h->d_flags, 0, sizeof(uint64_t) * n);
    if (e == hipSuccess && !h->d_err) e = hipMalloc(&h->d_err, sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(h->d_err, 0, sizeof(uint64_t));
    if (e == hipSuccess && !h->h_err) e = hipHostMalloc(&h->h_err, sizeof(uint32_t), hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&h->d_rpart, sizeof(Partial) * (size_t)max_sweeps * n);
    if (e == hipSuccess) e = hipMalloc(&h->d_rEM, sizeof(int64_t) * 2 * (size_t)max_sweeps);
    if (e != hipSuccess) {
        free_resident(h);
        return hip_fail(e, "ising_set_resident_tiles");
    }
    *h->h_err = 0;
    h->n_res = n;
    h->res_cols = w;
    h->res_block = block;
    h->res_sweeps = max_sweeps;
    h->res_lds = lds;
    return ISING_OK;
}

int ising_set_resident_wait(ising_lattice* h, uint64_t ticks) {
    if (!h) return fail(ISING_EINVAL, "ising_set_resident_wait: null handle");
    if (ticks > kResidentWaitTicks * 60)
        return fail(ISING_EINVAL, "ising_set_resident_wait: at most %llu ticks (one minute)",
                    (unsigned long long)(kResidentWaitTicks * 60));
    h->res_wait = ticks;  // 0: the default
    return ISING_OK;
}

int ising_get_resident_tiles(ising_lattice* h, int32_t* tile_cols, int32_t* block, int32_t* max_sweeps) {
    if (!h || !tile_cols || !block || !max_sweeps) return fail(ISING_EINVAL, "ising_get_resident_tiles: null argument");
    *tile_cols = h->res_cols;
    *block = h->res_cols ? h->res_block : 0;
    *max_sweeps = h->res_cols ? h->res_sweeps : 0;
    return ISING_OK;
}

int ising_get_tiling(ising_lattice* h, int32_t* sweeps_per_launch, int32_t* tile_cols, int32_t* block) {
    if (!h || !sweeps_per_launch || !tile_cols || !block) return fail(ISING_EINVAL, "ising_get_tiling: null argument");
    *sweeps_per_launch = h->tile_k;
    *tile_cols = h->tile_k ? h->tile_cols : 0;
    *block = h->tile_k ? h->tile_block : 0;
    return ISING_OK;
}

int ising_synchronize(ising_lattice* h) {
    if (!h) return fail(ISING_EINVAL, "ising_synchronize: null handle");
    ISING_HIP(hipStreamSynchronize(h->stream));
    return resident_error(h);
}

int ising_autotune(ising_lattice* h, double T, double* best_ms_per_sweep) {
    if (!h) return fail(ISING_EINVAL, "ising_autotune: null handle");
    if (!valid_T(T)) return fail(ISING_EINVAL, "ising_autotune: T must be finite and > 0");
    const size_t bytes = ising_required_bytes(h->g.L);
    uint64_t* scratch = nullptr;
    ISING_HIP(hipMalloc(&scratch, bytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = ISING_OK;
    double best = 1e300;
    int best_wpt = h->wpt, best_block = h->block;
    const double work = (double)h->g.L * (double)h->g.L;
    const int64_t n_time = std::max<int64_t>(2, std::min<int64_t>(50, (int64_t)(2e9 / work)));
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemcpyAsync(scratch, h->W, bytes, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) rc = hip_fail(e, "ising_autotune setup");
    const int wpts[3] = {1, 2, 4};
    const int blocks[3] = {64, 128, 256};
    for (int wi = 0; wi < 3 && rc == ISING_OK; ++wi) {
        for (int bi = 0; bi < 3 && rc == ISING_OK; ++bi) {
            rc = enqueue_sweeps(h, scratch, h->t, T, 1, 0, nullptr, nullptr, nullptr, wpts[wi], blocks[bi]);  // warm-up
            if (rc != ISING_OK) break;
            e = hipEventRecord(e0, h->stream);
            if (e == hipSuccess)
                rc = enqueue_sweeps(h, scratch, h->t, T, n_time, 0, nullptr, nullptr, nullptr, wpts[wi], blocks[bi]);
            if (rc != ISING_OK) break;
            if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = hip_fail(e, "ising_autotune timing");
                break;
            }
            const double per = ms / (double)n_time;
            if (per < best) {
                best = per;
                best_wpt = wpts[wi];
                best_block = blocks[bi];
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(h->stream);
    (void)hipFree(scratch);
    if (rc != ISING_OK) return rc;
    h->wpt = best_wpt;
    h->block = best_block;
    if (best_ms_per_sweep) *best_ms_per_sweep = best;
    return ISING_OK;
}

}  // extern "C"
