// gfx950 kernels of the multi-spin-coded checkerboard Metropolis sweep and
// their launchers.  See ising_device.hpp for the word layout and the
// per-word update.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ising_device.hpp"
#include "ising_launch.hpp"
#include "ising_moments.hpp"

namespace ising {

namespace {

constexpr int kTiledMaxBlock = 256;
constexpr int kResidentMaxBlock = 1024;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// ---------------------------------------------------------------------------
// Initial state.  One thread per word.  Hot start: a site is up iff its
// stream-0 draw at t = 0 is below 2^31 (the random initialisation of
// Section 5.1 with a reproducible generator).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_init(uint64_t* __restrict__ W, Geometry g, uint32_t k0, uint32_t k1,
                                              int hot) {
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n_words = (uint32_t)g.N * (uint32_t)g.L;
    if (idx >= n_words) return;
    const int I = (int)(idx / (uint32_t)g.L);
    const int J = (int)(idx - (uint32_t)I * (uint32_t)g.L);
    const uint64_t live = live_mask(I, g.L, g.N);
    if (!hot) {
        W[idx] = live;
        return;
    }
    const uint32_t row_base = (uint32_t)I * (uint32_t)g.L;
    uint64_t v = 0;
#pragma unroll
    for (int blk = 0; blk < 5; ++blk) {
        const U4 r = philox_lane_c1(0u, row_base + (uint32_t)J, 0u, (uint32_t)blk, k0, k1);
        const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = 4 * blk + j;
            v |= (uint64_t)(u[j] >> 31 ^ 1u) << (3 * (20 - p));
        }
    }
    {
        const uint32_t col = ((uint32_t)J & ~7u) | ((uint32_t)J & 1u);
        const U4 r = philox_lane_c1(0u, row_base + col, 0u, 5u, k0, k1);
        const uint32_t q = ((uint32_t)J >> 1) & 3u;
        const uint32_t u = q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w;
        v |= (uint64_t)(u >> 31 ^ 1u);
    }
    W[idx] = v & live;
}

// ---------------------------------------------------------------------------
// Half-sweep of one lattice held in global memory.  One thread per row
// segment; a segment holds WPT words of the colour being updated.
// ---------------------------------------------------------------------------
// Word accessors.  With OFF32 (lattice smaller than 4 GiB) the byte offset
// is a 32-bit value added to the wave-uniform base, which the global loads
// take directly (scalar base + 32-bit vector offset).
template <bool OFF32>
struct WordPtr {
    // global address space: word pointers read from a descriptor would
    // otherwise be generic, and generic (flat) accesses also wait on the
    // scalar-load counter
    using GlobalWord = __attribute__((address_space(1))) uint64_t;
    uint64_t* __restrict__ W;
    uint32_t L;
    __device__ __forceinline__ GlobalWord* at(int i, int j) const {
        GlobalWord* g = (GlobalWord*)W;
        if (OFF32)
            return (GlobalWord*)((__attribute__((address_space(1))) char*)g + (((uint32_t)i * L + (uint32_t)j) << 3));
        return g + ((size_t)i * L + (size_t)j);
    }
};

template <int WPT, bool MEASURE, bool OFF32>
__global__ void __launch_bounds__(kTiledMaxBlock)
    k_halfsweep_single(uint64_t* __restrict__ W, SweepArgs a, int32_t segs, int colour,
                       Partial* __restrict__ partials) {
    // word row = blockIdx.y: the row, its wrap cases, live slots and
    // counter base are wave-uniform (scalar unit); segment along x
    const int I = (int)blockIdx.y;
    const int seg = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    uint32_t anti = 0, ups = 0;
    if (seg < segs) {
        const int J0 = seg * 2 * WPT + ((I + colour) & 1);
        const WordPtr<OFF32> p{W, (uint32_t)a.L};
        auto ld = [&](int i, int j) { return *p.at(i, j); };
        auto st = [&](int i, int j, uint64_t v) { *p.at(i, j) = v; };
        update_segment<WPT, MEASURE>(ld, st, I, J0, a, anti, ups);
    }
    if (MEASURE) {
        anti = wave_sum_u32(anti);
        ups = wave_sum_u32(ups);
        const uint32_t wave = ((blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
        if (lane_id() == 0) partials[wave] = {anti, ups};
    }
}

// E = 2 A - 2 L^2 (A antiparallel bonds out of 2 L^2), M = 2 U - L^2.
__device__ __forceinline__ void energy_magnetisation(uint64_t anti, uint64_t ups, int32_t L, int64_t& E, int64_t& M) {
    const int64_t n = (int64_t)L * (int64_t)L;
    E = 2 * (int64_t)anti - 2 * n;
    M = 2 * (int64_t)ups - n;
}

// One wavefront turns a tiled lattice's wavefront partials of a measured
// sweep into its sample: series entry, moment sums, last E and M.
__device__ __forceinline__ void finalize_lattice(const LatticeDesc& d, LatticeState& st,
                                                 const Partial* __restrict__ partials) {
    // Every lane sums every 64th partial, eight loads in flight at a time: a
    // lattice has one partial per wavefront (6272 at L = 4096), and one load
    // waited for at a time made this wavefront, and with it the launch it
    // rides in, wait out ~100 memory latencies.  Indexes past the end are
    // clamped to the last partial (so every load is unconditional and in
    // bounds) and their values dropped.
    constexpr int kInFlight = 8;
    const Partial* __restrict__ part = partials + d.part_begin;
    const int n = d.part_count;
    unsigned long long anti = 0, ups = 0;
    for (int i0 = (int)lane_id(); i0 < n; i0 += 64 * kInFlight) {
        Partial v[kInFlight];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) v[k] = part[min(i0 + 64 * k, n - 1)];
#pragma unroll
        for (int k = 0; k < kInFlight; ++k) {
            const bool in = i0 + 64 * k < n;
            anti += in ? v[k].anti : 0u;
            ups += in ? v[k].ups : 0u;
        }
    }
    anti = wave_sum_u64(anti);
    ups = wave_sum_u64(ups);
    if (lane_id() == 0) {
        int64_t E, M;
        energy_magnetisation(anti, ups, d.L, E, M);
        const int64_t idx = st.series_idx;
        st.last_E = E;
        st.last_M = M;
        add_sample(st.mom, E, M);
        if (d.series_E) d.series_E[idx] = E;
        if (d.series_M) d.series_M[idx] = M;
        st.series_idx = idx + 1;
    }
}

// ---------------------------------------------------------------------------
// Half-sweep over a table of wavefronts covering many lattices.  Every
// wavefront belongs to one lattice, so the lattice's parameters (key, sweep
// index, thresholds) are wave-uniform and live in scalar registers.  With
// fin_partials set, the first wavefront of every lattice first finalizes the
// lattice's measured sweep fin_off from the partials that an earlier launch
// left (the launch boundary orders them), which saves a launch per sample.
// ---------------------------------------------------------------------------
template <int WPT, bool MEASURE, bool OFF32>
__global__ void __launch_bounds__(kTiledMaxBlock)
    k_halfsweep_multi(const LatticeDesc* __restrict__ descs, LatticeState* __restrict__ states,
                      const WaveItem* __restrict__ waves, uint32_t n_waves, int colour, uint32_t sweep_off,
                      Partial* __restrict__ partials, const Partial* __restrict__ fin_partials, uint32_t fin_off) {
    const uint32_t wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (wave >= n_waves) return;
    const WaveItem item = waves[wave];
    const LatticeDesc& d = descs[item.lattice];
    const uint64_t t = states[item.lattice].t + sweep_off;  // read before the finalize's stores: a scalar load
    if (fin_partials && wave == (uint32_t)d.part_begin && fin_off < (uint32_t)d.sweep_limit)
        finalize_lattice(d, states[item.lattice], fin_partials);
    if (sweep_off >= (uint32_t)d.sweep_limit) {  // this lattice has finished its sweeps of the chunk
        if (MEASURE && lane_id() == 0) partials[wave] = {0u, 0u};
        return;
    }
    const SweepArgs a = {d.L, d.N, d.istar, d.sh_star, (uint32_t)t, (uint32_t)(t >> 32), d.k0, d.k1, d.t4, d.t8};
    const int I = item.row;
    const int seg = item.seg0 + (int)lane_id();
    uint32_t anti = 0, ups = 0;
    if (seg < d.segs) {
        const int J0 = seg * 2 * WPT + ((I + colour) & 1);
        const WordPtr<OFF32> p{d.W, (uint32_t)a.L};
        auto ld = [&](int i, int j) { return *p.at(i, j); };
        auto st = [&](int i, int j, uint64_t v) { *p.at(i, j) = v; };
        update_segment<WPT, MEASURE>(ld, st, I, J0, a, anti, ups);
    }
    if (MEASURE) {
        anti = wave_sum_u32(anti);
        ups = wave_sum_u32(ups);
        if (lane_id() == 0) partials[wave] = {anti, ups};
    }
}

__device__ __forceinline__ void block_sum2(uint64_t& x, uint64_t& y, uint64_t* red /* 2 * 16 */) {
    x = wave_sum_u64(x);
    y = wave_sum_u64(y);
    const int wv = threadIdx.x >> 6;
    if (lane_id() == 0) {
        red[wv] = x;
        red[16 + wv] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        uint64_t sx = 0, sy = 0;
        for (int i = 0; i < nw; ++i) {
            sx += red[i];
            sy += red[16 + i];
        }
        x = sx;
        y = sy;
    }
    __syncthreads();
}

// Grid reduction of one lattice's wavefront partials: every workgroup sums a
// slice into block_sums[blockIdx.x]; the last workgroup to finish (ticket
// counter at device scope) adds the slices, turns them into E, M and resets
// the counter for the next call.
constexpr int kFinalizeBlocks = 256;

__global__ void __launch_bounds__(256) k_finalize_single(const Partial* __restrict__ partials, int64_t n_partials,
                                                         int32_t L, int64_t* series_E, int64_t* series_M,
                                                         int64_t idx, int64_t* out_EM, Moments* mom,
                                                         unsigned long long* __restrict__ block_sums,
                                                         unsigned int* __restrict__ ticket) {
    __shared__ uint64_t red[32];
    __shared__ bool last;
    uint64_t anti = 0, ups = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_partials;
         i += (int64_t)gridDim.x * blockDim.x) {
        anti += partials[i].anti;
        ups += partials[i].ups;
    }
    block_sum2(anti, ups, red);
    if (threadIdx.x == 0) {
        block_sums[2 * blockIdx.x] = anti;
        block_sums[2 * blockIdx.x + 1] = ups;
        __threadfence();
        last = atomicAdd(ticket, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    anti = 0;
    ups = 0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) {
        anti += __atomic_load_n(&block_sums[2 * i], __ATOMIC_RELAXED);
        ups += __atomic_load_n(&block_sums[2 * i + 1], __ATOMIC_RELAXED);
    }
    block_sum2(anti, ups, red);
    if (threadIdx.x == 0) {
        int64_t E, M;
        energy_magnetisation(anti, ups, L, E, M);
        if (series_E) series_E[idx] = E;
        if (series_M) series_M[idx] = M;
        if (out_EM) {
            out_EM[0] = E;
            out_EM[1] = M;
        }
        if (mom) add_sample(*mom, E, M);
        *ticket = 0u;
    }
}

// End of a chunk of sweeps, one wavefront per lattice: finalize the tiled
// lattices' measured sweep fin_off (with fin_partials set) and advance every
// lattice's sweep counter by the sweeps it ran.
__global__ void __launch_bounds__(64) k_chunk_end(const LatticeDesc* __restrict__ descs,
                                                  LatticeState* __restrict__ states,
                                                  const Partial* __restrict__ fin_partials, uint32_t fin_off,
                                                  uint32_t k) {
    const LatticeDesc& d = descs[blockIdx.x];
    LatticeState& st = states[blockIdx.x];
    if (fin_partials && !d.resident && fin_off < (uint32_t)d.sweep_limit) finalize_lattice(d, st, fin_partials);
    if (threadIdx.x == 0) st.t += min(k, (uint32_t)d.sweep_limit);
}

__global__ void k_reset_sums(LatticeState* __restrict__ states, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) states[i].mom = Moments{};
}

__global__ void k_begin_call(LatticeState* __restrict__ states, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) states[i].series_idx = 0;
}

// ---------------------------------------------------------------------------
// Resident lattices: one workgroup owns a lattice for K sweeps; colours are
// separated by workgroup barriers.  With IN_LDS the words live in LDS for
// the whole launch (read once, written once).
// ---------------------------------------------------------------------------
template <int WPT, bool IN_LDS>
__global__ void __launch_bounds__(kResidentMaxBlock)
    k_resident(const LatticeDesc* __restrict__ descs, LatticeState* __restrict__ states,
               const int32_t* __restrict__ ids, int32_t K, int32_t every) {
    extern __shared__ uint64_t lds_words[];
    __shared__ uint64_t red[32];
    const int32_t lat = ids[blockIdx.x];
    const LatticeDesc& d = descs[lat];
    LatticeState& state = states[lat];
    const int L = d.L, N = d.N;
    uint64_t* __restrict__ G = d.W;
    const uint32_t n_words = (uint32_t)N * (uint32_t)L;
    if (IN_LDS) {
        for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) lds_words[i] = G[i];
        __syncthreads();
    }
    uint64_t* __restrict__ W = IN_LDS ? lds_words : G;
    // word offsets: 32-bit inside LDS, 64-bit in global memory (N L may
    // exceed 2^31 words there)
    auto off = [&](int i, int j) {
        if constexpr (IN_LDS) return (uint32_t)i * (uint32_t)L + (uint32_t)j;
        else return (size_t)i * (size_t)L + (size_t)j;
    };
    auto ld = [&](int i, int j) { return W[off(i, j)]; };
    auto st = [&](int i, int j, uint64_t v) { W[off(i, j)] = v; };
    const int segs = (L + 2 * WPT - 1) / (2 * WPT);
    const uint32_t units = (uint32_t)N * (uint32_t)segs;
    const uint64_t t0 = state.t;
    const int32_t n_sweeps = min(K, d.sweep_limit);
    // sample accumulators stay in thread 0's registers for the whole launch
    int64_t series_idx = 0, last_E = 0, last_M = 0;
    Moments mom = {};
    int64_t* const series_E = d.series_E;
    int64_t* const series_M = d.series_M;
    if (threadIdx.x == 0) {
        series_idx = state.series_idx;
        mom = state.mom;
        last_E = state.last_E;
        last_M = state.last_M;
    }
    for (int s = 0; s < n_sweeps; ++s) {
        const uint64_t t = t0 + (uint64_t)s;
        const SweepArgs a = {L, N, d.istar, d.sh_star, (uint32_t)t, (uint32_t)(t >> 32), d.k0, d.k1, d.t4, d.t8};
        const bool meas = every > 0 && ((s + 1) % every) == 0;
        for (int colour = 0; colour < 2; ++colour) {
            uint32_t anti = 0, ups = 0;
            for (uint32_t u = threadIdx.x; u < units; u += blockDim.x) {
                const int I = (int)(u / (uint32_t)segs);
                const int seg = (int)(u - (uint32_t)I * (uint32_t)segs);
                const int J0 = seg * 2 * WPT + ((I + colour) & 1);
                if (meas && colour == 1) update_segment<WPT, true>(ld, st, I, J0, a, anti, ups);
                else update_segment<WPT, false>(ld, st, I, J0, a, anti, ups);
            }
            __syncthreads();
            if (meas && colour == 1) {
                uint64_t A = anti, U = ups;
                block_sum2(A, U, red);
                if (threadIdx.x == 0) {
                    int64_t E, M;
                    energy_magnetisation(A, U, L, E, M);
                    last_E = E;
                    last_M = M;
                    add_sample(mom, E, M);
                    if (series_E) series_E[series_idx] = E;
                    if (series_M) series_M[series_idx] = M;
                    series_idx += 1;
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        state.series_idx = series_idx;
        state.mom = mom;
        state.last_E = last_E;
        state.last_M = last_M;
    }
    if (IN_LDS) {
        for (uint32_t i = threadIdx.x; i < n_words; i += blockDim.x) G[i] = lds_words[i];
    }
}

// Observables of every lattice of a table, one workgroup per lattice:
// antiparallel right and down bonds (Section 5.3) and up spins.
__global__ void __launch_bounds__(256) k_observe_multi(const LatticeDesc* __restrict__ descs,
                                                       LatticeState* __restrict__ states,
                                                       const int32_t* __restrict__ ids, int64_t* __restrict__ out_EM) {
    __shared__ uint64_t red[32];
    const int32_t lat = ids ? ids[blockIdx.x] : (int32_t)blockIdx.x;
    const LatticeDesc& d = descs[lat];
    const int L = d.L, N = d.N;
    const uint64_t* __restrict__ W = d.W;
    auto ld = [&](int i, int j) { return W[(size_t)i * L + j]; };
    uint64_t anti = 0, ups = 0;
    const uint32_t n_words = (uint32_t)N * (uint32_t)L;
    for (uint32_t idx = threadIdx.x; idx < n_words; idx += blockDim.x) {
        const int I = (int)(idx / (uint32_t)L);
        const int J = (int)(idx - (uint32_t)I * (uint32_t)L);
        const uint64_t live = live_mask(I, L, N);
        const uint64_t w = ld(I, J);
        const uint64_t rt = ld(I, J == L - 1 ? 0 : J + 1);
        const uint64_t dn = down_word(ld, I, J, N, d.istar, d.sh_star);
        anti += __popcll((w ^ rt) & live) + __popcll((w ^ dn) & live);
        ups += __popcll(w & live);
    }
    block_sum2(anti, ups, red);
    if (threadIdx.x == 0) {
        int64_t E, M;
        energy_magnetisation(anti, ups, L, E, M);
        states[lat].last_E = E;
        states[lat].last_M = M;
        if (out_EM) {
            out_EM[2 * blockIdx.x] = E;
            out_EM[2 * blockIdx.x + 1] = M;
        }
    }
}

__global__ void __launch_bounds__(256) k_observe_single(const uint64_t* __restrict__ W, Geometry g,
                                                        Partial* __restrict__ partials) {
    const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n_words = (uint32_t)g.N * (uint32_t)g.L;
    uint32_t anti = 0, ups = 0;
    if (idx < n_words) {
        const int L = g.L;
        auto ld = [&](int i, int j) { return W[(size_t)i * L + j]; };
        const int I = (int)(idx / (uint32_t)L);
        const int J = (int)(idx - (uint32_t)I * (uint32_t)L);
        const uint64_t live = live_mask(I, L, g.N);
        const uint64_t w = ld(I, J);
        const uint64_t rt = ld(I, J == L - 1 ? 0 : J + 1);
        const uint64_t dn = down_word(ld, I, J, g.N, g.istar, g.sh_star);
        anti = __popcll((w ^ rt) & live) + __popcll((w ^ dn) & live);
        ups = __popcll(w & live);
    }
    anti = wave_sum_u32(anti);
    ups = wave_sum_u32(ups);
    if (lane_id() == 0) partials[idx >> 6] = {anti, ups};
}

__global__ void __launch_bounds__(256) k_unpack(const uint64_t* __restrict__ W, Geometry g, int32_t r0, int32_t c0,
                                                int32_t nrows, int32_t ncols, uint8_t* __restrict__ out) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)nrows * (uint64_t)ncols) return;
    const int i = (int)(idx / (uint64_t)ncols);
    const int j = (int)(idx - (uint64_t)i * (uint64_t)ncols);
    const int r = (int)(((int64_t)r0 + i) % g.L);
    const int c = (int)(((int64_t)c0 + j) % g.L);
    const int I = r % g.N, p = r / g.N;
    out[idx] = (uint8_t)((W[(size_t)I * g.L + c] >> (3 * (20 - p))) & 1ull);
}

// Write nrows lattice rows r0 .. r0 + nrows - 1 (row-major bytes, nonzero =
// up) into their words: row r is position r div N of word row r mod N.  With
// nrows <= N every word is touched by one row at most, so the bit updates of
// one launch never share a word.
__global__ void __launch_bounds__(256) k_pack_rows(const uint8_t* __restrict__ in, Geometry g, int32_t r0,
                                                   int32_t nrows, uint64_t* __restrict__ W) {
    const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (uint64_t)nrows * (uint64_t)g.L) return;
    const int i = (int)(idx / (uint64_t)g.L);
    const int c = (int)(idx - (uint64_t)i * (uint64_t)g.L);
    const int r = r0 + i;
    const int I = r % g.N, p = r / g.N;
    const uint64_t bit = 1ull << (3 * (20 - p));
    uint64_t* w = W + ((size_t)I * g.L + c);
    *w = in[idx] ? (*w | bit) : (*w & ~bit);
}

__global__ void __launch_bounds__(256) k_zero_words(uint64_t* __restrict__ p, uint64_t n) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

inline unsigned grid_for(uint64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

hipError_t launch_zero_words(uint64_t* p, uint64_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_init(uint64_t* W, const Geometry& g, uint64_t seed, int hot, hipStream_t s) {
    const uint64_t n = (uint64_t)g.N * (uint64_t)g.L;
    hipLaunchKernelGGL(k_init, dim3(grid_for(n, 256)), dim3(256), 0, s, W, g, (uint32_t)seed,
                       (uint32_t)(seed >> 32), hot);
    return hipGetLastError();
}

int64_t halfsweep_single_waves(const Geometry& g, int wpt, int block) {
    return (int64_t)grid_for((uint64_t)segments_per_row(g.L, wpt), block) * g.N * (block / 64);
}

hipError_t launch_halfsweep_single(int wpt, int block, uint64_t* W, const SweepArgs& a, int colour,
                                   Partial* partials, int64_t* n_waves, hipStream_t s) {
    const Geometry g = {a.L, a.N, a.istar, a.sh_star};
    const int32_t segs = segments_per_row(a.L, wpt);
    const dim3 grid(grid_for((uint64_t)segs, block), (unsigned)a.N), blk(block);
    if (n_waves) *n_waves = halfsweep_single_waves(g, wpt, block);
    const bool m = partials != nullptr;
    const bool off32 = (uint64_t)g.N * (uint64_t)g.L * 8u < (1ull << 32);
#define ISING_LAUNCH_HS2(WPT_, O_)                                                                                \
    if (m) hipLaunchKernelGGL((k_halfsweep_single<WPT_, true, O_>), grid, blk, 0, s, W, a, segs, colour, partials); \
    else hipLaunchKernelGGL((k_halfsweep_single<WPT_, false, O_>), grid, blk, 0, s, W, a, segs, colour, partials);
#define ISING_LAUNCH_HS(WPT_)            \
    if (off32) {                         \
        ISING_LAUNCH_HS2(WPT_, true)     \
    } else {                             \
        ISING_LAUNCH_HS2(WPT_, false)    \
    }
    switch (wpt) {
        case 1: ISING_LAUNCH_HS(1) break;
        case 2: ISING_LAUNCH_HS(2) break;
        case 4: ISING_LAUNCH_HS(4) break;
        default: return hipErrorInvalidValue;
    }
#undef ISING_LAUNCH_HS
#undef ISING_LAUNCH_HS2
    return hipGetLastError();
}

size_t finalize_scratch_bytes() { return 2 * kFinalizeBlocks * sizeof(unsigned long long) + 256; }

hipError_t launch_finalize_single(const Partial* partials, int64_t n_partials, int32_t L, int64_t* series_E,
                                  int64_t* series_M, int64_t idx, int64_t* out_EM, Moments* mom, void* scratch,
                                  hipStream_t s) {
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kFinalizeBlocks, (n_partials + 2047) / 2048));
    unsigned long long* sums = reinterpret_cast<unsigned long long*>(scratch);
    unsigned int* ticket = reinterpret_cast<unsigned int*>(reinterpret_cast<char*>(scratch) +
                                                           2 * kFinalizeBlocks * sizeof(unsigned long long));
    hipLaunchKernelGGL(k_finalize_single, dim3(blocks), dim3(256), 0, s, partials, n_partials, L, series_E, series_M,
                       idx, out_EM, mom, sums, ticket);
    return hipGetLastError();
}

int64_t observe_single_waves(const Geometry& g) { return (int64_t)grid_for((uint64_t)g.N * g.L, 256) * 4; }

hipError_t launch_observe_single(const uint64_t* W, const Geometry& g, Partial* partials, int64_t* n_waves,
                                 hipStream_t s) {
    const uint64_t n = (uint64_t)g.N * (uint64_t)g.L;
    if (n_waves) *n_waves = (int64_t)grid_for(n, 256) * 4;
    hipLaunchKernelGGL(k_observe_single, dim3(grid_for(n, 256)), dim3(256), 0, s, W, g, partials);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint64_t* W, const Geometry& g, int32_t r0, int32_t c0, int32_t nrows,
                         int32_t ncols, uint8_t* out, hipStream_t s) {
    const uint64_t n = (uint64_t)nrows * (uint64_t)ncols;
    hipLaunchKernelGGL(k_unpack, dim3(grid_for(n, 256)), dim3(256), 0, s, W, g, r0, c0, nrows, ncols, out);
    return hipGetLastError();
}

hipError_t launch_pack_rows(const uint8_t* in, const Geometry& g, int32_t r0, int32_t nrows, uint64_t* W,
                            hipStream_t s) {
    if (nrows < 1 || nrows > g.N || r0 < 0 || r0 + nrows > g.L) return hipErrorInvalidValue;
    const uint64_t n = (uint64_t)nrows * (uint64_t)g.L;
    hipLaunchKernelGGL(k_pack_rows, dim3(grid_for(n, 256)), dim3(256), 0, s, in, g, r0, nrows, W);
    return hipGetLastError();
}

hipError_t launch_halfsweep_multi(int wpt, int block, const LatticeDesc* descs, LatticeState* states,
                                  const WaveItem* waves, int64_t n_waves, int colour, uint32_t sweep_off,
                                  Partial* partials, const Partial* fin_partials, uint32_t fin_off, bool off32,
                                  hipStream_t s) {
    if (n_waves <= 0) return hipSuccess;
    const dim3 grid(grid_for((uint64_t)n_waves * 64, block)), blk(block);
    const bool m = partials != nullptr;
    const uint32_t nw = (uint32_t)n_waves;
#define ISING_LAUNCH_HM2(WPT_, O_)                                                                                  \
    if (m) hipLaunchKernelGGL((k_halfsweep_multi<WPT_, true, O_>), grid, blk, 0, s, descs, states, waves, nw,       \
                              colour, sweep_off, partials, fin_partials, fin_off);                                  \
    else hipLaunchKernelGGL((k_halfsweep_multi<WPT_, false, O_>), grid, blk, 0, s, descs, states, waves, nw,        \
                            colour, sweep_off, partials, fin_partials, fin_off);
#define ISING_LAUNCH_HM(WPT_)           \
    if (off32) {                        \
        ISING_LAUNCH_HM2(WPT_, true)    \
    } else {                            \
        ISING_LAUNCH_HM2(WPT_, false)   \
    }
    switch (wpt) {
        case 1: ISING_LAUNCH_HM(1) break;
        case 2: ISING_LAUNCH_HM(2) break;
        case 4: ISING_LAUNCH_HM(4) break;
        default: return hipErrorInvalidValue;
    }
#undef ISING_LAUNCH_HM
#undef ISING_LAUNCH_HM2
    return hipGetLastError();
}

hipError_t launch_chunk_end(const LatticeDesc* descs, LatticeState* states, int32_t n_lat,
                            const Partial* fin_partials, uint32_t fin_off, uint32_t k, hipStream_t s) {
    if (n_lat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chunk_end, dim3(n_lat), dim3(64), 0, s, descs, states, fin_partials, fin_off, k);
    return hipGetLastError();
}

hipError_t launch_reset_sums(LatticeState* states, int32_t n_lat, hipStream_t s) {
    if (n_lat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reset_sums, dim3(grid_for(n_lat, 256)), dim3(256), 0, s, states, n_lat);
    return hipGetLastError();
}

hipError_t launch_begin_call(LatticeState* states, int32_t n_lat, hipStream_t s) {
    if (n_lat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_begin_call, dim3(grid_for(n_lat, 256)), dim3(256), 0, s, states, n_lat);
    return hipGetLastError();
}

hipError_t launch_observe_multi(const LatticeDesc* descs, LatticeState* states, const int32_t* ids, int32_t n_lat,
                                int64_t* out_EM, hipStream_t s) {
    if (n_lat <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_observe_multi, dim3(n_lat), dim3(256), 0, s, descs, states, ids, out_EM);
    return hipGetLastError();
}

size_t resident_lds_limit(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return 0;
    const size_t static_bytes = 32 * sizeof(uint64_t) + 64;
    return v > (int)static_bytes ? (size_t)v - static_bytes : 0;
}

hipError_t set_resident_lds(int wpt, size_t lds_bytes) {
    const void* f = wpt == 1 ? reinterpret_cast<const void*>(&k_resident<1, true>)
                  : wpt == 2 ? reinterpret_cast<const void*>(&k_resident<2, true>)
                             : reinterpret_cast<const void*>(&k_resident<4, true>);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    int device = 0;
    if (e == hipSuccess) e = hipGetDevice(&device);
    if (e == hipSuccess) e = allow_small_lds(device);
    return e;
}

hipError_t launch_resident(int wpt, int block, const LatticeDesc* descs, LatticeState* states, const int32_t* ids,
                           int32_t n_ids, int32_t K, int32_t every, size_t lds_bytes, hipStream_t s) {
    if (n_ids <= 0 || K <= 0) return hipSuccess;
    if (block < 64 || block > kResidentMaxBlock || block % 64) return hipErrorInvalidValue;
    if (lds_bytes > 0) {
        // lattices small enough to keep the codes of two or more sweeps
        // beside them in LDS draw those ahead (k_small)
        int device = 0;
        hipError_t e = hipGetDevice(&device);
        if (e != hipSuccess) return e;
        const size_t limit = small_lds_limit(device);
        const int32_t batch = lds_bytes < limit ? (int32_t)std::min<size_t>(64, (limit - lds_bytes) / lds_bytes) : 0;
        if (batch >= 2)
            return launch_small(block, descs, states, ids, n_ids, K, every, batch, lds_bytes * (1 + batch), s);
    }
    const dim3 grid(n_ids), blk(block);
#define ISING_LAUNCH_RES(WPT_)                                                                                  \
    if (lds_bytes > 0) {                                                                                        \
        hipLaunchKernelGGL((k_resident<WPT_, true>), grid, blk, lds_bytes, s, descs, states, ids, K, every);    \
    } else {                                                                                                    \
        hipLaunchKernelGGL((k_resident<WPT_, false>), grid, blk, 0, s, descs, states, ids, K, every);           \
    }
    switch (wpt) {
        case 1: ISING_LAUNCH_RES(1) break;
        case 2: ISING_LAUNCH_RES(2) break;
        case 4: ISING_LAUNCH_RES(4) break;
        default: return hipErrorInvalidValue;
    }
#undef ISING_LAUNCH_RES
    return hipGetLastError();
}

}  // namespace ising
