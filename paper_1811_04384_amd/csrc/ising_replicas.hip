// gfx950 kernels of replica multi-spin coding: 21 independent L x L lattices
// (replicas) packed field by field into one word lattice, W[r][c] holding
// site (r, c) of replica k in field 20 - k (the coding family of Section 3
// applied across systems instead of down a column).  Replicas never
// interact; each runs the checkerboard Metropolis chain at its own
// temperature.  Neighbour words are the plain neighbours on the torus, every
// field is live, so the word update of ising_device.hpp applies with a
// threshold pair per field.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ising_device.hpp"
#include "ising_moments.hpp"
#include "ising_replicas.hpp"

namespace ising {

namespace {

constexpr uint32_t kStreamSweep = 6;  // Philox counter word 3 = g + 8 stream
constexpr uint32_t kStreamInit = 7;

// Draw of replica k at site (r, c): block g = k div 4 (k < 20) keyed by the
// site, output k mod 4; replica 20 shares block 5 among the four same-colour
// sites 8 (c div 8) + (c mod 2) + 2m of the row, output (c div 2) mod 4.
__device__ __forceinline__ uint32_t replica_draw(uint32_t t_lo, uint32_t t_hi, uint32_t stream, int L, int k, int r,
                                                 int c, uint32_t k0, uint32_t k1) {
    const uint32_t col = k < 20 ? (uint32_t)c : (((uint32_t)c & ~7u) | ((uint32_t)c & 1u));
    const uint32_t g = k < 20 ? (uint32_t)(k >> 2) : 5u;
    const U4 o = philox_lane_c1(t_lo, (uint32_t)r * (uint32_t)L + col, t_hi, g + 8u * stream, k0, k1);
    const uint32_t q = k < 20 ? (uint32_t)(k & 3) : (((uint32_t)c >> 1) & 3u);
    return q == 0 ? o.x : q == 1 ? o.y : q == 2 ? o.z : o.w;
}

__global__ void __launch_bounds__(256) k_replica_init(uint64_t* __restrict__ W, int L, uint32_t k0, uint32_t k1,
                                                     int hot) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)L * (uint64_t)L) return;
    const int r = (int)(i / (uint64_t)L), c = (int)(i - (uint64_t)r * (uint64_t)L);
    uint64_t w = 0;
    for (int k = 0; k < kReplicas; ++k) {
        const bool up = !hot || replica_draw(0u, 0u, kStreamInit, L, k, r, c, k0, k1) < 0x80000000u;
        w |= (uint64_t)up << (3 * (20 - k));
    }
    W[i] = w;
}

// One colour of every replica: one thread per row segment of 2 WPT columns
// (WPT same-colour words), as in the column-coded half-sweep.  The
// position-20 block of the segment's words is drawn once.
template <int WPT>
__global__ void __launch_bounds__(256) k_replica_halfsweep(uint64_t* __restrict__ W, ReplicaArgs a, int colour) {
    const int L = a.L;
    const int segs = (L / 2 + WPT - 1) / WPT;
    const uint64_t unit = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (unit >= (uint64_t)L * (uint64_t)segs) return;
    const int r = (int)(unit / (uint64_t)segs);
    const int seg = (int)(unit - (uint64_t)r * (uint64_t)segs);
    const int J0 = seg * 2 * WPT + ((r + colour) & 1);
    const int ru = r == 0 ? L - 1 : r - 1, rd = r == L - 1 ? 0 : r + 1;
    const uint32_t row_base = (uint32_t)r * (uint32_t)L;
    const uint32_t c3 = 8u * kStreamSweep;
    uint64_t* __restrict__ row = W + (size_t)r * (size_t)L;
    const uint64_t* __restrict__ row_up = W + (size_t)ru * (size_t)L;
    const uint64_t* __restrict__ row_dn = W + (size_t)rd * (size_t)L;

    const RoundKeys rk = round_keys(a.k0, a.k1);
    uint32_t u20[4] = {0u, 0u, 0u, 0u};
    {
        const uint32_t col = ((uint32_t)J0 & ~7u) | ((uint32_t)J0 & 1u);
        const U4 o = philox_lane_c1(a.t_lo, row_base + col, a.t_hi, 5u + c3, a.k0, a.k1, rk);
        const uint32_t q0 = ((uint32_t)J0 >> 1) & 3u;
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const uint32_t q = (q0 + (uint32_t)k) & 3u;
            u20[k] = q == 0 ? o.x : q == 1 ? o.y : q == 2 ? o.z : o.w;
        }
    }
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        const int J = J0 + 2 * k;
        if (J >= L) break;
        const uint64_t w = row[J];
        const uint64_t lf = row[J == 0 ? L - 1 : J - 1];
        const uint64_t rt = row[J == L - 1 ? 0 : J + 1];
        const uint64_t up = row_up[J];
        const uint64_t dn = row_dn[J];
        Codes codes = {0u, 0u, 0u};
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            const U4 o = philox_lane_c1(a.t_lo, row_base + (uint32_t)J, a.t_hi, (uint32_t)g + c3, a.k0, a.k1, rk);
            append_draw(codes, 4 * g + 0, o.x, a.t4[4 * g + 0], a.t8[4 * g + 0]);
            append_draw(codes, 4 * g + 1, o.y, a.t4[4 * g + 1], a.t8[4 * g + 1]);
            append_draw(codes, 4 * g + 2, o.z, a.t4[4 * g + 2], a.t8[4 * g + 2]);
            append_draw(codes, 4 * g + 3, o.w, a.t4[4 * g + 3], a.t8[4 * g + 3]);
        }
        append_draw(codes, 20, u20[k], a.t4[20], a.t8[20]);
        row[J] = w ^ flip_mask(w, up, dn, lf, rt, assemble_codes(codes), kSpinBits);
    }
}

// Per-replica antiparallel right+down bonds and up spins of all words.
// Each thread adds fields 0..19 in 6-bit lanes (even fields from bit 0, odd
// fields shifted down by 3), at most 2 per word, flushing to per-replica
// counters every 31 words; field 20 (bit 60, whose lane would have only 4
// bits) is counted directly.  The workgroup then sums the counters in LDS
// and adds them to totals[0..20] (bonds) and totals[21..41] (up spins).
constexpr uint64_t kLaneFields = 0x0041041041041041ull;  // bits 0, 6, ..., 54

__device__ __forceinline__ void flush_lanes(uint64_t& even, uint64_t& odd, uint32_t* cnt) {
#pragma unroll
    for (int f = 0; f < 20; ++f) {
        const uint64_t v = (f & 1) ? (odd >> (6 * (f >> 1))) : (even >> (6 * (f >> 1)));
        cnt[20 - f] += (uint32_t)(v & 63u);  // field f holds replica 20 - f
    }
    even = 0;
    odd = 0;
}

__global__ void __launch_bounds__(256) k_replica_observe(const uint64_t* __restrict__ W, int L,
                                                        unsigned long long* __restrict__ totals) {
    __shared__ uint32_t sums[2 * kReplicas];
    for (int i = threadIdx.x; i < 2 * kReplicas; i += blockDim.x) sums[i] = 0;
    __syncthreads();
    uint32_t anti[kReplicas], ups[kReplicas];
#pragma unroll
    for (int k = 0; k < kReplicas; ++k) anti[k] = ups[k] = 0;
    uint64_t ae = 0, ao = 0, ue = 0, uo = 0;
    int pending = 0;
    const uint64_t n = (uint64_t)L * (uint64_t)L;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        const int r = (int)(i / (uint64_t)L), c = (int)(i - (uint64_t)r * (uint64_t)L);
        const uint64_t w = W[i];
        const uint64_t xr = w ^ W[(size_t)r * L + (c == L - 1 ? 0 : c + 1)];
        const uint64_t xd = w ^ W[(size_t)(r == L - 1 ? 0 : r + 1) * L + c];
        ae += (xr & kLaneFields) + (xd & kLaneFields);
        ao += ((xr >> 3) & kLaneFields) + ((xd >> 3) & kLaneFields);
        ue += w & kLaneFields;
        uo += (w >> 3) & kLaneFields;
        anti[0] += (uint32_t)(xr >> 60) + (uint32_t)(xd >> 60);  // field 20 = replica 0
        ups[0] += (uint32_t)(w >> 60);
        if (++pending == 31) {
            flush_lanes(ae, ao, anti);
            flush_lanes(ue, uo, ups);
            pending = 0;
        }
    }
    flush_lanes(ae, ao, anti);
    flush_lanes(ue, uo, ups);
#pragma unroll
    for (int k = 0; k < kReplicas; ++k) {
        const uint32_t a = wave_sum_u32(anti[k]), u = wave_sum_u32(ups[k]);
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&sums[k], a);
            atomicAdd(&sums[kReplicas + k], u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 2 * kReplicas; i += blockDim.x) atomicAdd(&totals[i], (unsigned long long)sums[i]);
}

// totals -> E_k = 2 A_k - 2 L^2, M_k = 2 U_k - L^2; series slot `idx`
// (21 entries), moments, out_EM; totals cleared for the next observation.
__global__ void k_replica_finalize(unsigned long long* __restrict__ totals, int L, int64_t* series_E,
                                   int64_t* series_M, int64_t idx, Moments* mom, int64_t* out_EM) {
    const int k = threadIdx.x;
    if (k >= kReplicas) return;
    const int64_t n = (int64_t)L * (int64_t)L;
    const int64_t E = 2 * (int64_t)totals[k] - 2 * n;
    const int64_t M = 2 * (int64_t)totals[kReplicas + k] - n;
    if (series_E) series_E[idx * kReplicas + k] = E;
    if (series_M) series_M[idx * kReplicas + k] = M;
    if (mom) add_sample(mom[k], E, M);
    if (out_EM) {
        out_EM[k] = E;
        out_EM[kReplicas + k] = M;
    }
    totals[k] = 0;
    totals[kReplicas + k] = 0;
}

// Spins of replica k in rows r0 .. r0 + nrows - 1, row major.
__global__ void __launch_bounds__(256) k_replica_unpack(const uint64_t* __restrict__ W, int L, int k, int r0,
                                                       int nrows, uint8_t* __restrict__ out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)nrows * (uint64_t)L) return;
    out[i] = (uint8_t)((W[(uint64_t)r0 * (uint64_t)L + i] >> (3 * (20 - k))) & 1u);
}

inline unsigned rgrid(uint64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_replica_init(uint64_t* W, int L, uint64_t seed, int hot, hipStream_t s) {
    hipLaunchKernelGGL(k_replica_init, dim3(rgrid((uint64_t)L * L, 256)), dim3(256), 0, s, W, L, (uint32_t)seed,
                       (uint32_t)(seed >> 32), hot);
    return hipGetLastError();
}

hipError_t launch_replica_halfsweep(int wpt, uint64_t* W, const ReplicaArgs& a, int colour, hipStream_t s) {
    const uint64_t units = (uint64_t)a.L * (uint64_t)((a.L / 2 + wpt - 1) / wpt);
    const dim3 grid(rgrid(units, 256)), blk(256);
    switch (wpt) {
        case 1: hipLaunchKernelGGL(k_replica_halfsweep<1>, grid, blk, 0, s, W, a, colour); break;
        case 2: hipLaunchKernelGGL(k_replica_halfsweep<2>, grid, blk, 0, s, W, a, colour); break;
        case 4: hipLaunchKernelGGL(k_replica_halfsweep<4>, grid, blk, 0, s, W, a, colour); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_replica_observe(const uint64_t* W, int L, unsigned long long* totals, int64_t* series_E,
                                  int64_t* series_M, int64_t idx, Moments* mom, int64_t* out_EM, hipStream_t s) {
    const uint64_t n = (uint64_t)L * (uint64_t)L;
    const unsigned blocks = std::max(1u, std::min(rgrid(n, 256 * 32), 2048u));
    hipLaunchKernelGGL(k_replica_observe, dim3(blocks), dim3(256), 0, s, W, L, totals);
    hipLaunchKernelGGL(k_replica_finalize, dim3(1), dim3(64), 0, s, totals, L, series_E, series_M, idx, mom, out_EM);
    return hipGetLastError();
}

hipError_t launch_replica_unpack(const uint64_t* W, int L, int k, int r0, int nrows, uint8_t* out, hipStream_t s) {
    if (r0 < 0 || nrows < 1 || r0 + nrows > L) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_replica_unpack, dim3(rgrid((uint64_t)nrows * L, 256)), dim3(256), 0, s, W, L, k, r0, nrows,
                       out);
    return hipGetLastError();
}

}  // namespace ising
