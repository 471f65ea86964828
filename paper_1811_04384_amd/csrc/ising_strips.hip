// gfx950 kernels of the paper's own dynamics: random word picks inside
// vertical strips of the word lattice, left half then right half of every
// strip per iteration (Sections 4 and 5.2, Table 2), and their launchers.
// The per-word update (neighbour words, acceptance codes, flip mask) is the
// one of ising_device.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ising_device.hpp"
#include "ising_launch.hpp"

namespace ising {

namespace {

// ---------------------------------------------------------------------------
// Strip dynamics (random word picks, two phases per iteration): one thread
// per strip applies that strip's picks of one phase in order.  Strips never
// touch each other's words inside a phase, so threads need no
// synchronisation; a thread sees its own earlier stores.  Pick k draws its
// word from Philox counter (t lo, strip, k div 2, 8 (2 + phase) + 256 t hi)
// -- outputs (x, y) for even k, (z, w) for odd k; row floor(x N / 2^32),
// column off + floor(y width / 2^32) -- and its 21 uniforms from counters
// (t lo, strip, k, g + 8 (4 + phase) + 256 t hi), g = 0..5.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(64) k_strip_phase(uint64_t* __restrict__ W, StripArgs a) {
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= a.strips) return;
    const int L = a.L, N = a.N;
    auto ld = [&](int i, int j) { return W[(size_t)i * (size_t)L + (size_t)j]; };
    const uint32_t c3_pick = 8u * (2u + a.phase) + (a.t_hi << 8);
    const uint32_t c3_word = 8u * (4u + a.phase) + (a.t_hi << 8);
    const int col0 = p * a.S + a.off;
    const RoundKeys rk = round_keys(a.k0, a.k1);
    U4 pick = {0u, 0u, 0u, 0u};
    for (uint32_t k = 0; k < a.picks; ++k) {
        if ((k & 1u) == 0u) pick = philox_lane_c1(a.t_lo, (uint32_t)p, k >> 1, c3_pick, a.k0, a.k1);
        const uint32_t x = (k & 1u) ? pick.z : pick.x;
        const uint32_t y = (k & 1u) ? pick.w : pick.y;
        const int I = (int)(((uint64_t)x * (uint64_t)(uint32_t)N) >> 32);
        const int J = col0 + (int)(((uint64_t)y * (uint64_t)(uint32_t)a.width) >> 32);
        const uint64_t w = ld(I, J);
        const uint64_t lf = ld(I, J == 0 ? L - 1 : J - 1);
        const uint64_t rt = ld(I, J == L - 1 ? 0 : J + 1);
        const uint64_t up = up_word(ld, I, J, N, a.istar, a.sh_star);
        const uint64_t dn = down_word(ld, I, J, N, a.istar, a.sh_star);
        // every position draws (dead slots are masked by `live`), so lanes
        // with different rows run the same instructions
        Codes codes = {0u, 0u, 0u};
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            const U4 r = philox_lane_c1(a.t_lo, (uint32_t)p, k, (uint32_t)g + c3_word, a.k0, a.k1, rk);
            append_draw(codes, 4 * g + 0, r.x, a.t4, a.t8);
            append_draw(codes, 4 * g + 1, r.y, a.t4, a.t8);
            append_draw(codes, 4 * g + 2, r.z, a.t4, a.t8);
            append_draw(codes, 4 * g + 3, r.w, a.t4, a.t8);
        }
        const U4 r5 = philox_lane_c1(a.t_lo, (uint32_t)p, k, 5u + c3_word, a.k0, a.k1, rk);
        append_draw(codes, 20, r5.x, a.t4, a.t8);
        const uint64_t f = flip_mask(w, up, dn, lf, rt, assemble_codes(codes), live_mask(I, L, N));
        W[(size_t)I * (size_t)L + (size_t)J] = w ^ f;
    }
}

// The same phase in two steps.  The draws do not depend on the state, so a
// parallel kernel computes, for picks [k0, k0 + n_k) of every strip, the
// word (packed as I << 17 | column within the phase) and the 21 acceptance
// codes; then one lane per strip applies them in order with the strip's
// phase columns and its two frozen neighbour columns held in LDS.
constexpr int kStripColBits = 17;

__global__ void __launch_bounds__(256) k_strip_draws(StripArgs a, uint32_t k0, uint32_t n_k,
                                                    uint32_t* __restrict__ pos, uint64_t* __restrict__ codes_out) {
    const uint64_t total = (uint64_t)n_k * (uint64_t)a.strips;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const uint32_t kk = (uint32_t)(i / (uint64_t)a.strips);
    const uint32_t p = (uint32_t)(i - (uint64_t)kk * (uint64_t)a.strips);
    const uint32_t k = k0 + kk;
    const uint32_t c3_pick = 8u * (2u + a.phase) + (a.t_hi << 8);
    const uint32_t c3_word = 8u * (4u + a.phase) + (a.t_hi << 8);
    const U4 pick = philox_lane_c1(a.t_lo, p, k >> 1, c3_pick, a.k0, a.k1);
    const uint32_t x = (k & 1u) ? pick.z : pick.x;
    const uint32_t y = (k & 1u) ? pick.w : pick.y;
    const uint32_t I = (uint32_t)(((uint64_t)x * (uint64_t)(uint32_t)a.N) >> 32);
    const uint32_t jl = (uint32_t)(((uint64_t)y * (uint64_t)(uint32_t)a.width) >> 32);
    const RoundKeys rk = round_keys(a.k0, a.k1);
    Codes codes = {0u, 0u, 0u};
#pragma unroll
    for (int g = 0; g < 5; ++g) {
        const U4 r = philox_lane_c1(a.t_lo, p, k, (uint32_t)g + c3_word, a.k0, a.k1, rk);
        append_draw(codes, 4 * g + 0, r.x, a.t4, a.t8);
        append_draw(codes, 4 * g + 1, r.y, a.t4, a.t8);
        append_draw(codes, 4 * g + 2, r.z, a.t4, a.t8);
        append_draw(codes, 4 * g + 3, r.w, a.t4, a.t8);
    }
    const U4 r5 = philox_lane_c1(a.t_lo, p, k, 5u + c3_word, a.k0, a.k1, rk);
    append_draw(codes, 20, r5.x, a.t4, a.t8);
    pos[i] = (I << kStripColBits) | jl;
    codes_out[i] = assemble_codes(codes);
}

// One lane per strip; lanes >= chains of a workgroup idle.  LDS column cc of
// a chain: 0 = the frozen column left of the phase columns, 1..width = the
// phase columns, width + 1 = the frozen column right of them; N words each.
// After the chains' columns the LDS holds the live-slot mask of every word
// row.
__global__ void __launch_bounds__(64) k_strip_apply(uint64_t* __restrict__ W, StripArgs a, int chains,
                                                    uint32_t n_k, const uint32_t* __restrict__ pos,
                                                    const uint64_t* __restrict__ codes) {
    extern __shared__ uint64_t strip_lds[];
    const int lane = (int)threadIdx.x;
    const int p0 = (int)blockIdx.x * chains;
    const int n_chains = min(chains, a.strips - p0);
    const int L = a.L, N = a.N, width = a.width, cols = width + 2;
    // cooperative fill: entry e = (row I, chain q, LDS column cc) with
    // (q, cc) fastest, so neighbouring threads read neighbouring columns
    const int per_row = n_chains * cols;
    const int n_fill = per_row * N;
    auto fill_col = [&](int e, int& q, int& cc, int& I) {
        I = e / per_row;
        const int rem = e - I * per_row;
        q = rem / cols;
        cc = rem - q * cols;
    };
    for (int e0 = lane; e0 < n_fill; e0 += 64 * 8) {
        uint64_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 64 * u;
            if (e < n_fill) {
                int q, cc, I;
                fill_col(e, q, cc, I);
                const int J = ((p0 + q) * a.S + a.off + cc - 1 + L) % L;
                v[u] = W[(size_t)I * (size_t)L + (size_t)J];
            }
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + 64 * u;
            if (e < n_fill) {
                int q, cc, I;
                fill_col(e, q, cc, I);
                strip_lds[((size_t)q * cols + cc) * N + I] = v[u];
            }
        }
    }
    uint64_t* __restrict__ live_row = strip_lds + (size_t)chains * (size_t)cols * (size_t)N;
    for (int I = lane; I < N; I += 64) live_row[I] = live_mask(I, L, N);
    __syncthreads();
    if (lane < n_chains) {
        const int p = p0 + lane;
        uint64_t* __restrict__ my = strip_lds + (size_t)lane * (size_t)cols * (size_t)N;
        const size_t stride = (size_t)a.strips;
        auto apply = [&](uint32_t pk, uint64_t cd) {
            const int I = (int)(pk >> kStripColBits);
            const int cc = (int)(pk & ((1u << kStripColBits) - 1u)) + 1;
            uint64_t* __restrict__ col = my + cc * N;
            auto ld = [&](int i, int) { return col[i]; };
            const uint64_t w = col[I];
            const uint64_t lf = col[I - N];
            const uint64_t rt = col[I + N];
            const uint64_t up = up_word(ld, I, 0, N, a.istar, a.sh_star);
            const uint64_t dn = down_word(ld, I, 0, N, a.istar, a.sh_star);
            col[I] = w ^ flip_mask(w, up, dn, lf, rt, cd, live_row[I]);
        };
        // the pick data of the next four picks is in flight while one is applied
        auto at = [&](uint32_t kk) { return (size_t)min(kk, n_k - 1) * stride + (size_t)p; };
        uint32_t q0 = pos[at(0)], q1 = pos[at(1)], q2 = pos[at(2)], q3 = pos[at(3)];
        uint64_t d0 = codes[at(0)], d1 = codes[at(1)], d2 = codes[at(2)], d3 = codes[at(3)];
        uint32_t kk = 0;
        for (; kk + 4 <= n_k; kk += 4) {
            uint32_t q;
            uint64_t e;
            q = pos[at(kk + 4)], e = codes[at(kk + 4)], apply(q0, d0), q0 = q, d0 = e;
            q = pos[at(kk + 5)], e = codes[at(kk + 5)], apply(q1, d1), q1 = q, d1 = e;
            q = pos[at(kk + 6)], e = codes[at(kk + 6)], apply(q2, d2), q2 = q, d2 = e;
            q = pos[at(kk + 7)], e = codes[at(kk + 7)], apply(q3, d3), q3 = q, d3 = e;
        }
        if (kk < n_k) apply(q0, d0);
        if (kk + 1 < n_k) apply(q1, d1);
        if (kk + 2 < n_k) apply(q2, d2);
    }
    __syncthreads();
    // cooperative write-back of the phase columns (LDS columns 1..width)
    const int per_row_w = n_chains * width;
    const int n_back = per_row_w * N;
    for (int e = lane; e < n_back; e += 64) {
        const int I = e / per_row_w;
        const int rem = e - I * per_row_w;
        const int q = rem / width;
        const int cc = rem - q * width + 1;
        const int J = (p0 + q) * a.S + a.off + cc - 1;
        W[(size_t)I * (size_t)L + (size_t)J] = strip_lds[((size_t)q * cols + cc) * N + I];
    }
}

inline unsigned strip_grid(uint64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

hipError_t launch_strip_phase(uint64_t* W, const StripArgs& a, hipStream_t s) {
    if (a.strips <= 0 || a.picks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_strip_phase, dim3(strip_grid((uint64_t)a.strips, 64)), dim3(64), 0, s, W, a);
    return hipGetLastError();
}

size_t strip_chain_lds_bytes(const StripArgs& a) { return (size_t)(a.width + 2) * (size_t)a.N * sizeof(uint64_t); }

hipError_t launch_strip_draws(const StripArgs& a, uint32_t k0, uint32_t n_k, uint32_t* pos, uint64_t* codes,
                              hipStream_t s) {
    const uint64_t total = (uint64_t)n_k * (uint64_t)a.strips;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_strip_draws, dim3(strip_grid(total, 256)), dim3(256), 0, s, a, k0, n_k, pos, codes);
    return hipGetLastError();
}

hipError_t launch_strip_apply(uint64_t* W, const StripArgs& a, uint32_t n_k, const uint32_t* pos,
                              const uint64_t* codes, hipStream_t s) {
    if (a.strips <= 0 || n_k == 0) return hipSuccess;
    const size_t per_chain = strip_chain_lds_bytes(a);
    const size_t live_bytes = (size_t)a.N * sizeof(uint64_t);
    if (per_chain + live_bytes > kStripLdsBytes) return hipErrorInvalidValue;
    const int chains = (int)std::min<size_t>(64, (kStripLdsBytes - live_bytes) / per_chain);
    hipLaunchKernelGGL(k_strip_apply, dim3(strip_grid((uint64_t)a.strips, chains)), dim3(64),
                       chains * per_chain + live_bytes, s, W, a, chains, n_k, pos, codes);
    return hipGetLastError();
}

}  // namespace ising
