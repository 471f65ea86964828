// Small lattices whose acceptance codes are drawn by the whole chip and
// applied by one small workgroup per lattice.
//
// The acceptance codes of a site (Table 1's classes with the Metropolis rule
// of Section 2 applied to its uniform) do not depend on the spins, only on
// (seed, sweep, site) and the temperature.  A handful of small lattices (a
// temperature scan of a few L = 64 lattices, the paper's N = 4 lattice)
// leaves all but a few compute units idle when each lattice's workgroup
// draws its own codes; here a draw pass spreads the codes of many sweeps of
// every such lattice over the whole chip into a global buffer, and an apply
// pass then runs the sweeps: one workgroup of one to four wavefronts per
// lattice, the lattice in LDS, each thread's codes loaded into registers
// several sweeps ahead of their use.  What is left per half-sweep is one
// word update per thread and word -- a chain of a few hundred cycles -- and
// a workgroup barrier; with one wavefront not even that, as a wavefront's
// LDS operations complete in issue order, so one half-sweep's stores are
// seen by the next half-sweep's loads.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ising_device.hpp"
#include "ising_launch.hpp"
#include "ising_lds_word.hpp"
#include "ising_moments.hpp"

namespace ising {

namespace {

constexpr int kDrawBlock = 256;
constexpr int kApplyMaxBlock = 256;

// Order a lone wavefront's LDS stores of one half-sweep before the loads of
// the next (the hardware completes them in issue order; this keeps the
// compiler from moving them).
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace

// Draw pass: item f of lattice entry e (blockIdx.x div blocks_per_lat) is
// sweep j = f div n_draw of the pass (absolute sweep t = state.t +
// sweep_off + j) and (colour c, word row I, 8-column group); it writes the
// codes of the group's four words of that colour, drawn exactly as every
// other path draws them (Philox blocks 0..4 of counter (t, I L + J), the
// position-20 block 5 shared by the group).  Codes of sweep j, colour c are
// stored by word slot f = I (L/2) + h for column J = 2h + ((I + c) & 1), so
// the four words of an item are adjacent.  Sweeps past the lattice's sweep
// limit are not drawn.
__global__ void __launch_bounds__(kDrawBlock) k_draw_codes(const LatticeDesc* __restrict__ descs,
                                                           const LatticeState* __restrict__ states,
                                                           const DrawLat* __restrict__ lats, uint64_t* __restrict__ codes,
                                                           int32_t blocks_per_lat, int32_t sweep_off, int32_t S) {
    const int e = (int)(blockIdx.x / (unsigned)blocks_per_lat);
    const DrawLat dl = lats[e];
    const int f = (int)(blockIdx.x - (unsigned)e * (unsigned)blocks_per_lat) * kDrawBlock + (int)threadIdx.x;
    if (f >= S * dl.n_draw) return;
    const LatticeDesc& d = descs[dl.lat];
    const int L = d.L, N = d.N, istar = d.istar;
    const int j = f / dl.n_draw, r = f - j * dl.n_draw;
    if (sweep_off + j >= d.sweep_limit) return;
    const int groups = (L + 7) >> 3;
    const int c = r >= N * groups ? 1 : 0;
    const int rr = r - c * N * groups;
    const int I = rr / groups, grp = rr - I * groups;
    const int n_live = (L - 1) / N + (I <= istar ? 1 : 0);
    const uint64_t t = states[dl.lat].t + (uint64_t)(sweep_off + j);
    const uint32_t t_lo = (uint32_t)t, t_hi = (uint32_t)(t >> 32);
    const RoundKeys rk = round_keys(d.k0, d.k1);
    const int par = (I + c) & 1;
    const int half = L >> 1;
    uint4 u5 = make_uint4(0u, 0u, 0u, 0u);
    if (n_live == 21) {
        const U4 r5 = philox_lane_c1(t_lo, (uint32_t)I * (uint32_t)L + (uint32_t)(8 * grp + par), t_hi, 5u | (1u << 3),
                                     d.k0, d.k1, rk);
        u5 = make_uint4(r5.x, r5.y, r5.z, r5.w);
    }
    uint64_t* __restrict__ out = codes + dl.base + (size_t)j * (size_t)(N * L) + (size_t)(c * N * half + I * half + 4 * grp);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int J = 8 * grp + par + 2 * m;
        if (J >= L) break;
        Codes cd = {0u, 0u, 0u};
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            if (4 * g < n_live) {
                const U4 q = philox_lane_c1(t_lo, (uint32_t)I * (uint32_t)L + (uint32_t)J, t_hi, (uint32_t)g | (1u << 3),
                                            d.k0, d.k1, rk);
                append_draw(cd, 4 * g + 0, q.x, d.t4, d.t8);
                append_draw(cd, 4 * g + 1, q.y, d.t4, d.t8);
                append_draw(cd, 4 * g + 2, q.z, d.t4, d.t8);
                append_draw(cd, 4 * g + 3, q.w, d.t4, d.t8);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) append_code(cd, 4 * g + k, 0u);
            }
        }
        append_draw(cd, 20, pick4(u5, (uint32_t)m), d.t4, d.t8);  // a dead slot when n_live < 21
        out[m] = assemble_codes(cd);
    }
}

namespace {

// Issue the loads of sweep j's codes of this thread's words (slots past the
// last word load the last word's code, which is not used), without branches
// so that the compiler can count them and wait only for the oldest.
template <int WMAX>
__device__ __forceinline__ void load_codes(uint64_t (&cr)[2][WMAX], const uint64_t* __restrict__ cg, size_t NL,
                                           int words, int tid, int stride, int j) {
    const uint64_t* __restrict__ p = cg + (size_t)j * NL;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int k = 0; k < WMAX; ++k) cr[c][k] = __builtin_nontemporal_load(p + c * words + min(tid + stride * k, words - 1));
}

}  // namespace

// Apply pass: one workgroup of A = blockDim.x / 64 wavefronts (ONE_WAVE: A
// = 1) per lattice entry, S sweeps of the pass (local sweep index s =
// sweep_off + j of the chunk; a sample after it when (s + 1) % every == 0,
// every > 0).  LDS: the lattice [N][L], then one (antiparallel bonds, up
// spins) pair per sample of the pass.  Thread tid holds the word slots
// tid + 64 A k (k < WMAX) of each colour, and the codes of its words are
// loaded from the global buffer straight into registers, P sweeps ahead of
// their use.  In a half-sweep no word read is written (all neighbours, the
// wrap words and the patch word have the other colour), so every thread
// loads all of its neighbourhoods first and then flips and stores;
// half-sweeps are separated by a workgroup barrier, or, with one wavefront,
// by the in-order completion of its LDS operations.  A sampled sweep only
// adds its wavefront sums to its pair; after the sweeps the first wavefront
// turns the pairs into E, M, the series and the moment sums.
template <int WMAX, int P, bool ONE_WAVE>
__global__ void __launch_bounds__(kApplyMaxBlock) k_wave_apply(const LatticeDesc* __restrict__ descs,
                                                               LatticeState* __restrict__ states,
                                                               const DrawLat* __restrict__ lats,
                                                               const uint64_t* __restrict__ codes, int32_t sweep_off,
                                                               int32_t S, int32_t every) {
    extern __shared__ uint64_t lds[];
    const DrawLat dl = lats[blockIdx.x];
    const LatticeDesc& d = descs[dl.lat];
    LatticeState& state = states[dl.lat];
    const int n = min(S, d.sweep_limit - sweep_off);
    if (n <= 0) return;  // uniform over the workgroup
    const int L = d.L, N = d.N, istar = d.istar, sh_star = d.sh_star;
    const int NL = N * L;
    const int pstar = (L - 1) / N;
    const int half = L >> 1;
    const int words = N * half;  // words of one colour
    const int tid = threadIdx.x, B = blockDim.x;
    uint64_t* __restrict__ T = lds;
    uint32_t* __restrict__ stage = reinterpret_cast<uint32_t*>(lds + NL);  // [samples][2]
    const int n_samples = every > 0 ? (sweep_off + n) / every - sweep_off / every : 0;
    const uint64_t* __restrict__ cg = codes + dl.base;
    uint64_t* __restrict__ G = d.W;
    for (int i = tid; i < NL; i += B) T[i] = G[i];
    for (int i = tid; i < 2 * n_samples; i += B) stage[i] = 0u;
    int Iw[WMAX], Hw[WMAX];
    uint64_t live[WMAX];
#pragma unroll
    for (int k = 0; k < WMAX; ++k) {
        const int f = min(tid + B * k, words - 1);
        Iw[k] = f / half;
        Hw[k] = f - Iw[k] * half;
        const int n_live = pstar + (Iw[k] <= istar ? 1 : 0);
        live[k] = kSpinBits & (~0ull << (3 * (21 - n_live)));
    }
    uint64_t ring[P][2][WMAX];
#pragma unroll
    for (int r = 0; r < P; ++r) load_codes<WMAX>(ring[r], cg, (size_t)NL, words, tid, B, min(r, n - 1));
    __syncthreads();
    // sweeps left before the next sample, and the index of that sample
    int until = every > 0 ? every - 1 - sweep_off % every : 0x7FFFFFFF;
    int ks = 0;
    // the next sweep, with its codes cc
    auto sweep = [&](const uint64_t (&cc)[2][WMAX]) {
        const bool meas = until == 0;
        until = meas ? every - 1 : until - 1;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            Nbhd nb[WMAX];
#pragma unroll
            for (int k = 0; k < WMAX; ++k) {
                if (tid + B * k < words) {
                    const int I = Iw[k], J = 2 * Hw[k] + ((I + c) & 1);
                    nb[k] = lds_nbhd(T, L, N, istar, I, J, J == 0 ? L - 1 : J - 1, J == L - 1 ? 0 : J + 1);
                }
            }
            uint32_t anti = 0, ups = 0;
#pragma unroll
            for (int k = 0; k < WMAX; ++k) {
                if (tid + B * k < words) {
                    const int I = Iw[k], J = 2 * Hw[k] + ((I + c) & 1);
                    const uint64_t up = up_of(nb[k], I, sh_star);
                    const uint64_t dn = down_of(nb[k], I, N, istar, sh_star);
                    const uint64_t nw = nb[k].w ^ flip_mask(nb[k].w, up, dn, nb[k].lf, nb[k].rt, cc[c][k], live[k]);
                    T[I * L + J] = nw;
                    if (c == 1 && meas) measure_word(nw, up, dn, nb[k].lf, nb[k].rt, live[k], anti, ups);
                }
            }
            if (c == 1 && meas) {
                // one wavefront sum of both counts: a wavefront's words (at
                // most 256) have fewer than 2^16 antiparallel bonds (84 per
                // word) and up spins (42 per word, with the left neighbour's)
                const uint32_t both = wave_sum_u32((anti << 16) | ups);
                if ((tid & 63) == 0) {
                    if (ONE_WAVE) {
                        stage[2 * ks] = both >> 16;
                        stage[2 * ks + 1] = both & 0xFFFFu;
                    } else {
                        atomicAdd(&stage[2 * ks], both >> 16);
                        atomicAdd(&stage[2 * ks + 1], both & 0xFFFFu);
                    }
                }
                ks += 1;
            }
            if (ONE_WAVE)
                wave_lds_order();
            else
                __syncthreads();
        }
    };
    // whole groups of P sweeps: slot r's codes are used, then reloaded with
    // those P sweeps later
    int j0 = 0;
    for (; j0 + P <= n; j0 += P) {
#pragma unroll
        for (int r = 0; r < P; ++r) {
            sweep(ring[r]);
            load_codes<WMAX>(ring[r], cg, (size_t)NL, words, tid, B, min(j0 + r + P, n - 1));
        }
    }
#pragma unroll
    for (int r = 0; r < P; ++r)
        if (j0 + r < n) sweep(ring[r]);
    __syncthreads();
    // the samples of the pass, in the first wavefront: lane l takes samples
    // l, l + 64, ...; the moment sums are merged across lanes exactly
    if (tid < 64 && n_samples > 0) {
        const int64_t nn = (int64_t)L * (int64_t)L;
        const int64_t idx = state.series_idx;
        Moments part = {};
        for (int k = tid; k < n_samples; k += 64) {
            const int64_t E = 2 * (int64_t)stage[2 * k] - 2 * nn, M = 2 * (int64_t)stage[2 * k + 1] - nn;
            if (d.series_E) d.series_E[idx + k] = E;
            if (d.series_M) d.series_M[idx + k] = M;
            add_sample(part, E, M);
        }
        wave_merge_moments(part);
        if (tid == 0) {
            Moments m = state.mom;
            merge_moments(m, part);
            state.mom = m;
            const int k = n_samples - 1;
            state.last_E = 2 * (int64_t)stage[2 * k] - 2 * nn;
            state.last_M = 2 * (int64_t)stage[2 * k + 1] - nn;
            state.series_idx = idx + n_samples;
        }
    }
    for (int i = tid; i < NL; i += B) G[i] = T[i];
}

int32_t wave_apply_words_per_thread(int32_t L, int32_t N, int32_t block) {
    const int32_t w = (N * (L / 2) + block - 1) / block;
    return w <= 1 ? 1 : w <= 2 ? 2 : w <= 4 ? 4 : 0;
}

size_t wave_apply_lds_bytes(int32_t NL, int32_t max_samples) { return (size_t)NL * 8 + (size_t)max_samples * 8; }

hipError_t allow_wave_apply_lds(int device) {
    const int lim = (int)resident_lds_limit(device);
    const void* fs[] = {reinterpret_cast<const void*>(&k_wave_apply<1, 8, true>),
                        reinterpret_cast<const void*>(&k_wave_apply<2, 8, true>),
                        reinterpret_cast<const void*>(&k_wave_apply<4, 4, true>),
                        reinterpret_cast<const void*>(&k_wave_apply<1, 8, false>),
                        reinterpret_cast<const void*>(&k_wave_apply<2, 8, false>),
                        reinterpret_cast<const void*>(&k_wave_apply<4, 4, false>)};
    for (const void* f : fs) {
        const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lim);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_draw_codes(const LatticeDesc* descs, const LatticeState* states, const DrawLat* lats, int32_t n_lats,
                             int32_t max_n_draw, uint64_t* codes, int32_t sweep_off, int32_t S, hipStream_t s) {
    if (n_lats <= 0 || S <= 0) return hipSuccess;
    const int64_t bpl = ((int64_t)S * max_n_draw + kDrawBlock - 1) / kDrawBlock;
    if (bpl * n_lats > 0x7FFFFFFF || (int64_t)S * max_n_draw > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_draw_codes, dim3((unsigned)(bpl * n_lats)), dim3(kDrawBlock), 0, s, descs, states, lats, codes,
                       (int32_t)bpl, sweep_off, S);
    return hipGetLastError();
}

hipError_t launch_wave_apply(int wmax, int block, const LatticeDesc* descs, LatticeState* states, const DrawLat* lats,
                             int32_t n_lats, const uint64_t* codes, int32_t sweep_off, int32_t S, int32_t every,
                             size_t lds_bytes, hipStream_t s) {
    if (n_lats <= 0 || S <= 0) return hipSuccess;
    if (block < 64 || block > kApplyMaxBlock || block % 64) return hipErrorInvalidValue;
    const dim3 grid(n_lats), blk(block);
#define ISING_WAVE_APPLY(W_, P_)                                                                                 \
    if (block == 64)                                                                                             \
        hipLaunchKernelGGL((k_wave_apply<W_, P_, true>), grid, blk, lds_bytes, s, descs, states, lats, codes,   \
                           sweep_off, S, every);                                                                 \
    else                                                                                                         \
        hipLaunchKernelGGL((k_wave_apply<W_, P_, false>), grid, blk, lds_bytes, s, descs, states, lats, codes,  \
                           sweep_off, S, every);
    switch (wmax) {
        case 1: ISING_WAVE_APPLY(1, 8) break;
        case 2: ISING_WAVE_APPLY(2, 8) break;
        case 4: ISING_WAVE_APPLY(4, 4) break;
        default: return hipErrorInvalidValue;
    }
#undef ISING_WAVE_APPLY
    return hipGetLastError();
}

}  // namespace ising
