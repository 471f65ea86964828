// Small lattices held whole in one workgroup's LDS, with the random draws
// taken off the sweep's critical path.
//
// A lattice of a few hundred words leaves most of a workgroup idle in each
// half-sweep, and one word's update is a long dependent chain (five Philox
// blocks and 21 acceptance codes), so a half-sweep lasts as long as that
// chain.  The acceptance codes do not depend on the spins (Table 1's
// classes are applied to them only at the flip), so they are drawn ahead:
// for a batch of sweeps, every thread of the workgroup computes codes --
// all words, both colours, every sweep of the batch -- into LDS; then the
// sweeps run from LDS, each half-sweep only loading a word, its neighbours
// and its code and flipping, with a workgroup barrier between half-sweeps.
// Samples (E, M after a sweep) are reduced in the workgroup and added to the
// lattice's sums directly.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ising_device.hpp"
#include "ising_launch.hpp"
#include "ising_lds_word.hpp"
#include "ising_moments.hpp"

namespace ising {

namespace {

constexpr int kSmallMaxBlock = 1024;
constexpr int kSmallMaxBatch = 64;  // sweeps whose codes are drawn together

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

}  // namespace

// One workgroup per listed lattice (ids), K sweeps (each lattice at most its
// sweep limit); a sample after local sweep s when (s + 1) % every == 0
// (every > 0).  LDS: the words [N][L], then the codes of `batch` sweeps
// [batch][N][L] (bit 3k: code >= 1 at field k, bit 3k + 1: code = 2).
__global__ void __launch_bounds__(kSmallMaxBlock) k_small(const LatticeDesc* __restrict__ descs,
                                                           LatticeState* __restrict__ states,
                                                           const int32_t* __restrict__ ids, int32_t K, int32_t every,
                                                           int32_t batch) {
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t red[2 * (kSmallMaxBlock / 64)];
    const int32_t lat = ids[blockIdx.x];
    const LatticeDesc& d = descs[lat];
    LatticeState& state = states[lat];
    const int L = d.L, N = d.N, istar = d.istar, sh_star = d.sh_star;
    const int pstar = (L - 1) / N;
    const int NL = N * L;
    uint64_t* __restrict__ T = lds;
    uint64_t* __restrict__ codes = lds + NL;
    const int tid = threadIdx.x, B = blockDim.x;
    uint64_t* __restrict__ G = d.W;
    for (int i = tid; i < NL; i += B) T[i] = G[i];
    const uint64_t t0 = state.t;
    const int n_sweeps = min(K, d.sweep_limit);
    const RoundKeys rk = round_keys(d.k0, d.k1);
    // sample accumulators stay in thread 0's registers for the whole launch
    int64_t series_idx = 0, last_E = 0, last_M = 0;
    Moments mom = {};
    if (tid == 0) {
        series_idx = state.series_idx;
        mom = state.mom;
        last_E = state.last_E;
        last_M = state.last_M;
    }
    const int groups = (L + 7) >> 3;  // 8-column groups of a row
    const int n_draw = 2 * N * groups;  // draw items per sweep: (colour, row, group)
    const float rcp_draw = 1.0f / (float)n_draw, rcp_g = 1.0f / (float)groups, rcp_half = 2.0f / (float)L;
    const int half = L >> 1;  // words of one colour per row
    __syncthreads();

    // the next sampled local sweep, counted rather than divided out per sweep
    int64_t next_sample = every > 0 ? every - 1 : -1;
    for (int s0 = 0; s0 < n_sweeps; s0 += batch) {
        const int nb = min(batch, n_sweeps - s0);
        // draws: item (sweep, colour, row, group) -> the codes of the group's
        // four words of that colour (one position-20 block shared by them)
        for (int f = tid; f < nb * n_draw; f += B) {
            int j, r;
            divmod_small(f, n_draw, rcp_draw, j, r);
            const int c = r >= N * groups ? 1 : 0;
            int I, grp;
            divmod_small(r - c * N * groups, groups, rcp_g, I, grp);
            const uint64_t t = t0 + (uint64_t)(s0 + j);
            const int n_live = pstar + (I <= istar ? 1 : 0);
            const uint32_t t_lo = (uint32_t)t, t_hi = (uint32_t)(t >> 32);
            const int par = (I + c) & 1;
            uint4 u5 = make_uint4(0u, 0u, 0u, 0u);
            if (n_live == 21) {
                const U4 r5 = philox_lane_c1(t_lo, (uint32_t)I * (uint32_t)L + (uint32_t)(8 * grp + par), t_hi,
                                             5u | (1u << 3), d.k0, d.k1, rk);
                u5 = make_uint4(r5.x, r5.y, r5.z, r5.w);
            }
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int J = 8 * grp + par + 2 * m;
                if (J >= L) break;
                Codes cd = {0u, 0u, 0u};
#pragma unroll
                for (int g = 0; g < 5; ++g) {
                    if (4 * g < n_live) {
                        const U4 rr = philox_lane_c1(t_lo, (uint32_t)I * (uint32_t)L + (uint32_t)J, t_hi,
                                                     (uint32_t)g | (1u << 3), d.k0, d.k1, rk);
                        append_draw(cd, 4 * g + 0, rr.x, d.t4, d.t8);
                        append_draw(cd, 4 * g + 1, rr.y, d.t4, d.t8);
                        append_draw(cd, 4 * g + 2, rr.z, d.t4, d.t8);
                        append_draw(cd, 4 * g + 3, rr.w, d.t4, d.t8);
                    } else {
#pragma unroll
                        for (int k = 0; k < 4; ++k) append_code(cd, 4 * g + k, 0u);
                    }
                }
                append_draw(cd, 20, pick4(u5, (uint32_t)m), d.t4, d.t8);  // a dead slot when n_live < 21
                codes[(size_t)j * NL + I * L + J] = assemble_codes(cd);
            }
        }
        __syncthreads();
        // the sweeps of the batch, from LDS
        for (int j = 0; j < nb; ++j) {
            const bool meas = s0 + j == next_sample;
            if (meas) next_sample += every;
            const uint64_t* __restrict__ cj = codes + (size_t)j * NL;
            for (int c = 0; c < 2; ++c) {
                uint32_t anti = 0, ups = 0;
                for (int f = tid; f < N * half; f += B) {
                    int I, q;
                    divmod_small(f, half, rcp_half, I, q);
                    const int J = 2 * q + ((I + c) & 1);
                    const Nbhd nb = lds_nbhd(T, L, N, istar, I, J, J == 0 ? L - 1 : J - 1, J == L - 1 ? 0 : J + 1);
                    const int n_live = pstar + (I <= istar ? 1 : 0);
                    const uint64_t live = kSpinBits & (~0ull << (3 * (21 - n_live)));
                    const uint64_t up = up_of(nb, I, sh_star);
                    const uint64_t dn = down_of(nb, I, N, istar, sh_star);
                    const uint64_t nw = nb.w ^ flip_mask(nb.w, up, dn, nb.lf, nb.rt, cj[I * L + J], live);
                    T[I * L + J] = nw;
                    if (meas && c == 1) measure_word(nw, up, dn, nb.lf, nb.rt, live, anti, ups);
                }
                if (meas && c == 1) {
                    anti = wave_sum_u32(anti);
                    ups = wave_sum_u32(ups);
                    if (lane_id() == 0) {
                        red[2 * (tid >> 6)] = anti;
                        red[2 * (tid >> 6) + 1] = ups;
                    }
                }
                __syncthreads();
                if (meas && c == 1 && tid == 0) {
                    uint64_t A = 0, U = 0;
                    for (int wv = 0; wv < (B + 63) / 64; ++wv) {
                        A += red[2 * wv];
                        U += red[2 * wv + 1];
                    }
                    const int64_t n = (int64_t)L * (int64_t)L;
                    const int64_t E = 2 * (int64_t)A - 2 * n, M = 2 * (int64_t)U - n;
                    last_E = E;
                    last_M = M;
                    add_sample(mom, E, M);
                    if (d.series_E) d.series_E[series_idx] = E;
                    if (d.series_M) d.series_M[series_idx] = M;
                    series_idx += 1;
                }
            }
        }
        // the next batch's draws overwrite the codes only after every thread
        // has passed the last half-sweep's barrier
    }
    if (tid == 0) {
        state.series_idx = series_idx;
        state.mom = mom;
        state.last_E = last_E;
        state.last_M = last_M;
    }
    for (int i = tid; i < NL; i += B) G[i] = T[i];
}

size_t small_lds_bytes(int32_t L, int32_t N, int32_t batch) { return (size_t)N * (size_t)L * 8 * (1 + batch); }

size_t small_lds_limit(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return 0;
    const size_t static_bytes = sizeof(uint32_t) * 2 * (kSmallMaxBlock / 64) + 128;
    return v > (int)static_bytes ? (size_t)v - static_bytes : 0;
}

hipError_t allow_small_lds(int device) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_small), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)small_lds_limit(device));
}

hipError_t launch_small(int block, const LatticeDesc* descs, LatticeState* states, const int32_t* ids, int32_t n_ids,
                        int32_t K, int32_t every, int32_t batch, size_t lds_bytes, hipStream_t s) {
    if (n_ids <= 0 || K <= 0) return hipSuccess;
    if (block < 64 || block > kSmallMaxBlock || block % 64 || batch < 1 || batch > kSmallMaxBatch)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_small, dim3(n_ids), dim3(block), lds_bytes, s, descs, states, ids, K, every, batch);
    return hipGetLastError();
}

}  // namespace ising
