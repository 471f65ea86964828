// Several sweeps per launch on LDS tiles with redundant halos (temporal
// blocking of the checkerboard sweep).
//
// A tile is every word row of a band of word columns: the interior columns
// [c0, c0 + w) and a halo of R = 2K columns on each side (columns wrap
// modulo L).  One workgroup loads the tile into LDS, runs K sweeps on it --
// 2K half-sweeps separated by workgroup barriers -- and stores the interior
// back.  A half-sweep changes a word from its four neighbours, so after
// half-sweep s only the columns [s, width - s) of the tile still hold the
// true state; with R = 2K the interior is exact after the last one, and each
// half-sweep only updates the columns that stay exact.  Every random number
// is a function of (seed, sweep, site), so the halo columns draw the same
// numbers as the tiles that own them and the result equals the plain
// half-sweep launches bit for bit.  This is the one-GPU form of the paper's
// sub-lattice with ghost columns (Sections 4 and 5.2, Figs. 3 and 5): the
// ghost region is R columns wide instead of one, so that the neighbouring
// tiles need to meet only once every K sweeps, at a launch boundary.
//
// A tile with w >= L holds the whole lattice: no halo, columns wrap inside
// LDS, and any number of sweeps fits in one launch.
//
// The workgroups of a launch do not all start together (more tiles than fit
// on the chip at once, or other work holding compute units), so a tile may
// finish and store its interior before a neighbour has loaded it as halo.
// The halo columns are therefore copied out of the lattice words by a small
// kernel ahead of the tiles (k_tile_halos), and a tile loads its halo from
// that copy and only its own interior from the lattice words, which no
// other tile writes.
//
// All word rows of a column are in the tile, so the periodic wrap between
// the first and last word rows, including the row-(L-1) patch, is resolved
// inside LDS exactly as in the global-memory kernels (fix_up, fix_down).
//
// Position 20 of a word draws from Philox block 5 keyed by its 8-column
// group and the word's colour, one block shared by the group's four words
// of that colour.  Those blocks are drawn once per group, row and
// half-sweep into an LDS table during the previous half-sweep (the draws do
// not depend on the state), and every word reads its output there.
#include <hip/hip_runtime.h>

#include "ising_device.hpp"
#include "ising_launch.hpp"
#include "ising_lds_word.hpp"
#include "ising_moments.hpp"

namespace ising {

namespace {

constexpr int kTileMaxBlock = 1024;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Columns of the tile: local column x is global column gx0 + x (mod L).  The
// 8-column groups it touches are numbered in local order ("slots"): the
// groups from gx0's group up to the lattice's last group, then, when the
// tile wraps, the groups from column 0 on.
struct TileCols {
    int L, gx0, width, A, g_first;
    __device__ __forceinline__ int col(int x) const {
        const int u = gx0 + x;
        return u < L ? u : u - L;
    }
    __device__ __forceinline__ int slot(int x) const {
        const int u = gx0 + x;
        return u < L ? (u >> 3) - g_first : A + ((u - L) >> 3);
    }
    __device__ __forceinline__ int group_of_slot(int s) const { return s < A ? g_first + s : s - A; }
};

// Sweeps of a tile of lattice d in launch a (<= 0: the lattice has finished
// the sweeps of its chunk).
__device__ __forceinline__ int tile_sweeps_of(const TileLaunch& a, const LatticeDesc& d) {
    return a.states ? min(a.K, d.sweep_limit - (int)a.sweep_off) : a.K;
}

}  // namespace

// ---------------------------------------------------------------------------
// The halo columns of every tile narrower than its lattice, as they stand
// before the launch: tile b's words at H[b stride + (side N + I) R + k] for
// word row I and k < R = 2K, side 0 the R columns left of the interior
// (global columns c0 - R + k), side 1 the R columns right of it (c0 + w + k),
// modulo L.  One workgroup per tile.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_tile_halos(TileLaunch a, uint64_t* __restrict__ H, int64_t stride) {
    const TileWork tw = a.tiles[blockIdx.x];
    const LatticeDesc& d = a.descs[tw.lattice];
    const int L = d.L, N = d.N;
    if (tw.w >= L) return;
    const int K = tile_sweeps_of(a, d);
    if (K <= 0) return;
    const int R = 2 * K, NR = N * R;
    const uint64_t* __restrict__ G = d.W;
    uint64_t* __restrict__ Hb = H + (size_t)blockIdx.x * (size_t)stride;
    for (int i = threadIdx.x; i < 2 * NR; i += blockDim.x) {
        const int side = i >= NR ? 1 : 0, r = i - side * NR;
        const int I = r / R, k = r - I * R;
        int u = side ? tw.c0 + tw.w + k : tw.c0 - R + k;
        u = u < 0 ? u + L : (u >= L ? u - L : u);
        Hb[i] = G[(size_t)((uint32_t)I * (uint32_t)L + (uint32_t)u)];
    }
}

// ---------------------------------------------------------------------------
// One workgroup per tile.  LDS: the tile's words [N][width], then two tables
// of position-20 blocks [slot][N] (uint4), the one read by the current
// half-sweep and the one filled for the next.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kTileMaxBlock) k_tiles(TileLaunch a, const uint64_t* __restrict__ H,
                                                          int64_t stride) {
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t red[2 * (kTileMaxBlock / 64)];
    const TileWork tw = a.tiles[blockIdx.x];
    const LatticeDesc& d = a.descs[tw.lattice];
    const int L = d.L, N = d.N, istar = d.istar, sh_star = d.sh_star;
    const int pstar = (L - 1) / N;  // rows I <= istar have pstar + 1 live positions, the others pstar
    uint64_t t0;
    uint32_t t4, t8, k0, k1;
    int K = a.K;
    if (a.states) {
        t0 = a.states[tw.lattice].t + a.sweep_off;
        k0 = d.k0;
        k1 = d.k1;
        t4 = d.t4;
        t8 = d.t8;
        K = tile_sweeps_of(a, d);
        if (K <= 0) return;  // this lattice has finished the sweeps of the chunk
    } else {
        t0 = a.t0;
        k0 = a.k0;
        k1 = a.k1;
        t4 = a.t4;
        t8 = a.t8;
    }
    const bool whole = tw.w >= L;
    const int R = whole ? 0 : 2 * K;
    const int width = whole ? L : tw.w + 2 * R;
    TileCols tc;
    tc.L = L;
    tc.gx0 = whole ? 0 : (tw.c0 - R < 0 ? tw.c0 - R + L : tw.c0 - R);
    tc.width = width;
    tc.g_first = tc.gx0 >> 3;
    tc.A = ((L - 1) >> 3) - tc.g_first + 1;
    const int n_slots = tc.slot(width - 1) + 1;
    uint64_t* __restrict__ T = lds;
    uint4* __restrict__ u5tab = reinterpret_cast<uint4*>(lds + (size_t)N * width);
    const int tid = threadIdx.x, B = blockDim.x;
    const uint64_t* __restrict__ G = d.W;
    const RoundKeys rk = round_keys(k0, k1);

    // load the tile, eight loads in flight per thread: the interior from the
    // lattice words, the halo from the copy taken ahead of the launch
    {
        constexpr int kInFlight = 8;
        const float rcp = 1.0f / (float)width;
        const int n = N * width;
        const uint64_t* __restrict__ Hb = H + (whole ? 0 : (size_t)blockIdx.x * (size_t)stride);
        for (int i0 = tid; i0 < n; i0 += kInFlight * B) {
            uint64_t v[kInFlight];
#pragma unroll
            for (int k = 0; k < kInFlight; ++k) {
                const int i = i0 + k * B;
                if (i < n) {
                    int I, x;
                    divmod_small(i, width, rcp, I, x);
                    if (whole || (x >= R && x < R + tw.w))
                        v[k] = G[(size_t)((uint32_t)I * (uint32_t)L + (uint32_t)tc.col(x))];
                    else
                        v[k] = Hb[(x < R ? I : N + I) * R + (x < R ? x : x - R - tw.w)];
                }
            }
#pragma unroll
            for (int k = 0; k < kInFlight; ++k)
                if (i0 + k * B < n) T[i0 + k * B] = v[k];
        }
    }

    // position-20 blocks of half-sweep s (1-based) into table buf: items
    // (row, slot) over the slots of the columns that half-sweep updates
    auto u5_items = [&](int s, int& slot_lo) {
        const int lo = whole ? 0 : s, hi = whole ? width : width - s;
        slot_lo = tc.slot(lo);
        return tc.slot(hi - 1) - slot_lo + 1;
    };
    const bool all_blocks = pstar >= 16;  // every row has more than 16 live positions
    auto sweep_of = [&](int s) {  // the shared parameters of half-sweep s (1-based)
        const uint64_t t = t0 + (uint64_t)((s - 1) >> 1);
        return LdsSweep{L, N, istar, sh_star, pstar, (uint32_t)t, (uint32_t)(t >> 32), k0, k1, t4, t8, all_blocks};
    };
    auto u5_draw = [&](int s, int item, int n_sl, float rcp_sl, int slot_lo) {
        int I, k;
        divmod_small(item, n_sl, rcp_sl, I, k);
        const int sl = slot_lo + k;
        if (pstar + (I <= istar ? 1 : 0) < 21) return;  // position 20 of this row is a dead slot
        u5tab[(size_t)((s & 1) * n_slots + sl) * N + I] = block5(sweep_of(s), rk, I, tc.group_of_slot(sl), (s - 1) & 1);
    };
    {
        int slot_lo;
        const int n_sl = u5_items(1, slot_lo);
        const float rcp_sl = 1.0f / (float)n_sl;
        for (int i = tid; i < N * n_sl; i += B) u5_draw(1, i, n_sl, rcp_sl, slot_lo);
    }
    __syncthreads();

    const int n_steps = 2 * K;
    for (int s = 1; s <= n_steps; ++s) {
        const int c = (s - 1) & 1;
        const int j = (s - 1) >> 1;  // sweep of the launch
        const LdsSweep sw = sweep_of(s);
        const bool meas = c == 1 && ((a.sample_mask >> j) & 1u);
        const int lo = whole ? 0 : s, hi = whole ? width : width - s;
        const int P = (hi - lo) >> 1;  // words of this colour per row in [lo, hi)
        const int n_words = N * P;
        const float rcp = 1.0f / (float)P;
        const uint4* __restrict__ u5cur = u5tab + (size_t)(s & 1 ? 1 : 0) * n_slots * N;
        uint32_t anti = 0, ups = 0;
        for (int f = tid; f < n_words; f += B) {
            int I, q;
            divmod_small(f, P, rcp, I, q);
            const int x = lo + 2 * q + ((lo + tc.gx0 + I + c) & 1);
            const int J = tc.col(x);
            const int xl = whole && x == 0 ? L - 1 : x - 1;
            const int xr = whole && x == L - 1 ? 0 : x + 1;
            const Nbhd nb = lds_nbhd(T, width, N, istar, I, x, xl, xr);
            const uint32_t u20 = pick4(u5cur[(size_t)tc.slot(x) * N + I], ((uint32_t)J >> 1) & 3u);
            const bool interior = whole || (x >= R && x < R + tw.w);
            T[I * width + x] = lds_word_update(sw, rk, nb, I, J, u20, meas, interior, anti, ups);
        }
        if (s < n_steps) {  // the next half-sweep's position-20 blocks
            int nx_slot_lo;
            const int nx_sl = u5_items(s + 1, nx_slot_lo);
            const float rcp_sl = 1.0f / (float)nx_sl;
            for (int f = tid; f < N * nx_sl; f += B) u5_draw(s + 1, f, nx_sl, rcp_sl, nx_slot_lo);
        }
        if (meas) {  // this tile's share of the sample: bonds and up spins of its interior
            anti = wave_sum_u32(anti);
            ups = wave_sum_u32(ups);
            if (lane_id() == 0) {
                red[2 * (tid >> 6)] = anti;
                red[2 * (tid >> 6) + 1] = ups;
            }
        }
        __syncthreads();
        if (meas && tid == 0) {
            uint32_t sa_ = 0, su = 0;
            for (int wv = 0; wv < (B + 63) / 64; ++wv) {
                sa_ += red[2 * wv];
                su += red[2 * wv + 1];
            }
            const int ord = __popc(a.sample_mask & ((1u << j) - 1u));
            a.partials[(size_t)ord * a.n_tiles + tw.part] = {sa_, su};
        }
    }

    // store the interior
    {
        const int w = whole ? L : tw.w;
        const float rcp = 1.0f / (float)w;
        uint64_t* __restrict__ Gw = d.W;
        for (int i = tid; i < N * w; i += B) {
            int I, xi;
            divmod_small(i, w, rcp, I, xi);
            const int x = R + xi;
            Gw[(size_t)((uint32_t)I * (uint32_t)L + (uint32_t)tc.col(x))] = T[I * width + x];
        }
    }
}

// E and M of n_samples samples of one lattice from the tiles' partial sums
// (sample k in partials[k n_tiles .. k n_tiles + n_tiles)), in sample order:
// series entries idx0 + k (each series may be null), the moment sums *mom
// (may be null), and the last sample into out_EM (may be null).  One
// workgroup.
__global__ void __launch_bounds__(256) k_finalize_samples(const Partial* __restrict__ partials, int32_t n_tiles,
                                                          int32_t n_samples, int32_t L, int64_t* series_E,
                                                          int64_t* series_M, int64_t idx0, Moments* mom,
                                                          int64_t* out_EM) {
    __shared__ unsigned long long red[2 * 4];
    for (int k = 0; k < n_samples; ++k) {
        unsigned long long anti = 0, ups = 0;
        for (int i = threadIdx.x; i < n_tiles; i += blockDim.x) {
            const Partial p = partials[(size_t)k * n_tiles + i];
            anti += p.anti;
            ups += p.ups;
        }
        anti = wave_sum_u64(anti);
        ups = wave_sum_u64(ups);
        if (lane_id() == 0) {
            red[2 * (threadIdx.x >> 6)] = anti;
            red[2 * (threadIdx.x >> 6) + 1] = ups;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long A = 0, U = 0;
            for (int wv = 0; wv < (int)(blockDim.x + 63) / 64; ++wv) {
                A += red[2 * wv];
                U += red[2 * wv + 1];
            }
            const int64_t n = (int64_t)L * (int64_t)L;
            const int64_t E = 2 * (int64_t)A - 2 * n, M = 2 * (int64_t)U - n;
            if (series_E) series_E[idx0 + k] = E;
            if (series_M) series_M[idx0 + k] = M;
            if (mom) add_sample(*mom, E, M);
            if (out_EM && k == n_samples - 1) {
                out_EM[0] = E;
                out_EM[1] = M;
            }
        }
        __syncthreads();
    }
}

// The samples of one tile launch for every tiled lattice of a batch, one
// wavefront per listed lattice: sample ordinal k (bit j of sample_mask, in
// order) is the sum of the lattice's tile partials partials[k n_tiles +
// part_begin ...], which becomes its next series entry, a moment sample and
// its last E, M.  Samples past a lattice's sweep limit were not taken.
__global__ void __launch_bounds__(64) k_finalize_tiles(const LatticeDesc* __restrict__ descs,
                                                       LatticeState* __restrict__ states,
                                                       const int32_t* __restrict__ ids,
                                                       const Partial* __restrict__ partials, int32_t n_tiles,
                                                       uint32_t sample_mask, uint32_t sweep_off) {
    const int32_t lat = ids[blockIdx.x];
    const LatticeDesc& d = descs[lat];
    LatticeState& st = states[lat];
    uint32_t m = sample_mask;
    for (int ord = 0; m; ++ord) {
        const int j = __ffs(m) - 1;
        m &= m - 1u;
        if ((int)(sweep_off + (uint32_t)j) >= d.sweep_limit) continue;
        const Partial* __restrict__ part = partials + (size_t)ord * n_tiles + d.part_begin;
        unsigned long long anti = 0, ups = 0;
        for (int i = lane_id(); i < d.part_count; i += 64) {
            anti += part[i].anti;
            ups += part[i].ups;
        }
        anti = wave_sum_u64(anti);
        ups = wave_sum_u64(ups);
        if (lane_id() == 0) {
            const int64_t n = (int64_t)d.L * (int64_t)d.L;
            const int64_t E = 2 * (int64_t)anti - 2 * n, M = 2 * (int64_t)ups - n;
            const int64_t idx = st.series_idx;
            st.last_E = E;
            st.last_M = M;
            add_sample(st.mom, E, M);
            if (d.series_E) d.series_E[idx] = E;
            if (d.series_M) d.series_M[idx] = M;
            st.series_idx = idx + 1;
        }
    }
}

size_t tile_lds_bytes(int32_t L, int32_t N, int32_t w, int32_t K) {
    const bool whole = w >= L;
    const int64_t width = whole ? L : (int64_t)w + 4 * K;
    // slots: the groups of `width` consecutive columns, one more where the
    // columns wrap past a lattice end that is not a multiple of 8
    const int64_t slots = whole ? (L + 7) / 8 : width / 8 + 3;
    return (size_t)(8 * (int64_t)N * width + 2 * 16 * slots * (int64_t)N);
}

size_t tile_lds_limit(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return 0;
    const size_t static_bytes = sizeof(uint32_t) * 2 * (kTileMaxBlock / 64) + 128;
    return v > (int)static_bytes ? (size_t)v - static_bytes : 0;
}

hipError_t allow_tile_lds(int device) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tiles), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)tile_lds_limit(device));
}

int64_t tile_halo_stride(int32_t N, int32_t K) { return 4 * (int64_t)K * (int64_t)N; }

hipError_t launch_tiles(const TileLaunch& a, int32_t n_tiles_launched, int block, size_t lds_bytes, uint64_t* halo,
                        int64_t halo_stride, hipStream_t s) {
    if (n_tiles_launched <= 0 || a.K <= 0) return hipSuccess;
    if (block < 64 || block > kTileMaxBlock || block % 64 || a.K > kTileMaxSweeps) return hipErrorInvalidValue;
    if (halo_stride > 0) {
        if (!halo) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_tile_halos, dim3(n_tiles_launched), dim3(256), 0, s, a, halo, halo_stride);
    }
    hipLaunchKernelGGL(k_tiles, dim3(n_tiles_launched), dim3(block), lds_bytes, s, a, halo, halo_stride);
    return hipGetLastError();
}

hipError_t launch_finalize_samples(const Partial* partials, int32_t n_tiles, int32_t n_samples, int32_t L,
                                   int64_t* series_E, int64_t* series_M, int64_t idx0, Moments* mom, int64_t* out_EM,
                                   hipStream_t s) {
    if (n_samples <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_samples, dim3(1), dim3(256), 0, s, partials, n_tiles, n_samples, L, series_E,
                       series_M, idx0, mom, out_EM);
    return hipGetLastError();
}

}  // namespace ising

namespace ising {

hipError_t launch_finalize_tiles(const LatticeDesc* descs, LatticeState* states, const int32_t* ids, int32_t n_lat,
                                 const Partial* partials, int32_t n_tiles, uint32_t sample_mask, uint32_t sweep_off,
                                 hipStream_t s) {
    if (n_lat <= 0 || sample_mask == 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_tiles, dim3(n_lat), dim3(64), 0, s, descs, states, ids, partials, n_tiles,
                       sample_mask, sweep_off);
    return hipGetLastError();
}

}  // namespace ising
