// Resident LDS tiles that exchange their boundary columns: many sweeps per
// launch with no redundant work.
//
// Every word row of a band of word columns [c0, c0 + w) of a lattice stays in
// one workgroup's LDS for all sweeps of a launch, beside two ghost columns
// (c0 - 1 and c0 + w, modulo L) holding copies of the neighbouring tiles'
// boundary words.  This is the paper's decomposition (Sections 4 and 5.2,
// Figs. 3 and 5: each process owns a vertical strip of the word lattice and
// trades its border columns with the processes beside it), with the
// workgroups of one GPU in the place of the MPI processes and the
// checkerboard in the place of the two-phase protocol.  Half-sweep s of
// colour c in a tile is one pass over its words of colour c:
//   - the boundary words (local columns 1 and w) come first; each reads its
//     ghost neighbour straight from the neighbouring tile's publication of
//     half-sweep s - 1 (from LDS in a launch's first half-sweep), and is
//     published at once to an exchange buffer in global memory; the thread
//     that publishes the last of them raises the tile's flag (to a value
//     that grows with the lattice's sweep counter and the half-sweep);
//   - then the interior words (columns 2 .. w - 1), while the boundary words
//     travel, and the Philox blocks of the next half-sweep's position 20
//     (and, with at most two words of a colour per thread, the acceptance
//     codes of the next half-sweep's words, drawn into an LDS code table
//     while each word's own loads are in flight);
//   - at the end, before the workgroup barrier, one thread waits until both
//     neighbours' flags show this half-sweep (their publications are
//     normally done long before).
// Only colour-c words are exchanged, because the next half-sweep only reads
// those from a ghost column.  The exchange buffer alternates between two
// halves on the half-sweep's parity: a tile overwrites a half two
// half-sweeps later, after its neighbours have raised their flags past the
// half-sweep that read it (each publisher reads its ghost word before it
// publishes).
//
// Every tile of a launch must be resident at once (the host launches at most
// as many tiles as the device holds).  Each wait is bounded in time: when
// it expires the launch sets an error word and every tile stops waiting, so
// a launch always ends; the host reports the error.
//
// A lattice with a single tile (w = L) keeps all its columns in LDS and
// wraps them there: no exchange at all.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "ising_device.hpp"
#include "ising_launch.hpp"
#include "ising_lds_word.hpp"
#include "ising_moments.hpp"

namespace ising {

namespace {

constexpr int kPersistMaxBlock = 1024;
constexpr uint32_t kMaxPolls = 1u << 21;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t clock_ticks() { return __builtin_amdgcn_s_memrealtime(); }

// LDS seen as what it is (address space 3), so that 32-bit LDS addresses
// can be kept in registers and loaded from with no base added
typedef __attribute__((address_space(3))) uint64_t lds_u64;
typedef __attribute__((address_space(3))) uint32_t lds_u32;
__device__ __forceinline__ uint32_t lds_addr(const lds_u64* p) { return (uint32_t)(size_t)p; }
__device__ __forceinline__ uint64_t lds_load64(uint32_t addr) { return *(const lds_u64*)(size_t)addr; }
__device__ __forceinline__ void lds_store64(uint32_t addr, uint64_t v) { *(lds_u64*)(size_t)addr = v; }
__device__ __forceinline__ uint32_t lds_load32(uint32_t addr) { return *(const lds_u32*)(size_t)addr; }

// One word item of a half-sweep: the LDS addresses of the word and of its
// neighbourhood words, the byte offset of its position-20 uniform in the
// table of the half-sweep, its Philox counter word I L + J, its row and its
// side (-1 interior, 0 the left boundary column, 1 the right one).
struct WordItem {
    uint32_t w, lf, rt, up, dn, patch, u20, c1;
    int32_t I, side;
    uint32_t code;  // byte offset of its codes in a half-sweep's code table
};


}  // namespace

__global__ void __launch_bounds__(kPersistMaxBlock) k_persist(PersistLaunch a) {
    extern __shared__ uint64_t lds[];
    __shared__ uint32_t red[2 * (kPersistMaxBlock / 64)];
    __shared__ int stop;
    __shared__ uint32_t published;  // boundary words published in this launch
    const PersistTile tp = a.tiles[blockIdx.x];
    const LatticeDesc& d = a.descs[tp.lattice];
    const int L = d.L, N = d.N, istar = d.istar, sh_star = d.sh_star;
    const int pstar = (L - 1) / N;
    uint64_t t0;
    uint32_t t4, t8, k0, k1;
    if (a.states) {
        t0 = a.states[tp.lattice].t + a.sweep_off;
        k0 = d.k0;
        k1 = d.k1;
        t4 = d.t4;
        t8 = d.t8;
    } else {
        t0 = a.t0;
        k0 = a.k0;
        k1 = a.k1;
        t4 = a.t4;
        t8 = a.t8;
    }
    const int K = a.K;
    const bool whole = tp.w >= L;
    const int w = whole ? L : tp.w;
    const int width = whole ? L : w + 2;  // local column x <-> global c0 - 1 + x (halo form)
    const int gx0 = whole ? 0 : (tp.c0 == 0 ? L - 1 : tp.c0 - 1);
    auto col = [&](int x) {
        const int u = gx0 + x;
        return u < L ? u : u - L;
    };
    // position-20 blocks: one per (8-column group, row) of the interior
    // columns, for the current half-sweep
    const int xi0 = whole ? 0 : 1, xi1 = whole ? L : w + 1;  // interior local columns [xi0, xi1)
    const int g_lo = col(xi0) >> 3;
    const int g_hi_raw = col(xi1 - 1) >> 3;
    // the interior never wraps past the lattice end (tiles start at c0 >= 0
    // and end at c0 + w <= L), so its groups are g_lo .. g_hi_raw
    const int n_groups = g_hi_raw - g_lo + 1;
    uint64_t* __restrict__ T = lds;
    // two tables [n_groups][N]: this half-sweep's and the next one's
    uint4* __restrict__ u5tab = reinterpret_cast<uint4*>(lds + (size_t)N * width);
    const int tid = threadIdx.x, B = blockDim.x;
    const RoundKeys rk = round_keys(k0, k1);
    const bool all_blocks = pstar >= 16;
    auto sweep_of = [&](int hs) {  // half-sweep hs (0-based) of the launch
        const uint64_t t = t0 + (uint64_t)(hs >> 1);
        return LdsSweep{L, N, istar, sh_star, pstar, (uint32_t)t, (uint32_t)(t >> 32), k0, k1, t4, t8, all_blocks};
    };
    if (tid == 0) {
        stop = 0;
        published = 0;
    }

    // load the band and its ghost columns, eight loads in flight per thread
    {
        constexpr int kInFlight = 8;
        const float rcp = 1.0f / (float)width;
        const int n = N * width;
        const uint64_t* __restrict__ G = d.W;
        for (int i0 = tid; i0 < n; i0 += kInFlight * B) {
            uint64_t v[kInFlight];
#pragma unroll
            for (int k = 0; k < kInFlight; ++k) {
                const int i = i0 + k * B;
                if (i < n) {
                    int I, x;
                    divmod_small(i, width, rcp, I, x);
                    v[k] = G[(size_t)((uint32_t)I * (uint32_t)L + (uint32_t)col(x))];
                }
            }
#pragma unroll
            for (int k = 0; k < kInFlight; ++k)
                if (i0 + k * B < n) T[i0 + k * B] = v[k];
        }
    }
    {  // position-20 blocks of the first half-sweep
        const LdsSweep sw0 = sweep_of(0);
        const float rcp = 1.0f / (float)n_groups;
        for (int f = tid; f < N * n_groups; f += B) {
            int I, k;
            divmod_small(f, n_groups, rcp, I, k);
            if (pstar + (I <= istar ? 1 : 0) == 21) u5tab[(size_t)k * N + I] = block5(sw0, rk, I, g_lo + k, 0);
        }
    }
    __syncthreads();

    const int n_hs = 2 * K;
    const int n_b = whole ? 0 : N;                  // boundary items (columns 1 and w)
    const int P = whole ? (L >> 1) : ((w - 2) >> 1);  // interior words of a colour per row
    const int n_i = N * P;
    const float rcp_P = P > 0 ? 1.0f / (float)P : 0.0f;
    const float rcp_g = 1.0f / (float)n_groups;
    const int64_t tw = a.exch_tile_words;
    const int n_w = n_b + n_i;  // word items of a half-sweep
    const lds_u64* T3 = (const lds_u64*)T;
    // word item f of a half-sweep of colour c: boundary items first (items
    // f < N/2 in column 1, the others in column w, on the rows with
    // (I + J) % 2 == c), then the interior words row by row
    auto make_item = [&](int f, int c) {
        int I, x, side = -1;
        if (f < n_b) {
            side = f >= (N >> 1) ? 1 : 0;
            x = side ? w : 1;
            I = 2 * (f - side * (N >> 1)) + ((col(x) + c) & 1);
        } else {
            int q;
            divmod_small(f - n_b, P, rcp_P, I, q);
            x = whole ? 2 * q + ((I + c) & 1) : 2 + 2 * q + ((2 + gx0 + I + c) & 1);
        }
        const int J = col(x);
        const int xl = whole && x == 0 ? L - 1 : x - 1;
        const int xr = whole && x == L - 1 ? 0 : x + 1;
        const int row = I * width;
        WordItem it;
        it.w = lds_addr(T3 + row + x);
        it.lf = lds_addr(T3 + row + xl);
        it.rt = lds_addr(T3 + row + xr);
        it.up = lds_addr(T3 + (I > 0 ? I - 1 : N - 1) * width + x);
        it.dn = lds_addr(T3 + (I < N - 1 ? I + 1 : 0) * width + x);
        // the patch word (row I* for I = 0, row 0 for I = I*); other rows
        // read row 0 and ignore it
        it.patch = lds_addr(T3 + (I == 0 ? istar : 0) * width + x);
        it.u20 = 16u * (uint32_t)(((J >> 3) - g_lo) * N + I) + 4u * (((uint32_t)J >> 1) & 3u);
        it.c1 = (uint32_t)I * (uint32_t)L + (uint32_t)J;
        it.I = I;
        it.side = side;
        it.code = 8u * (uint32_t)f;
        return it;
    };
    // With at most two word items per thread and colour (the usual tile
    // shapes), every thread's items are the same in every half-sweep of a
    // colour and are formed once, and the codes of positions 0..19 of every
    // word are drawn a half-sweep ahead into a code table (two, by the
    // half-sweep's parity, after the position-20 tables): in a half-sweep a
    // thread updates its words from the table and draws the codes of its
    // words of the other colour for the next one, while the loads of the
    // word's neighbourhood are in flight.  Otherwise every item is formed
    // and drawn in its half-sweep.
    const bool pre = n_w <= 2 * B;
    const uint32_t ctab = lds_addr((const lds_u64*)(u5tab + (size_t)2 * n_groups * N));
    WordItem cur0{}, cur1{}, oth0{}, oth1{};  // word items, this colour and the other
    auto draw_codes = [&](const WordItem& it, const LdsSweep& swc, uint32_t table) {
        // the sweep index made opaque to the compiler (see the words below)
        LdsSweep swi = swc;
        asm volatile("" : "+s"(swi.t_lo), "+s"(swi.t_hi));
        lds_store64(table + it.code, lds_word_codes(swi, rk, it.I, it.c1));
    };
    if (pre) {
        if (tid < n_w) {
            cur0 = make_item(tid, 0);
            oth0 = make_item(tid, 1);
        }
        if (tid + B < n_w) {
            cur1 = make_item(tid + B, 0);
            oth1 = make_item(tid + B, 1);
        }
        // the codes of the first half-sweep
        const LdsSweep sw0 = sweep_of(0);
        if (tid < n_w) draw_codes(cur0, sw0, ctab);
        if (tid + B < n_w) draw_codes(cur1, sw0, ctab);
        __syncthreads();
    }
    // the next half-sweep's position-20 blocks (of the rows with 21 live
    // positions) are dealt to the threads in rank order, items rank5,
    // rank5 + E5, ...  When the last round of words is partial, none go to
    // the wavefronts 0, 4, 8, ... (a workgroup's wavefronts go to the four
    // SIMDs in turn, so those share the SIMD that carries the most rounds
    // of words) and threads with fewer word items come first; otherwise the
    // threads in order (the oldest wavefronts, which the instruction arbiter
    // favours, first).  Both orders were the faster one in their case.
    const int rows21 = pstar == 20 ? istar + 1 : 0;
    const int r0 = n_w % B;  // threads below r0 have one word item more
    const bool skip0 = B >= 256 && (r0 & 255) != 0;
    auto elig_before = [&](int x) {  // eligible threads below x
        return skip0 ? x - ((x >> 8) * 64 + min(x & 255, 64)) : x;
    };
    const int E5 = elig_before(B);
    const int rank5 = !skip0                       ? tid
                      : ((tid >> 6) & 3) == 0       ? -1
                      : tid >= r0                   ? elig_before(tid) - elig_before(r0)
                                                    : E5 - elig_before(r0) + elig_before(tid);
    // the launch's next sampled sweep (a sample after sweep j iff
    // (sample_base + j + 1) % every == 0; -1 for none) and the samples taken
    // so far: counted, not divided out per half-sweep (a 64-bit division is
    // a long scalar routine)
    int64_t next_sample = a.every > 0 ? (int64_t)a.every - 1 - a.sample_base % a.every : -1;
    int n_taken = 0;
    // one half-sweep: the word items of its colour (cur0, cur1) and of the
    // other colour (oth0, oth1), whose codes it draws for the next one;
    // returns whether the launch stops
    auto half_sweep = [&](const int hs, const WordItem& cur0, const WordItem& cur1, const WordItem& oth0,
                          const WordItem& oth1) __attribute__((always_inline)) -> bool {
        const int c = hs & 1;
        const int j = hs >> 1;
        const LdsSweep sw = sweep_of(hs);
        const bool meas = c == 1 && j == next_sample;
        const uint32_t u5cur_addr = lds_addr((const lds_u64*)(u5tab + (size_t)(hs & 1) * n_groups * N));
        uint4* __restrict__ u5next = u5tab + (size_t)((hs + 1) & 1) * n_groups * N;
        const int n_u = hs + 1 < n_hs ? rows21 * n_groups : 0;
        const LdsSweep sw_next = sweep_of(hs + 1);
        // where the neighbours published the ghost words this half-sweep
        // reads: their boundary words of colour 1 - c, half-sweep hs - 1
        const uint64_t* __restrict__ gl = a.exch + (size_t)tp.left * tw + (size_t)(1 - c) * 2 * N + N;  // its right side
        const uint64_t* __restrict__ gr = a.exch + (size_t)tp.right * tw + (size_t)(1 - c) * 2 * N;      // its left side
        uint64_t* __restrict__ ex = a.exch + (size_t)blockIdx.x * tw + (size_t)c * 2 * N;
        uint32_t anti = 0, ups = 0;
        // one word item: its neighbourhood from LDS (the ghost word of a
        // boundary item straight from the neighbour's publication after the
        // launch's first half-sweep) and the word `early` gives, then
        // `between` (while the loads are in flight), the update (by `update`,
        // from the neighbourhood, the position-20 uniform and that word),
        // and the publication of a boundary word; the
        // last of the N boundary words raises the flag (every publisher waits
        // for its own store first, and the exchange words and flags are
        // device-coherent atomics, so no cache writeback or invalidation is
        // needed).  The loads of an item that does not exist (valid false)
        // read LDS at the item's default address 0 and are not used.
        auto word = [&](const WordItem& it, bool valid, auto early, auto between, auto update) {
            Nbhd nb;
            nb.w = lds_load64(it.w);
            nb.lf = lds_load64(it.lf);
            nb.rt = lds_load64(it.rt);
            nb.up = lds_load64(it.up);
            nb.dn = lds_load64(it.dn);
            nb.patch = lds_load64(it.patch);
            const uint32_t u20 = lds_load32(u5cur_addr + it.u20);
            const uint64_t e = early(it);
            if (!valid) return;
            if (it.side >= 0 && hs > 0) {
                if (it.side == 0) nb.lf = __hip_atomic_load(&gl[it.I], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                else nb.rt = __hip_atomic_load(&gr[it.I], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            between();
            const uint64_t nw = update(it, nb, u20, e);
            lds_store64(it.w, nw);
            if (it.side >= 0) {
                __hip_atomic_store(&ex[it.side * N + it.I], nw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_s_waitcnt(0);
                if (atomicAdd(&published, 1u) == (uint32_t)(hs + 1) * (uint32_t)N - 1u)
                    __hip_atomic_store(&a.flags[blockIdx.x], 2 * t0 + (uint64_t)hs + 1, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
        };
        if (pre) {
            // the words from the code table of this half-sweep; meanwhile the
            // codes of the same threads' words of the other colour for the
            // next half-sweep into the other table
            const uint32_t ccur = ctab + (uint32_t)(hs & 1) * 8u * (uint32_t)n_w;
            const uint32_t cnext = ctab + (uint32_t)((hs + 1) & 1) * 8u * (uint32_t)n_w;
            const bool draw = hs + 1 < n_hs;
            auto codes = [&](const WordItem& it) { return lds_load64(ccur + it.code); };
            auto from_table = [&](const WordItem& it, const Nbhd& nb, uint32_t u20, uint64_t cd) {
                return lds_word_apply(sw, nb, it.I, cd, u20, meas, true, anti, ups);
            };
            word(cur0, tid < n_w, codes, [&] { if (draw) draw_codes(oth0, sw_next, cnext); }, from_table);
            word(cur1, tid + B < n_w, codes, [&] { if (draw) draw_codes(oth1, sw_next, cnext); }, from_table);
        } else {
            // the words f = tid, tid + B, ..., each drawing its own codes:
            // the sweep index made opaque to the compiler, so that the
            // wave-uniform parts of the Philox rounds are formed per item on
            // the scalar unit instead of being hoisted out of the loop for
            // all five blocks (which overflows the scalar registers into
            // vector-lane spills)
            auto drawing = [&](const WordItem& it, const Nbhd& nb, uint32_t u20, uint64_t) {
                LdsSweep swi = sw;
                asm volatile("" : "+s"(swi.t_lo), "+s"(swi.t_hi));
                return lds_word_update_c1(swi, rk, nb, it.I, it.c1, u20, meas, true, anti, ups);
            };
            auto none = [](const WordItem&) { return 0ull; };
            for (int fw = tid; fw < n_w; fw += B) word(make_item(fw, c), true, none, [] {}, drawing);
        }
        // then the next half-sweep's position-20 blocks, in a loop of their
        // own so that it keeps only its own wave-uniform values live
        if (rank5 >= 0) {
            for (int b = rank5; b < n_u; b += E5) {
                int I, k;
                divmod_small(b, n_groups, rcp_g, I, k);
                u5next[(size_t)k * N + I] = block5(sw_next, rk, I, g_lo + k, c ^ 1);
            }
        }
        if (meas) {
            if (pre) {
                // at most two words per thread: a wavefront's antiparallel
                // bonds (at most 168 per thread) and up spins (84) each fit
                // in 16 bits, so one sum covers both
                const uint32_t both = wave_sum_u32((anti << 16) | ups);
                anti = both >> 16;
                ups = both & 0xFFFFu;
            } else {
                anti = wave_sum_u32(anti);
                ups = wave_sum_u32(ups);
            }
            if (lane_id() == 0) {
                red[2 * (tid >> 6)] = anti;
                red[2 * (tid >> 6) + 1] = ups;
            }
        }
        // before the next half-sweep reads them: both neighbours' boundary
        // words of this half-sweep must be published
        if (!whole && tid == 0 && hs + 1 < n_hs) {
            const uint64_t want = 2 * t0 + (uint64_t)hs + 1;
            const uint64_t start = clock_ticks();
            bool ok = true;
            // bounded twice: by the clock and by the number of polls (each
            // poll is two loads from memory and a short sleep)
            for (uint32_t polls = 0; ok; ++polls) {
                const uint64_t fl = __hip_atomic_load(&a.flags[tp.left], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t fr = __hip_atomic_load(&a.flags[tp.right], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (fl >= want && fr >= want) break;
                if (__hip_atomic_load(a.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    clock_ticks() - start > a.wait_ticks || polls > kMaxPolls) {
                    __hip_atomic_store(a.error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = false;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            if (!ok) stop = 1;
        }
        __syncthreads();
        if (meas && tid >= B - 64) {
            // the tile's sums, by the last wavefront: lane l reads
            // wavefront l's pair, one sum over the lanes for each count
            const int l = tid - (B - 64);
            const bool in = l < (B >> 6);
            const uint32_t sa = wave_sum_u32(in ? red[2 * l] : 0u), su = wave_sum_u32(in ? red[2 * l + 1] : 0u);
            if (l == 0) a.partials[(size_t)n_taken * a.n_tiles + tp.part] = {sa, su};
        }
        if (meas) {
            next_sample += a.every;
            ++n_taken;
        }
        return stop != 0;
    };
    if (pre) {
        // two half-sweeps per trip, so that the items of each colour stay in
        // the same registers (no exchange of the two sets between half-sweeps)
        for (int hs = 0; hs < n_hs; hs += 2) {
            if (half_sweep(hs, cur0, cur1, oth0, oth1)) break;
            if (half_sweep(hs + 1, oth0, oth1, cur0, cur1)) break;
        }
    } else {
        for (int hs = 0; hs < n_hs; ++hs)
            if (half_sweep(hs, cur0, cur1, oth0, oth1)) break;
    }
    // the ghost columns in LDS are stale past the first half-sweep, but the
    // band's own words are exact

    // store the band (the ghost columns belong to the neighbours)
    {
        const float rcp = 1.0f / (float)w;
        uint64_t* __restrict__ G = d.W;
        for (int i = tid; i < N * w; i += B) {
            int I, xi;
            divmod_small(i, w, rcp, I, xi);
            const int x = xi0 + xi;
            G[(size_t)((uint32_t)I * (uint32_t)L + (uint32_t)col(x))] = T[I * width + x];
        }
    }
}

size_t persist_lds_bytes(int32_t L, int32_t N, int32_t w, int32_t block) {
    // a tile of width wi: its band with the ghost columns, two position-20
    // tables (a bound on their groups) and, with at most two word items per
    // thread and colour, two code tables; the widest need of the lattice's
    // tiles (all of width w but the last)
    auto need = [&](int64_t wi) {
        const bool whole = wi >= L;
        const int64_t width = whole ? L : wi + 2;
        const int64_t groups = whole ? (L + 7) / 8 : wi / 8 + 2;
        const int64_t items = (int64_t)N * (whole ? L : wi) / 2;
        const int64_t codes = items <= 2 * (int64_t)block ? 16 * items : 0;
        return (size_t)(8 * (int64_t)N * width + 2 * 16 * groups * (int64_t)N + codes);
    };
    const int64_t wf = w >= L ? L : w;
    const int64_t last = L - ((L + wf - 1) / wf - 1) * wf;
    return std::max(need(wf), need(last));
}

size_t persist_lds_limit(int device) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, device) != hipSuccess) return 0;
    const size_t static_bytes = sizeof(uint32_t) * 2 * (kPersistMaxBlock / 64) + 256;
    return v > (int)static_bytes ? (size_t)v - static_bytes : 0;
}

hipError_t allow_persist_lds(int device) {
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_persist), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)persist_lds_limit(device));
}

hipError_t persist_capacity(int block, size_t lds_bytes, int device, int64_t* tiles) {
    int per_cu = 0, cus = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_persist),
                                                                block, lds_bytes);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    *tiles = (int64_t)per_cu * cus;
    return hipSuccess;
}

hipError_t launch_persist(const PersistLaunch& a, int32_t n_tiles, int block, size_t lds_bytes, hipStream_t s) {
    if (n_tiles <= 0 || a.K <= 0) return hipSuccess;
    if (block < 64 || block > kPersistMaxBlock || block % 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_persist, dim3(n_tiles), dim3(block), lds_bytes, s, a);
    return hipGetLastError();
}

// The completion of the last launch that holds resident tiles, per device
// (null until the first one).  Two such launches on different streams could
// each hold compute units that the other's remaining workgroups need, and
// both would then wait out their bound and fail; ordering every one after
// the device's previous one rules that out.
namespace {
std::mutex g_gate_mutex;
std::vector<hipEvent_t> g_gate;
}  // namespace

hipError_t resident_gate(int device, hipStream_t s, const std::function<hipError_t()>& launch) {
    std::lock_guard<std::mutex> lock(g_gate_mutex);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(s, &cs);
    if (e != hipSuccess) return e;
    int current = -1;
    e = hipGetDevice(&current);
    if (e != hipSuccess) return e;
    // inside a capture a dependency on work outside it is not allowed, and
    // the event belongs to the device current when it was made
    if (cs != hipStreamCaptureStatusNone || device < 0 || current != device) return launch();
    if ((size_t)device >= g_gate.size()) g_gate.resize((size_t)device + 1, nullptr);
    if (g_gate[device]) {
        e = hipStreamWaitEvent(s, g_gate[device], 0);
    } else {
        e = hipEventCreateWithFlags(&g_gate[device], hipEventDisableTiming);
    }
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    return hipEventRecord(g_gate[device], s);
}

}  // namespace ising

namespace ising {

namespace {

// E and M of sample k from the tiles' partial sums (one workgroup per
// sample): out_E[k], out_M[k].
__global__ void __launch_bounds__(256) k_samples_em(const Partial* __restrict__ partials, int32_t n_tiles, int32_t L,
                                                    int64_t* __restrict__ out_E, int64_t* __restrict__ out_M) {
    __shared__ unsigned long long red[2 * 4];
    const int k = blockIdx.x;
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
        out_E[k] = 2 * (int64_t)A - 2 * n;
        out_M[k] = 2 * (int64_t)U - n;
    }
}

// Moment sums of n samples added to *mom, by one wavefront: per-lane sums
// of samples l, l + 64, ..., merged exactly.
__global__ void __launch_bounds__(64) k_samples_moments(const int64_t* __restrict__ E, const int64_t* __restrict__ M,
                                                        int32_t n, Moments* mom) {
    Moments part = {};
    for (int k = lane_id(); k < n; k += 64) add_sample(part, E[k], M[k]);
    wave_merge_moments(part);
    if (lane_id() == 0) {
        Moments m = *mom;
        merge_moments(m, part);
        *mom = m;
    }
}

}  // namespace

namespace {

// The samples of one launch of resident tiles for every tiled lattice of a
// batch, one wavefront per listed lattice: lane l takes samples l, l + 64,
// ... (the sum of the lattice's tile partials), writes their E, M to the
// series and adds them to its own moment sums; the lanes' sums are then
// merged exactly, and lane 0 adds them to the lattice's with the last E, M.
__global__ void __launch_bounds__(64) k_finalize_resident(const LatticeDesc* __restrict__ descs,
                                                          LatticeState* __restrict__ states,
                                                          const int32_t* __restrict__ ids,
                                                          const Partial* __restrict__ partials, int32_t n_tiles,
                                                          int32_t n_samples) {
    const int32_t lat = ids[blockIdx.x];
    const LatticeDesc& d = descs[lat];
    LatticeState& st = states[lat];
    const int n = min(n_samples, d.sweep_limit);  // a lattice past its limit took fewer samples
    if (n <= 0) return;
    const int64_t spins = (int64_t)d.L * (int64_t)d.L;
    const int64_t idx = st.series_idx;
    Moments part = {};
    int64_t E = 0, M = 0;
    for (int o = lane_id(); o < n; o += 64) {
        unsigned long long anti = 0, ups = 0;
        const Partial* __restrict__ p = partials + (size_t)o * n_tiles + d.part_begin;
        for (int i = 0; i < d.part_count; ++i) {
            anti += p[i].anti;
            ups += p[i].ups;
        }
        E = 2 * (int64_t)anti - 2 * spins;
        M = 2 * (int64_t)ups - spins;
        if (d.series_E) d.series_E[idx + o] = E;
        if (d.series_M) d.series_M[idx + o] = M;
        add_sample(part, E, M);
    }
    wave_merge_moments(part);
    // the lane that took the last sample holds its E, M
    const int last = (n - 1) & 63;
    const int64_t lE = __shfl(E, last, 64), lM = __shfl(M, last, 64);
    if (lane_id() == 0) {
        Moments m = st.mom;
        merge_moments(m, part);
        st.mom = m;
        st.last_E = lE;
        st.last_M = lM;
        st.series_idx = idx + n;
    }
}

}  // namespace

hipError_t launch_finalize_resident(const LatticeDesc* descs, LatticeState* states, const int32_t* ids,
                                    int32_t n_lat, const Partial* partials, int32_t n_tiles, int32_t n_samples,
                                    hipStream_t s) {
    if (n_lat <= 0 || n_samples <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_resident, dim3(n_lat), dim3(64), 0, s, descs, states, ids, partials, n_tiles,
                       n_samples);
    return hipGetLastError();
}

hipError_t launch_samples(const Partial* partials, int32_t n_tiles, int32_t n_samples, int32_t L, int64_t* out_E,
                          int64_t* out_M, Moments* mom, hipStream_t s) {
    if (n_samples <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_samples_em, dim3(n_samples), dim3(256), 0, s, partials, n_tiles, L, out_E, out_M);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !mom) return e;
    hipLaunchKernelGGL(k_samples_moments, dim3(1), dim3(64), 0, s, out_E, out_M, n_samples, mom);
    return hipGetLastError();
}

}  // namespace ising
