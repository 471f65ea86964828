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

// Apply the drawn picks of a phase.  A workgroup (one wavefront) holds
// `chains` strips (1, 2 or 4) in LDS and gives each G = 64 / chains lanes.
// A strip's picks are applied in windows of G picks in pick order: first the
// picks deferred by the previous step, then the next fresh ones.  A pick of
// the window conflicts with an earlier pick of the window iff the earlier
// pick's word is its own word or one it reads (left, right, up, down, the
// wrap-row patch word); this relation is symmetric (each of these neighbour
// relations has its mirror).  Every pick without such a conflict is applied
// now, the others are deferred, in order: a pick applied now commutes with
// every earlier deferred one (neither reads the other's word), and the
// picks applied together read no word another of them writes, while every
// lane of a step loads before any lane stores, so the state is exactly that
// of applying the picks one by one.  The first pick of a window never
// conflicts, so every step applies at least one.  Conflicts are found
// through a claim per word: each lane takes the minimum of its index and the
// claim of its word, then a lane conflicts iff a word it reads carries a
// smaller index.
//
// LDS per strip q: words [q][cc][I] (cc = 0: the frozen column left of the
// phase columns, 1..width: the phase columns, width + 1: the frozen column
// right of them), claims of the same words, the pick data of the current
// block of kStripBlock picks and the deferred picks; then the live-slot mask
// of every word row.
constexpr int kStripBlock = 256;

__global__ void __launch_bounds__(64) k_strip_apply(uint64_t* __restrict__ W, StripArgs a, int chains,
                                                    uint32_t n_k, const uint32_t* __restrict__ pos,
                                                    const uint64_t* __restrict__ codes) {
    extern __shared__ uint64_t strip_lds[];
    const int lane = (int)threadIdx.x;
    const int p0 = (int)blockIdx.x * chains;
    const int n_chains = min(chains, a.strips - p0);
    const int L = a.L, N = a.N, width = a.width, cols = width + 2;
    const int chain_words = cols * N;
    uint64_t* __restrict__ words = strip_lds;
    uint64_t* __restrict__ live_row = words + (size_t)chains * chain_words;
    uint64_t* __restrict__ blk_codes = live_row + N;
    uint32_t* __restrict__ claims = reinterpret_cast<uint32_t*>(blk_codes + (size_t)chains * kStripBlock);
    uint32_t* __restrict__ blk_pos = claims + (size_t)chains * chain_words;
    uint32_t* __restrict__ deferred = blk_pos + (size_t)chains * kStripBlock;  // 64 entries, G per strip

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
                words[(size_t)q * chain_words + (size_t)cc * N + I] = v[u];
            }
        }
    }
    for (int I = lane; I < N; I += 64) live_row[I] = live_mask(I, L, N);
    for (int e = lane; e < chains * chain_words; e += 64) claims[e] = 0xFFFFFFFFu;

    // lanes of a strip: group q = lane / G, index i = lane % G
    const int G = 64 / chains;
    const int q = lane / G;
    const int i = lane - q * G;
    const bool has_chain = q < n_chains;
    uint64_t* __restrict__ my = words + (size_t)q * chain_words;
    uint32_t* __restrict__ my_claim = claims + (size_t)q * chain_words;
    const int istar = a.istar, sh_star = a.sh_star;
    const size_t stride = (size_t)a.strips;

    // pick data of a block: entry e = (chain qq, pick j) with j fastest;
    // held in registers while the previous block is applied
    constexpr int kPer = kStripBlock * 4 / 64;  // entries per lane for up to 4 chains
    const int n_entries = chains * kStripBlock;
    uint32_t rq[kPer];
    uint64_t rd[kPer];
    auto fetch = [&](uint32_t b0) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = lane + 64 * u;
            const int qq = e / kStripBlock, j = e - (e / kStripBlock) * kStripBlock;
            const uint32_t k = min(b0 + (uint32_t)j, n_k - 1);
            const bool ok = e < n_entries && qq < n_chains;
            const size_t idx = (size_t)k * stride + (size_t)(p0 + (ok ? qq : 0));
            rq[u] = ok ? pos[idx] : 0u;
            rd[u] = ok ? codes[idx] : 0ull;
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = lane + 64 * u;
            if (e < n_entries) {
                blk_pos[e] = rq[u];
                blk_codes[e] = rd[u];
            }
        }
    };
    fetch(0u);
    __syncthreads();

    for (uint32_t b0 = 0; b0 < n_k; b0 += kStripBlock) {
        stash();
        fetch(b0 + kStripBlock);  // in flight while this block is applied
        __syncthreads();
        const uint32_t bend = min(b0 + (uint32_t)kStripBlock, n_k);
        uint32_t kk = b0;     // next fresh pick of this strip (same in all its lanes)
        uint32_t n_def = 0;   // picks of this strip deferred by the previous step
        const uint64_t gbits = (G == 64) ? ~0ull : (((1ull << G) - 1ull) << (q * G));
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));  // lanes before this one
        while (true) {
            const bool pending = has_chain && (n_def > 0u || kk < bend);
            if (__ballot(pending) == 0ull) break;  // every strip of the workgroup is through the block
            uint32_t k;
            bool act;
            if ((uint32_t)i < n_def) {
                k = deferred[q * G + i];
                act = true;
            } else {
                k = kk + ((uint32_t)i - n_def);
                act = has_chain && k < bend;
            }
            int w = 0, lf = 0, rt = 0, up = 0, dn = 0, patch = 0, I = 0;
            uint64_t cd = 0;
            if (act) {
                const uint32_t pk = blk_pos[q * kStripBlock + (int)(k - b0)];
                cd = blk_codes[q * kStripBlock + (int)(k - b0)];
                I = (int)(pk >> kStripColBits);
                const int base = ((int)(pk & ((1u << kStripColBits) - 1u)) + 1) * N;
                w = base + I;
                lf = w - N;
                rt = w + N;
                up = base + (I > 0 ? I - 1 : N - 1);
                dn = base + (I < N - 1 ? I + 1 : 0);
                // the patch word of the wrap rows (row I* for I = 0, row 0
                // for I = I*); other rows read their own word again
                patch = I == 0 ? base + istar : (I == istar ? base : w);
                atomicMin(&my_claim[w], (uint32_t)i);
            }
            bool conflict = false;
            uint64_t vw = 0, vlf = 0, vrt = 0, vup = 0, vdn = 0, vpatch = 0, vlive = 0;
            if (act) {
                // all twelve loads in flight together: the claims combined
                // without short-circuit, which would make six dependent round
                // trips of them
                const uint32_t ui = (uint32_t)i;
                const uint32_t c_w = my_claim[w], c_lf = my_claim[lf], c_rt = my_claim[rt], c_up = my_claim[up],
                               c_dn = my_claim[dn], c_pa = my_claim[patch];
                conflict = (c_w < ui) | (c_lf < ui) | (c_rt < ui) | (c_up < ui) | (c_dn < ui) | (c_pa < ui);
                vw = my[w];
                vlf = my[lf];
                vrt = my[rt];
                vup = my[up];
                vdn = my[dn];
                vpatch = my[patch];
                vlive = live_row[I];
            }
            if (act && !conflict) {
                uint64_t vu = vup, vd = vdn;
                if (I == 0) vu = (vu >> 3) | (((vpatch >> sh_star) & 1ull) << 60);
                if (I == N - 1) vd = (vd << 3) & kLow63;
                if (I == istar) vd = (vd & ~(1ull << sh_star)) | (((vpatch >> 60) & 1ull) << sh_star);
                my[w] = vw ^ flip_mask(vw, vu, vd, vlf, vrt, cd, vlive);
            }
            if (act) my_claim[w] = 0xFFFFFFFFu;
            // the conflicting picks, in order, head the next window
            const uint64_t cmask = __ballot(act && conflict) & gbits;
            const uint64_t amask = __ballot(act) & gbits;
            if (act && conflict) deferred[q * G + __builtin_popcountll(cmask & below)] = k;
            kk += (uint32_t)__builtin_popcountll(amask) - n_def;  // fresh picks taken into this window
            n_def = (uint32_t)__builtin_popcountll(cmask);
        }
        __syncthreads();
    }

    __syncthreads();
    // cooperative write-back of the phase columns (LDS columns 1..width)
    const int per_row_w = n_chains * width;
    const int n_back = per_row_w * N;
    for (int e = lane; e < n_back; e += 64) {
        const int I = e / per_row_w;
        const int rem = e - I * per_row_w;
        const int qq = rem / width;
        const int cc = rem - qq * width + 1;
        const int J = (p0 + qq) * a.S + a.off + cc - 1;
        W[(size_t)I * (size_t)L + (size_t)J] = words[(size_t)qq * chain_words + (size_t)cc * N + I];
    }
}

inline unsigned strip_grid(uint64_t n, int block) { return (unsigned)((n + block - 1) / block); }

}  // namespace

size_t strip_apply_lds_bytes(const StripArgs& a, int chains) {
    const size_t words = (size_t)chains * (size_t)(a.width + 2) * (size_t)a.N;
    return words * (sizeof(uint64_t) + sizeof(uint32_t)) + (size_t)a.N * sizeof(uint64_t) +
           (size_t)chains * kStripBlock * (sizeof(uint64_t) + sizeof(uint32_t)) + 64 * sizeof(uint32_t);
}

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
    int chains = 2;  // two strips of 32 lanes per wavefront (measured best of 1, 2, 4)
    while (chains > 1 && strip_apply_lds_bytes(a, chains) > kStripLdsBytes) chains /= 2;
    const size_t lds = strip_apply_lds_bytes(a, chains);
    if (lds > kStripLdsBytes) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_strip_apply, dim3(strip_grid((uint64_t)a.strips, chains)), dim3(64), lds, s, W, a, chains,
                       n_k, pos, codes);
    return hipGetLastError();
}

}  // namespace ising
