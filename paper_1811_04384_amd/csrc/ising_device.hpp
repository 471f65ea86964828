// Device-side building blocks of the multi-spin-coded checkerboard Metropolis
// sweep for gfx950: Philox4x32-10 draws, neighbour-word assembly with the
// periodic wrap between the first and last word rows, bit-sliced neighbour
// counting and acceptance, and wavefront reductions.
//
// Word layout (paper Section 3, Fig. 1): W[I][J] (uint64) holds the spins of
// rows I, I+N, ..., I+20N of column J; position p (row I + pN) occupies the
// 3-bit field ("slot") k = 20 - p, i.e. bits 3k..3k+2, and only bit 3k is
// ever set ("001" = up, "000" = down).  Bit 63 is always 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_common.hpp"

namespace ising {

// Bit 3k of every field, k = 0..20.
constexpr uint64_t kSpinBits = 0x1249249249249249ull;
constexpr uint64_t kLow63 = 0x7FFFFFFFFFFFFFFFull;

constexpr uint32_t kPhiloxM0 = 0xD2511F53u;  // multiplies counter word 0
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;  // multiplies counter word 2
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;  // key increment, word 0
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;  // key increment, word 1

struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    // gfx950 three-input bitwise op; truth table 0x96 = a ^ b ^ c
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon et al., SC'11) for the counter shape used by every
// draw of this library: words 0, 2, 3 of the counter and the key are the same
// for all lanes of a wavefront, only word 1 differs.  Rounds 1-3 are written
// with plain XORs so the compiler keeps their wave-uniform parts on the
// scalar unit (round 1 is entirely scalar, rounds 2 and 3 need one 64-bit
// product each); rounds 4-10 use the three-input XOR.
__device__ __forceinline__ U4 philox_lane_c1(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kPhiloxM0 * c0;
        const uint64_t pb = (uint64_t)kPhiloxM1 * c2;
        uint32_t n0, n2;
        if (r < 3) {
            n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        } else {
            n0 = xor3((uint32_t)(pb >> 32), c1, k0);
            n2 = xor3((uint32_t)(pa >> 32), c3, k1);
        }
        c1 = (uint32_t)pb;
        c3 = (uint32_t)pa;
        c0 = n0;
        c2 = n2;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
    return {c0, c1, c2, c3};
}

// Live-spin mask of word row I: positions p with I + pN < L.
__device__ __forceinline__ uint64_t live_mask(int I, int L, int N) {
    const int n_live = min(21, (L - 1 - I) / N + 1);
    return kSpinBits & (~0ull << (3 * (21 - n_live)));
}

// Up neighbour word of word (I, J): row I-1, or for I = 0 the last word row
// shifted one field down (position p takes position p-1 of row N-1) with
// position 0 taken from the word holding row L-1 (row I*, slot sh_star/3).
template <class Load>
__device__ __forceinline__ uint64_t up_word(const Load& ld, int I, int J, int N, int istar, int sh_star) {
    if (I > 0) return ld(I - 1, J);
    const uint64_t last = ld(N - 1, J);
    const uint64_t wrap = ld(istar, J);
    return (last >> 3) | (((wrap >> sh_star) & 1ull) << 60);
}

// Down neighbour word of word (I, J): row I+1, or for I = N-1 the first word
// row shifted one field up (position p takes position p+1 of row 0); in word
// row I* the slot of row L-1 takes row 0 (position 0 of word row 0).
template <class Load>
__device__ __forceinline__ uint64_t down_word(const Load& ld, int I, int J, int N, int istar, int sh_star) {
    uint64_t d = (I < N - 1) ? ld(I + 1, J) : ((ld(0, J) << 3) & kLow63);
    if (I == istar) {
        const uint64_t first = ld(0, J);
        d = (d & ~(1ull << sh_star)) | (((first >> 60) & 1ull) << sh_star);
    }
    return d;
}

// Acceptance bits of one position: 1 if u < t4, 3 if u < t8 (t8 <= t4, so
// u < t8 implies u < t4), else 0.  Field bit 0 says "accepted if dE = +4",
// bit 1 says "accepted if dE = +8".
__device__ __forceinline__ uint32_t accept_code(uint32_t u, uint32_t t4, uint32_t t8) {
    uint32_t x = (u < t4) ? 1u : 0u;
    return (u < t8) ? 3u : x;
}

// The 21 per-position acceptance codes of one word packed in word layout
// (code of position p in field 20 - p), built from the six Philox blocks:
// block g < 5 serves positions 4g..4g+3, block 5 serves position 20 (taken
// from output q5 of a block shared by four same-colour words).
struct Codes {
    uint32_t hi;  // fields 11..20 -> word bits 33..62 (stored as bits 1..30)
    uint32_t mid; // field 10     -> word bits 30..32
    uint32_t lo;  // fields 0..9  -> word bits 0..29
};

// Flip mask of a word.  a..d = w XOR neighbour (only bit 3k meaningful);
// n = number of set inputs per field.  A spin flips iff n >= 2 (dE <= 0), or
// n = 1 and u < t4 (dE = +4), or n = 0 and u < t8 (dE = +8) (Table 1 and the
// Metropolis rule of Section 2).  With the code bits c0 (u < t4) and
// c1 (u < t8, which implies c0): flip = c1 | (c0 & n>=1) | n>=2.
__device__ __forceinline__ uint64_t flip_mask(uint64_t w, uint64_t up, uint64_t dn, uint64_t lf, uint64_t rt,
                                              uint64_t codes, uint64_t live) {
    const uint64_t a = w ^ up, b = w ^ dn, c = w ^ lf, d = w ^ rt;
    const uint64_t ab_or = a | b, cd_or = c | d;
    const uint64_t ge1 = ab_or | cd_or;
    const uint64_t ge2 = (a & b) | (c & d) | (ab_or & cd_or);
    return ((codes >> 1) | (codes & ge1) | ge2) & live;
}

__device__ __forceinline__ uint64_t assemble_codes(const Codes& c) {
    return ((uint64_t)c.hi << 33) | ((uint64_t)c.mid << 30) | (uint64_t)c.lo;
}

// Antiparallel bonds (4 per live spin) of an updated colour-1 word and the up
// spins of it and of its left neighbour (colour 0): summed over all colour-1
// words this counts every bond of the lattice once and every spin once.
__device__ __forceinline__ void measure_word(uint64_t w, uint64_t up, uint64_t dn, uint64_t lf, uint64_t rt,
                                             uint64_t live, uint32_t& anti, uint32_t& ups) {
    anti += __popcll((w ^ up) & live) + __popcll((w ^ dn) & live) + __popcll((w ^ lf) & live) +
            __popcll((w ^ rt) & live);
    ups += __popcll(w & live) + __popcll(lf & live);
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Update the WPT same-colour words (I, J0 + 2k), k < WPT, of one row segment.
// `ld(I, J)` / `st(I, J, v)` access the word lattice (global memory or LDS).
// J0 = base + parity; words with J >= L do not exist (ragged last segment).
// The draws of position 20 come from block 5 keyed by word column
// 8*(J div 8) + (J mod 2) and output (J div 2) mod 4; one block per thread
// serves all of its words.
template <int WPT, bool MEASURE, class Load, class Store>
__device__ __forceinline__ void update_segment(const Load& ld, const Store& st, int I, int J0, const SweepArgs& a,
                                               uint32_t& anti, uint32_t& ups) {
    const int L = a.L, N = a.N;
    const uint64_t live = live_mask(I, L, N);
    const int n_live = min(21, (L - 1 - I) / N + 1);
    const uint32_t row_base = (uint32_t)I * (uint32_t)L;

    uint64_t w[WPT], up[WPT], dn[WPT], lf[WPT], rt[WPT];
    bool ok[WPT];
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        const int J = J0 + 2 * k;
        ok[k] = J < L;
        const int Jc = ok[k] ? J : J0;  // keep loads in bounds for the ragged tail
        w[k] = ld(I, Jc);
        lf[k] = ld(I, Jc == 0 ? L - 1 : Jc - 1);
        rt[k] = ld(I, Jc == L - 1 ? 0 : Jc + 1);
        up[k] = up_word(ld, I, Jc, N, a.istar, a.sh_star);
        dn[k] = down_word(ld, I, Jc, N, a.istar, a.sh_star);
    }

    Codes codes[WPT];
#pragma unroll
    for (int k = 0; k < WPT; ++k) codes[k] = {0u, 0u, 0u};

    // blocks g = 0..4: positions 4g..4g+3 of each word
#pragma unroll
    for (int g = 0; g < 5; ++g) {
        if (4 * g >= n_live) break;  // every position of the block is a dead slot
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const uint32_t col = (uint32_t)min(J0 + 2 * k, L - 1);
            const U4 r = philox_lane_c1(a.t_lo, row_base + col, a.t_hi, (uint32_t)g | (1u << 3), a.k0, a.k1);
            const uint32_t u[4] = {r.x, r.y, r.z, r.w};
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int p = 4 * g + j;  // position; field 20 - p
                const int field = 20 - p;
                const uint32_t cde = accept_code(u[j], a.t4, a.t8);
                if (field >= 11) codes[k].hi |= cde << (3 * field - 33);
                else if (field == 10) codes[k].mid = cde;
                else codes[k].lo |= cde << (3 * field);
            }
        }
    }
    // block 5: position 20 (field 0).  The words J0 + 2k of one thread lie in
    // one aligned group of eight columns (2 WPT divides 8), so one block keyed
    // by that group's same-colour base column serves all of them, word k
    // taking output (J0 div 2 + k) mod 4.
    if (n_live == 21) {
        const uint32_t col = ((uint32_t)J0 & ~7u) | ((uint32_t)J0 & 1u);
        const U4 r = philox_lane_c1(a.t_lo, row_base + col, a.t_hi, 5u | (1u << 3), a.k0, a.k1);
        const uint32_t q0 = ((uint32_t)J0 >> 1) & 3u;
#pragma unroll
        for (int k = 0; k < WPT; ++k) {
            const uint32_t q = (q0 + (uint32_t)k) & 3u;
            const uint32_t u = WPT == 4 ? (k == 0 ? r.x : k == 1 ? r.y : k == 2 ? r.z : r.w)
                                        : (q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w);
            codes[k].lo |= accept_code(u, a.t4, a.t8);
        }
    }

#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        if (!ok[k]) continue;
        const uint64_t f = flip_mask(w[k], up[k], dn[k], lf[k], rt[k], assemble_codes(codes[k]), live);
        const uint64_t nw = w[k] ^ f;
        st(I, J0 + 2 * k, nw);
        if (MEASURE) measure_word(nw, up[k], dn[k], lf[k], rt[k], live, anti, ups);
    }
}

}  // namespace ising
