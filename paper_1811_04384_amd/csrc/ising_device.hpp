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

// A vector-register copy of a wave-uniform value.  On gfx950, simple 32-bit
// vector instructions (add, xor, three-input bitwise) that read a scalar
// register take about 4.4 cycles per wave64 instruction when they follow
// each other, against about 2.6 when all operands are vector registers or
// constants (the instruction-rate microbenchmark, valu_rates.hip); the
// Philox rounds therefore read their round keys from vector registers.
__device__ __forceinline__ uint32_t in_vgpr(uint32_t s) {
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// Philox4x32-10 (Salmon et al., SC'11) for the counter shape used by every
// draw of this library: words 0, 2, 3 of the counter and the key are the same
// for all lanes of a wavefront, only word 1 differs.  Rounds 1-3 are written
// with plain XORs so the compiler keeps their wave-uniform parts on the
// scalar unit (round 1 is entirely scalar, rounds 2 and 3 need one 64-bit
// product each); rounds 4-10 use the three-input XOR.  With RK, the round
// keys that the three-input XORs of rounds 4-10 read come from vector
// registers (RoundKeys, computed once per thread).
struct RoundKeys {
    uint32_t k0[7], k1[7];  // keys of rounds 4..10
};

__device__ __forceinline__ RoundKeys round_keys(uint32_t k0, uint32_t k1) {
    RoundKeys rk;
#pragma unroll
    for (int r = 3; r < 10; ++r) {
        rk.k0[r - 3] = in_vgpr(k0 + (uint32_t)r * kPhiloxW0);
        rk.k1[r - 3] = in_vgpr(k1 + (uint32_t)r * kPhiloxW1);
    }
    return rk;
}

template <bool RK>
__device__ __forceinline__ U4 philox_rounds(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1, const RoundKeys* rk) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)kPhiloxM0 * c0;
        const uint64_t pb = (uint64_t)kPhiloxM1 * c2;
        uint32_t n0, n2;
        if (r < 3) {
            n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
            n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        } else if (r == 3) {  // word 3 is still wave-uniform: c3 ^ k1 on the scalar unit
            n0 = xor3((uint32_t)(pb >> 32), c1, RK ? rk->k0[0] : k0);
            n2 = (uint32_t)(pa >> 32) ^ (c3 ^ k1);
        } else {
            n0 = xor3((uint32_t)(pb >> 32), c1, RK ? rk->k0[r - 3] : k0);
            n2 = xor3((uint32_t)(pa >> 32), c3, RK ? rk->k1[r - 3] : k1);
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

__device__ __forceinline__ U4 philox_lane_c1(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1) {
    return philox_rounds<false>(c0, c1, c2, c3, k0, k1, nullptr);
}

// The same block with the keys of rounds 4-10 taken from rk (which must hold
// round_keys(k0, k1)).
__device__ __forceinline__ U4 philox_lane_c1(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                             uint32_t k1, const RoundKeys& rk) {
    return philox_rounds<true>(c0, c1, c2, c3, k0, k1, &rk);
}

// Live-spin mask of word row I: positions p with I + pN < L.
__device__ __forceinline__ uint64_t live_mask(int I, int L, int N) {
    const int n_live = min(21, (L - 1 - I) / N + 1);
    return kSpinBits & (~0ull << (3 * (21 - n_live)));
}

// The raw neighbourhood of word (I, J), loaded before any arithmetic needs it
// so that the random numbers are drawn while the loads are in flight:
// the word, its left and right words (columns wrap), the words above and
// below (rows wrap: row N-1 above row 0, row 0 below row N-1), and the
// patch word of the two wrap rows (row I* for I = 0, row 0 for I = I*;
// I* = (L-1) mod N is odd, so never 0).  fix_up / fix_down finish the
// vertical neighbours.
struct Nbhd {
    uint64_t w, lf, rt, up, dn, patch;
};

template <class Load>
__device__ __forceinline__ Nbhd load_nbhd(const Load& ld, int I, int J, int L, int N, int istar) {
    Nbhd n;
    n.w = ld(I, J);
    n.lf = ld(I, J == 0 ? L - 1 : J - 1);
    n.rt = ld(I, J == L - 1 ? 0 : J + 1);
    n.up = ld(I > 0 ? I - 1 : N - 1, J);
    n.dn = ld(I < N - 1 ? I + 1 : 0, J);
    n.patch = (I == 0) ? ld(istar, J) : (I == istar) ? ld(0, J) : 0ull;
    return n;
}

// Up neighbour word: row I-1, or for I = 0 the last word row shifted one
// field down (position p takes position p-1 of row N-1) with position 0
// taken from the word holding row L-1 (row I*, slot sh_star/3).
__device__ __forceinline__ uint64_t fix_up(const Nbhd& n, int I, int sh_star) {
    if (I > 0) return n.up;
    return (n.up >> 3) | (((n.patch >> sh_star) & 1ull) << 60);
}

// Down neighbour word: row I+1, or for I = N-1 the first word row shifted
// one field up (position p takes position p+1 of row 0); in word row I* the
// slot of row L-1 takes row 0 (position 0 of word row 0).
__device__ __forceinline__ uint64_t fix_down(const Nbhd& n, int I, int N, int istar, int sh_star) {
    uint64_t d = (I < N - 1) ? n.dn : ((n.dn << 3) & kLow63);
    if (I == istar) d = (d & ~(1ull << sh_star)) | (((n.patch >> 60) & 1ull) << sh_star);
    return d;
}

// The same vertical neighbours loaded and finished in one step, for code
// that visits a word at a time (strips, observables).
template <class Load>
__device__ __forceinline__ uint64_t up_word(const Load& ld, int I, int J, int N, int istar, int sh_star) {
    if (I > 0) return ld(I - 1, J);
    const uint64_t last = ld(N - 1, J);
    const uint64_t wrap = ld(istar, J);
    return (last >> 3) | (((wrap >> sh_star) & 1ull) << 60);
}

template <class Load>
__device__ __forceinline__ uint64_t down_word(const Load& ld, int I, int J, int N, int istar, int sh_star) {
    uint64_t d = (I < N - 1) ? ld(I + 1, J) : ((ld(0, J) << 3) & kLow63);
    if (I == istar) {
        const uint64_t first = ld(0, J);
        d = (d & ~(1ull << sh_star)) | (((first >> 60) & 1ull) << sh_star);
    }
    return d;
}

// Acceptance code of one position: the number of thresholds above its
// uniform, (u < t4) + (u < t8) in {0, 1, 2} (t8 <= t4, so u < t8 implies
// u < t4).  A move with dE = +4 is accepted iff the code is >= 1, one with
// dE = +8 iff it is 2 (Section 2, step 3 with the energies of Table 1).
__device__ __forceinline__ uint32_t accept_code(uint32_t u, uint32_t t4, uint32_t t8) {
    const uint32_t x = (u < t4) ? 1u : 0u;
    return (u < t8) ? 2u : x;
}

// The 21 per-position acceptance codes of one word packed in word layout
// (code of position p in field 20 - p).  They are appended in position order
// with acc = (acc << 3) | code, so every code is a small inline constant.
struct Codes {
    uint32_t hi;  // positions 0..9  = fields 20..11 -> word bits 33..62 (bits 0..29 here)
    uint32_t mid; // position 10     = field 10     -> word bits 30..31
    uint32_t lo;  // positions 11..20 = fields 9..0  -> word bits 0..29
};

__device__ __forceinline__ void append_code(Codes& c, int p, uint32_t code) {
    if (p < 10) c.hi = (c.hi << 3) | code;
    else if (p == 10) c.mid = code;
    else c.lo = (c.lo << 3) | code;
}

// acc = (acc << 3) | accept_code(u), as five VALU instructions: two compares
// into lane masks, two selects of inline constants, one shift-or.  Written
// out because the compiler otherwise folds the shift into selects of
// pre-shifted literals, which need extra moves on this target.  The s_nop
// gives the lane masks the wait states a VALU read of a VALU-written SGPR
// needs.  ALU instructions only (no memory access).
__device__ __forceinline__ uint32_t append_accept(uint32_t acc, uint32_t u, uint32_t t4, uint32_t t8) {
    uint32_t x;
    uint64_t m4, m8;
    asm("v_cmp_gt_u32_e64 %[m4], %[t4], %[u]\n\t"
        "v_cmp_gt_u32_e64 %[m8], %[t8], %[u]\n\t"
        "s_nop 1\n\t"
        "v_cndmask_b32_e64 %[x], 0, 1, %[m4]\n\t"
        "v_cndmask_b32_e64 %[x], %[x], 2, %[m8]\n\t"
        "v_lshl_or_b32 %[acc], %[acc], 3, %[x]"
        : [acc] "+v"(acc), [x] "=&v"(x), [m4] "=&s"(m4), [m8] "=&s"(m8)
        : [u] "v"(u), [t4] "s"(t4), [t8] "s"(t8));
    return acc;
}

// accept_code(u) as four VALU instructions (the first code of an
// accumulator needs no shift-or).
__device__ __forceinline__ uint32_t first_accept(uint32_t u, uint32_t t4, uint32_t t8) {
    uint32_t x;
    uint64_t m4, m8;
    asm("v_cmp_gt_u32_e64 %[m4], %[t4], %[u]\n\t"
        "v_cmp_gt_u32_e64 %[m8], %[t8], %[u]\n\t"
        "s_nop 1\n\t"
        "v_cndmask_b32_e64 %[x], 0, 1, %[m4]\n\t"
        "v_cndmask_b32_e64 %[x], %[x], 2, %[m8]"
        : [x] "=&v"(x), [m4] "=&s"(m4), [m8] "=&s"(m8)
        : [u] "v"(u), [t4] "s"(t4), [t8] "s"(t8));
    return x;
}

__device__ __forceinline__ void append_draw(Codes& c, int p, uint32_t u, uint32_t t4, uint32_t t8) {
    if (p == 0) c.hi = first_accept(u, t4, t8);
    else if (p < 10) c.hi = append_accept(c.hi, u, t4, t8);
    else if (p == 10) c.mid = first_accept(u, t4, t8);
    else if (p == 11) c.lo = first_accept(u, t4, t8);
    else c.lo = append_accept(c.lo, u, t4, t8);
}

// Three-input bitwise operation with truth table TT (operand bits x, y, z
// index bit 4x + 2y + z of TT).
template <int TT>
__device__ __forceinline__ uint32_t lop3(uint32_t x, uint32_t y, uint32_t z) {
    return __builtin_amdgcn_bitop3_b32(x, y, z, TT);
}

// One 32-bit half of the flip mask.  A spin flips iff n >= 2 antiparallel
// neighbours (dE <= 0), or n = 1 and code >= 1 (dE = +4), or n = 0 and
// code = 2 (dE = +8) (Table 1 and the Metropolis rule of Section 2).  With
// t = [differs from up or down], p = [differs from both] and t', p' the
// same for left and right: n >= 1 is t | t', n >= 2 is p | p' | (t & t').
// With code bits c0 = [code = 1], c1 = [code = 2]:
// flip = c1 | ((c0 | c1) & n>=1) | n>=2.
__device__ __forceinline__ uint32_t flip_half(uint32_t w, uint32_t up, uint32_t dn, uint32_t lf, uint32_t rt,
                                              uint32_t c0, uint32_t c1, uint32_t live) {
    const uint32_t t1 = lop3<0x7E>(w, up, dn);  // (w ^ up) | (w ^ dn)
    const uint32_t p1 = lop3<0x18>(w, up, dn);  // (w ^ up) & (w ^ dn)
    const uint32_t t2 = lop3<0x7E>(w, lf, rt);
    const uint32_t p2 = lop3<0x18>(w, lf, rt);
    const uint32_t ge1 = t1 | t2;
    const uint32_t ge2 = lop3<0xFE>(p1, p2, t1 & t2);  // or of the three
    const uint32_t x = lop3<0xA8>(c0, c1, ge1);         // (c0 | c1) & ge1
    return lop3<0xFE>(c1, x, ge2) & live;
}

// Flip mask of a word (only bit 3k of each field is meaningful).
__device__ __forceinline__ uint64_t flip_mask(uint64_t w, uint64_t up, uint64_t dn, uint64_t lf, uint64_t rt,
                                              uint64_t codes, uint64_t live) {
    const uint64_t c1 = codes >> 1;
    const uint32_t lo = flip_half((uint32_t)w, (uint32_t)up, (uint32_t)dn, (uint32_t)lf, (uint32_t)rt, (uint32_t)codes,
                                  (uint32_t)c1, (uint32_t)live);
    const uint32_t hi = flip_half((uint32_t)(w >> 32), (uint32_t)(up >> 32), (uint32_t)(dn >> 32), (uint32_t)(lf >> 32),
                                  (uint32_t)(rt >> 32), (uint32_t)(codes >> 32), (uint32_t)(c1 >> 32),
                                  (uint32_t)(live >> 32));
    return ((uint64_t)hi << 32) | lo;
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

// Sums over the 64 lanes of a wavefront, returned to every lane; every lane
// must be active.  Data-parallel-primitive moves inside the vector unit, no
// LDS: within each row of 16 lanes, add the neighbour (quad_perm [1,0,3,2]),
// the neighbouring pair ([2,3,0,1]), the mirror within 8 and the mirror
// within 16, so that every lane holds its row's sum; then rows 1 and 3 add
// lane 15 of the row before (row_bcast:15), rows 2 and 3 add lane 31
// (row_bcast:31), and lane 63 holds the total.  Lanes of a row that a step
// leaves out add 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
    return ((unsigned long long)dpp_u32<CTRL, ROWS>((uint32_t)(v >> 32)) << 32) | dpp_u32<CTRL, ROWS>((uint32_t)v);
}

template <class T, class Move>
__device__ __forceinline__ T wave_sum_steps(T v, Move) {
    v += Move::template step<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
    v += Move::template step<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
    v += Move::template step<0x141, 0xF>(v);  // row_half_mirror
    v += Move::template step<0x140, 0xF>(v);  // row_mirror
    v += Move::template step<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
    v += Move::template step<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
    return v;
}

struct DppMove32 {
    template <int C, int R>
    __device__ static uint32_t step(uint32_t v) { return dpp_u32<C, R>(v); }
};
struct DppMove64 {
    template <int C, int R>
    __device__ static unsigned long long step(unsigned long long v) { return dpp_u64<C, R>(v); }
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    v = wave_sum_steps(v, DppMove32{});
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    v = wave_sum_steps(v, DppMove64{});
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

// Update the WPT same-colour words (I, J0 + 2k), k < WPT, of one row segment.
// `ld(I, J)` / `st(I, J, v)` access the word lattice (global memory or LDS).
// J0 = base + parity; words with J >= L do not exist (ragged last segment).
// The draws of position 20 come from block 5 keyed by word column
// 8*(J div 8) + (J mod 2) and output (J div 2) mod 4.  The words J0 + 2k of
// one thread lie in one aligned group of eight columns (2 WPT divides 8), so
// one block, drawn first, serves all of them; the words are then updated one
// after another, each with its five independent blocks g = 0..4, which keeps
// few registers live.
template <int WPT, bool MEASURE, class Load, class Store>
__device__ __forceinline__ void update_segment(const Load& ld, const Store& st, int I, int J0, const SweepArgs& a,
                                               uint32_t& anti, uint32_t& ups) {
    const int L = a.L, N = a.N;
    const int n_live = min(21, (L - 1 - I) / N + 1);
    const uint64_t live = kSpinBits & (~0ull << (3 * (21 - n_live)));
    const uint32_t row_base = (uint32_t)I * (uint32_t)L;
    const RoundKeys rk = round_keys(a.k0, a.k1);

    // position-20 draws of the segment's words, word k's draw in u5[k]
    uint32_t u5[4] = {0u, 0u, 0u, 0u};
    if (n_live == 21) {
        const uint32_t col = ((uint32_t)J0 & ~7u) | ((uint32_t)J0 & 1u);
        const U4 r = philox_lane_c1(a.t_lo, row_base + col, a.t_hi, 5u | (1u << 3), a.k0, a.k1, rk);
        if (WPT == 4) {  // segments are 8-aligned: output k belongs to word k
            u5[0] = r.x;
            u5[1] = r.y;
            u5[2] = r.z;
            u5[3] = r.w;
        } else {
            const uint32_t q0 = ((uint32_t)J0 >> 1) & 3u;  // first word's output
#pragma unroll
            for (int k = 0; k < WPT; ++k) {
                const uint32_t q = (q0 + (uint32_t)k) & 3u;
                u5[k] = q == 0 ? r.x : q == 1 ? r.y : q == 2 ? r.z : r.w;
            }
        }
    }

    // every word's neighbourhood is loaded first (a thread's words and their
    // neighbourhoods are disjoint from the words it stores); with one word
    // per thread the neighbours are finished at once instead
    Nbhd nb[WPT];
#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        const int J = J0 + 2 * k;
        if (J >= L) break;
        if constexpr (WPT == 1) {
            nb[k].w = ld(I, J);
            nb[k].lf = ld(I, J == 0 ? L - 1 : J - 1);
            nb[k].rt = ld(I, J == L - 1 ? 0 : J + 1);
            nb[k].up = up_word(ld, I, J, N, a.istar, a.sh_star);
            nb[k].dn = down_word(ld, I, J, N, a.istar, a.sh_star);
        } else {
            nb[k] = load_nbhd(ld, I, J, L, N, a.istar);
        }
    }

#pragma unroll
    for (int k = 0; k < WPT; ++k) {
        const int J = J0 + 2 * k;
        if (J >= L) break;

        Codes codes = {0u, 0u, 0u};
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            if (4 * g < n_live) {
                const U4 r =
                    philox_lane_c1(a.t_lo, row_base + (uint32_t)J, a.t_hi, (uint32_t)g | (1u << 3), a.k0, a.k1, rk);
                append_draw(codes, 4 * g + 0, r.x, a.t4, a.t8);
                append_draw(codes, 4 * g + 1, r.y, a.t4, a.t8);
                append_draw(codes, 4 * g + 2, r.z, a.t4, a.t8);
                append_draw(codes, 4 * g + 3, r.w, a.t4, a.t8);
            } else {  // positions past the last live one are dead slots: code 0
#pragma unroll
                for (int j = 0; j < 4; ++j) append_code(codes, 4 * g + j, 0u);
            }
        }
        append_draw(codes, 20, u5[k], a.t4, a.t8);  // dead slot when n_live < 21

        const uint64_t w = nb[k].w, lf = nb[k].lf, rt = nb[k].rt;
        const uint64_t up = WPT == 1 ? nb[k].up : fix_up(nb[k], I, a.sh_star);
        const uint64_t dn = WPT == 1 ? nb[k].dn : fix_down(nb[k], I, N, a.istar, a.sh_star);
        const uint64_t f = flip_mask(w, up, dn, lf, rt, assemble_codes(codes), live);
        const uint64_t nw = w ^ f;
        st(I, J, nw);
        if (MEASURE) measure_word(nw, up, dn, lf, rt, live, anti, ups);
    }
}

}  // namespace ising
