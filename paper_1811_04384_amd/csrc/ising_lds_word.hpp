// The update of one word held in LDS, shared by the kernels that keep a
// band of word columns (every word row of them) in LDS: the multi-sweep
// tiles with redundant halos and the resident tiles that exchange their
// boundary columns.  Lanes of a wavefront may hold words of different rows,
// so the row-dependent parts (live slots, the wrap between the first and
// last word rows, the row-(L-1) patch) are selects, the last two under a
// branch taken only by wavefronts that hold one of those rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ising_device.hpp"

namespace ising {

// q = n div d, r = n mod d for 0 <= n < 2^24, 1 <= d < 2^16, from a float
// estimate (relative error below 2^-22, so off by at most one) and one
// correction, without branches.
__device__ __forceinline__ void divmod_small(int n, int d, float rcp, int& q, int& r) {
    q = (int)((float)n * rcp);
    r = n - q * d;
    const int lo = r < 0 ? 1 : 0, hi = r >= d ? 1 : 0;
    q += hi - lo;
    r += (lo - hi) * d;
}

// What every word update of one lattice in one half-sweep shares
// (wave-uniform).
struct LdsSweep {
    int L, N, istar, sh_star, pstar;  // pstar = (L - 1) div N
    uint32_t t_lo, t_hi, k0, k1, t4, t8;
    bool all_blocks;                  // every row has more than 16 live positions
};

// Neighbourhood words of (I, x) read from LDS: T is the band [N][width],
// xl / xr the local columns of the left / right neighbours.
__device__ __forceinline__ Nbhd lds_nbhd(const uint64_t* __restrict__ T, int width, int N, int istar, int I, int x,
                                         int xl, int xr) {
    Nbhd nb;
    const int row = I * width;
    nb.w = T[row + x];
    nb.lf = T[row + xl];
    nb.rt = T[row + xr];
    nb.up = T[(I > 0 ? I - 1 : N - 1) * width + x];
    nb.dn = T[(I < N - 1 ? I + 1 : 0) * width + x];
    // the patch word (row I* for I = 0, row 0 for I = I*); other rows read
    // row 0 and ignore it
    nb.patch = T[(I == 0 ? istar : 0) * width + x];
    return nb;
}

// Vertical neighbours with the wrap of Section 3 (Fig. 2) and the row-(L-1)
// patch, as fix_up / fix_down, written as selects on the lane's row.
__device__ __forceinline__ uint64_t up_of(const Nbhd& n, int I, int sh_star) {
    const uint64_t wrapped = (n.up >> 3) | (((n.patch >> sh_star) & 1ull) << 60);
    return I > 0 ? n.up : wrapped;
}
__device__ __forceinline__ uint64_t down_of(const Nbhd& n, int I, int N, int istar, int sh_star) {
    const uint64_t d = I < N - 1 ? n.dn : ((n.dn << 3) & kLow63);
    const uint64_t patched = (d & ~(1ull << sh_star)) | (((n.patch >> 60) & 1ull) << sh_star);
    return I == istar ? patched : d;
}

// The sums of measure_word with fewer counts: live has only the spin bit 3k
// of each field, so the masked bond words for up and down shifted by one
// and two bits fill the two free bits of every field, and one count covers
// three of them (likewise for the two up-spin counts).
__device__ __forceinline__ void measure_word_packed(uint64_t w, uint64_t up, uint64_t dn, uint64_t lf, uint64_t rt,
                                                    uint64_t live, uint32_t& anti, uint32_t& ups) {
    const uint64_t b3 = ((w ^ lf) & live) | (((w ^ up) & live) << 1) | (((w ^ dn) & live) << 2);
    anti += __popcll(b3) + __popcll((w ^ rt) & live);
    ups += __popcll((w & live) | ((lf & live) << 1));
}

// The acceptance codes of positions 0..19 of the word with Philox counter
// word c1 = I L + J at sweep t: blocks g = 0..4 of counter (t, c1), four
// positions each (blocks past the last live position skipped on small
// lattices, whose rows have at most 16 live positions).
__device__ __forceinline__ void lds_word_codes19(const LdsSweep& s, const RoundKeys& rk, int n_live, uint32_t c1,
                                                 Codes& codes) {
    if (s.all_blocks) {
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            const U4 r = philox_lane_c1(s.t_lo, c1, s.t_hi, (uint32_t)g | (1u << 3), s.k0, s.k1, rk);
            append_draw(codes, 4 * g + 0, r.x, s.t4, s.t8);
            append_draw(codes, 4 * g + 1, r.y, s.t4, s.t8);
            append_draw(codes, 4 * g + 2, r.z, s.t4, s.t8);
            append_draw(codes, 4 * g + 3, r.w, s.t4, s.t8);
        }
    } else {
#pragma unroll
        for (int g = 0; g < 5; ++g) {
            if (4 * g < n_live) {
                const U4 r = philox_lane_c1(s.t_lo, c1, s.t_hi, (uint32_t)g | (1u << 3), s.k0, s.k1, rk);
                append_draw(codes, 4 * g + 0, r.x, s.t4, s.t8);
                append_draw(codes, 4 * g + 1, r.y, s.t4, s.t8);
                append_draw(codes, 4 * g + 2, r.z, s.t4, s.t8);
                append_draw(codes, 4 * g + 3, r.w, s.t4, s.t8);
            } else {
#pragma unroll
                for (int k = 0; k < 4; ++k) append_code(codes, 4 * g + k, 0u);
            }
        }
    }
}

// The bit-sliced flip of Table 1 and the Metropolis rule applied to the word
// with the assembled codes of all its positions; with meas (wave-uniform),
// adds the word's antiparallel bonds and its and its left neighbour's up
// spins when count (per lane) is set.
__device__ __forceinline__ uint64_t lds_word_flip(const LdsSweep& s, const Nbhd& nb, int I, uint64_t live,
                                                  uint64_t codes, bool meas, bool count, uint32_t& anti,
                                                  uint32_t& ups) {
    // only rows 0, N - 1 and I* wrap or take the patch: the selects run
    // only in the wavefronts that hold such a row
    uint64_t up = nb.up, dn = nb.dn;
    if (I == 0 || I == s.N - 1 || I == s.istar) {
        up = up_of(nb, I, s.sh_star);
        dn = down_of(nb, I, s.N, s.istar, s.sh_star);
    }
    const uint64_t nw = nb.w ^ flip_mask(nb.w, up, dn, nb.lf, nb.rt, codes, live);
    if (meas) {
        uint32_t a = 0, u = 0;
        measure_word_packed(nw, up, dn, nb.lf, nb.rt, live, a, u);
        anti += count ? a : 0u;
        ups += count ? u : 0u;
    }
    return nw;
}

__device__ __forceinline__ uint64_t live_mask(const LdsSweep& s, int I) {
    const int n_live = s.pstar + (I <= s.istar ? 1 : 0);
    return kSpinBits & (~0ull << (3 * (21 - n_live)));
}

// New value of the word (I, J) from its neighbourhood: the 21 acceptance
// codes, those of positions 0..19 as above and that of position 20 from the
// uniform u20 (drawn from the shared block 5 of the word's 8-column group),
// then the flip.
__device__ __forceinline__ uint64_t lds_word_update_c1(const LdsSweep& s, const RoundKeys& rk, const Nbhd& nb, int I,
                                                       uint32_t c1, uint32_t u20, bool meas, bool count,
                                                       uint32_t& anti, uint32_t& ups) {
    Codes codes = {0u, 0u, 0u};
    lds_word_codes19(s, rk, s.pstar + (I <= s.istar ? 1 : 0), c1, codes);
    append_draw(codes, 20, u20, s.t4, s.t8);  // a dead slot when n_live < 21 (masked by live)
    return lds_word_flip(s, nb, I, live_mask(s, I), assemble_codes(codes), meas, count, anti, ups);
}

// The codes of positions 0..19 of a word, assembled, with field 0 (position
// 20) left 0: drawn ahead of the word's update.
__device__ __forceinline__ uint64_t lds_word_codes(const LdsSweep& s, const RoundKeys& rk, int I, uint32_t c1) {
    Codes codes = {0u, 0u, 0u};
    lds_word_codes19(s, rk, s.pstar + (I <= s.istar ? 1 : 0), c1, codes);
    append_code(codes, 20, 0u);
    return assemble_codes(codes);
}

// The update of a word whose codes of positions 0..19 were drawn ahead:
// the code of position 20 from u20 joins them in field 0.
__device__ __forceinline__ uint64_t lds_word_apply(const LdsSweep& s, const Nbhd& nb, int I, uint64_t codes19,
                                                   uint32_t u20, bool meas, bool count, uint32_t& anti,
                                                   uint32_t& ups) {
    const uint64_t codes = codes19 | first_accept(u20, s.t4, s.t8);  // a dead slot when n_live < 21
    return lds_word_flip(s, nb, I, live_mask(s, I), codes, meas, count, anti, ups);
}

// The same, forming c1 from (I, J).
__device__ __forceinline__ uint64_t lds_word_update(const LdsSweep& s, const RoundKeys& rk, const Nbhd& nb, int I,
                                                    int J, uint32_t u20, bool meas, bool count, uint32_t& anti,
                                                    uint32_t& ups) {
    return lds_word_update_c1(s, rk, nb, I, (uint32_t)I * (uint32_t)s.L + (uint32_t)J, u20, meas, count, anti, ups);
}

__device__ __forceinline__ uint32_t pick4(const uint4& v, uint32_t q) {
    return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w;
}

// Philox block 5 of word row I, 8-column group grp and colour c at sweep t:
// the position-20 uniforms of the group's four words of that colour.
__device__ __forceinline__ uint4 block5(const LdsSweep& s, const RoundKeys& rk, int I, int grp, int c) {
    const uint32_t col = (uint32_t)(8 * grp) | (uint32_t)((I + c) & 1);
    const U4 r = philox_lane_c1(s.t_lo, (uint32_t)I * (uint32_t)s.L + col, s.t_hi, 5u | (1u << 3), s.k0, s.k1, rk);
    return make_uint4(r.x, r.y, r.z, r.w);
}

}  // namespace ising
