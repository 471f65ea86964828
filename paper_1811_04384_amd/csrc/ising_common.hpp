// Types shared by the host library and its kernels.
#pragma once

#include <stdint.h>

namespace ising {

// Largest supported linear size; keeps the Philox counter word I*L + J
// below 2^32 (N(L) * L < 2^32 for L <= 2^18).
constexpr int32_t kMaxL = 1 << 18;

// Geometry of one lattice (Section 3 layout with the even-N reading).
struct Geometry {
    int32_t L;        // linear size (even)
    int32_t N;        // word rows: smallest even N with 21 N >= L
    int32_t istar;    // word row holding lattice row L-1: (L-1) mod N
    int32_t sh_star;  // its bit: 3 * (20 - (L-1) div N)
};

inline Geometry make_geometry(int32_t L) {
    Geometry g;
    g.L = L;
    int32_t n = (L + 20) / 21;
    if (n & 1) n += 1;
    g.N = n;
    g.istar = (L - 1) % n;
    g.sh_star = 3 * (20 - (L - 1) / n);
    return g;
}

// Everything a half-sweep of one lattice needs; wave-uniform.
struct SweepArgs {
    int32_t L, N, istar, sh_star;
    uint32_t t_lo, t_hi;  // absolute sweep index
    uint32_t k0, k1;      // Philox key = seed
    uint32_t t4, t8;      // acceptance thresholds
};

// One phase of the strip dynamics (random word picks inside vertical strips
// of S word columns): every strip applies `picks` picks, in order, to the
// `width` columns starting at its column `off`.
struct StripArgs {
    int32_t L, N, istar, sh_star;
    int32_t S, off, width, strips;
    uint32_t picks;       // picks per strip in this phase
    uint32_t phase;       // 0: left half, 1: right half
    uint32_t t_lo, t_hi;  // absolute iteration index
    uint32_t k0, k1;      // Philox key = seed
    uint32_t t4, t8;      // acceptance thresholds
};

// Per-lattice parameters of a batch, written by the host before each call
// and read-only for every kernel.
struct LatticeDesc {
    uint64_t* W;              // word lattice, N x L
    int32_t L, N, istar, sh_star;
    uint32_t k0, k1;          // seed
    uint32_t t4, t8;          // thresholds of the current call
    int64_t units;            // tiled work units (row segments) of one colour
    int32_t segs;             // segments per row for the current tiled plan
    int32_t resident;         // 1: advanced by the resident kernel
    int32_t part_begin;       // first partial-sum slot of this lattice
    int32_t part_count;       // number of partial-sum slots
    int32_t sweep_limit;      // sweeps of the current chunk this lattice takes part in
    int32_t pad_;
    int64_t* series_E;        // per-call sample outputs (may be null)
    int64_t* series_M;
};

// Exact sums over sampled (E, M): the wide ones in little-endian 64-bit
// limbs.  Same layout as ising_moments of the C interface.
struct Moments {
    int64_t n;             // samples
    int64_t sum_E;         // sum of E
    uint64_t sum_E2[2];    // sum of E^2 (128 bits)
    int64_t sum_absM;      // sum of |M|
    uint64_t sum_M2[2];    // sum of M^2 (128 bits)
    uint64_t sum_M4[3];    // sum of M^4 (192 bits)
};

// Per-lattice state of a batch, written only by kernels (the host reads it
// back and zeroes it at creation).
struct LatticeState {
    uint64_t t;               // absolute index of the next sweep
    int64_t series_idx;       // next sample slot of the current call
    Moments mom;              // sums over the samples since the last reset
    int64_t last_E, last_M;   // most recent sample or observation
};

// One wavefront of a tiled half-sweep launch: 64 consecutive row segments
// of one word row of one lattice (segments beyond the row's `segs` idle), so
// the lattice and the row are wave-uniform.
struct WaveItem {
    int32_t lattice;
    int32_t row;   // word row I
    int32_t seg0;  // segment handled by lane 0
};

// Partial sums of one wavefront (or tile): antiparallel bonds and up spins.
struct Partial {
    uint32_t anti;
    uint32_t ups;
};

// One LDS tile of a multi-sweep launch: every word row of the interior word
// columns [c0, c0 + w) of a lattice (w >= L: the whole lattice).
struct TileWork {
    int32_t lattice;  // index into the launch's descriptors
    int32_t c0;       // first interior column
    int32_t w;        // interior columns (even)
    int32_t part;     // this tile's slot in the partial sums of a sample
};

// Largest number of sweeps of one multi-sweep launch.
constexpr int kTileMaxSweeps = 16;

// A multi-sweep launch over a table of tiles.  With `states` the sweep index
// of lattice i is states[i].t + sweep_off and its thresholds and sweep limit
// come from descs[i]; without, every tile uses t0, the key (k0, k1) and
// t4, t8 of the launch, and only the geometry and words of descs.  Sample j of the
// launch (bit j of sample_mask: after its j-th sweep) goes to
// partials[ordinal * n_tiles + tile.part], ordinal = the number of samples
// before it in this launch.
struct TileLaunch {
    const TileWork* tiles;
    const LatticeDesc* descs;
    LatticeState* states;
    uint64_t t0;
    uint32_t k0, k1;  // key (without states)
    uint32_t t4, t8;
    uint32_t sweep_off;
    int32_t K;
    uint32_t sample_mask;
    int32_t n_tiles;
    Partial* partials;
};

}  // namespace ising

namespace ising {

// One resident tile: every word row of the interior word columns
// [c0, c0 + w) of a lattice (w >= L: the whole lattice), and the tiles that
// own the columns beside it (their indices in the launch).
struct PersistTile {
    int32_t lattice;
    int32_t c0, w;
    int32_t left, right;
    int32_t part;  // slot in the partial sums of a sample
};

// A launch of resident tiles: K sweeps of every listed tile.  The sweep
// index, key and thresholds come from states/descs or from the launch as for
// TileLaunch.  Sample after sweep j of the launch iff (sample_base + j + 1)
// is a multiple of every (every = 0: none); the sample's partial sums go to
// partials[ordinal * n_tiles + tile.part].  exch holds exch_tile_words
// (>= 4 N) words per tile, flags one word per tile; both persist between
// launches.  A tile's flag reaches 2 t + s + 1 when it has published its
// boundary words of half-sweep s (0 or 1) of its lattice's absolute sweep
// t, so flags only grow while sweep counters do (a counter set back needs
// its lattice's flags zeroed).  A wait longer than wait_ticks (100 MHz
// clock) sets *error and ends the launch early.
struct PersistLaunch {
    const PersistTile* tiles;
    const LatticeDesc* descs;
    LatticeState* states;
    uint64_t t0;
    uint32_t k0, k1, t4, t8;
    uint32_t sweep_off;
    int32_t K;
    int32_t every;
    int64_t sample_base;
    int32_t n_tiles;
    Partial* partials;
    uint64_t* exch;
    int64_t exch_tile_words;
    uint64_t* flags;
    uint32_t* error;
    uint64_t wait_ticks;
};

// A small lattice whose acceptance codes are drawn ahead by a chip-wide
// launch into a global buffer: its codes of sweep j of a draw pass start at
// codes + base + j N L (layout [sweeps][N][L]); n_draw = 2 N ceil(L / 8)
// draw items per sweep (colour, word row, 8-column group).
struct DrawLat {
    int32_t lat;
    int32_t n_draw;
    int64_t base;
};

}  // namespace ising
