// Host-side launchers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>

#include "ising_common.hpp"

namespace ising {

// Tiled work of one colour of a lattice: segments of 2*wpt columns per row.
inline int32_t segments_per_row(int32_t L, int32_t wpt) { return (L + 2 * wpt - 1) / (2 * wpt); }
inline int64_t units_per_colour(const Geometry& g, int32_t wpt) {
    return (int64_t)g.N * segments_per_row(g.L, wpt);
}
// Wavefronts of a tiled half-sweep of one lattice: every word row starts a
// new wavefront.
inline int64_t waves_per_colour(const Geometry& g, int32_t wpt) {
    return (int64_t)g.N * ((segments_per_row(g.L, wpt) + 63) / 64);
}

// Zero n 64-bit words with a kernel (usable inside a captured graph).
hipError_t launch_zero_words(uint64_t* p, uint64_t n, hipStream_t s);

// Spins of a fresh lattice: cold (all up) or hot (Philox stream 0 draw < 2^31).
hipError_t launch_init(uint64_t* W, const Geometry& g, uint64_t seed, int hot, hipStream_t s);

// One half-sweep of one lattice (colour 0 or 1).  With `partials` non-null
// (colour 1 only) every wavefront stores its bond/spin counts in
// partials[wave]; the number of launched wavefronts (the slots written) is
// returned in *n_waves.
hipError_t launch_halfsweep_single(int wpt, int block, uint64_t* W, const SweepArgs& a, int colour,
                                   Partial* partials, int64_t* n_waves, hipStream_t s);
int64_t halfsweep_single_waves(const Geometry& g, int wpt, int block);

// Sum the partials of one lattice into E, M and store them: sample index
// `idx` of series (if non-null), out_EM[0..1] (if non-null), and add them to
// the moment sums `mom` (if non-null, device memory).  `scratch`
// is finalize_scratch_bytes() of device memory, zeroed once before first use
// (the kernel leaves it ready for the next call); calls sharing a scratch
// buffer must be ordered on one stream.
size_t finalize_scratch_bytes();
hipError_t launch_finalize_single(const Partial* partials, int64_t n_partials, int32_t L, int64_t* series_E,
                                  int64_t* series_M, int64_t idx, int64_t* out_EM, Moments* mom, void* scratch,
                                  hipStream_t s);

// One phase of the strip dynamics over all strips of one lattice, in one
// kernel (each lane draws and applies its strip's picks).
hipError_t launch_strip_phase(uint64_t* W, const StripArgs& a, hipStream_t s);

// The same phase split in chunks of picks: launch_strip_draws computes the
// words and acceptance codes of picks [k0, k0 + n_k) of every strip into
// pos / codes (n_k * strips entries, pick-major), launch_strip_apply applies
// them in order (a window of picks per step, committing the prefix without
// conflicts), the strips' columns held in LDS.  Usable when one strip fits:
// strip_apply_lds_bytes(a, 1) <= kStripLdsBytes.
constexpr size_t kStripLdsBytes = 64 * 1024;
size_t strip_chain_lds_bytes(const StripArgs& a);
size_t strip_apply_lds_bytes(const StripArgs& a, int chains);
hipError_t launch_strip_draws(const StripArgs& a, uint32_t k0, uint32_t n_k, uint32_t* pos, uint64_t* codes,
                              hipStream_t s);
hipError_t launch_strip_apply(uint64_t* W, const StripArgs& a, uint32_t n_k, const uint32_t* pos,
                              const uint64_t* codes, hipStream_t s);

// Observables of one lattice: per-wavefront partials of right+down
// antiparallel bonds and up spins over all words.
hipError_t launch_observe_single(const uint64_t* W, const Geometry& g, Partial* partials, int64_t* n_waves,
                                 hipStream_t s);
int64_t observe_single_waves(const Geometry& g);

// Unpack an nrows x ncols window (indices mod L) to bytes; write the bytes
// of lattice rows r0 .. r0 + nrows - 1 (1 <= nrows <= N) into their words.
hipError_t launch_unpack(const uint64_t* W, const Geometry& g, int32_t r0, int32_t c0, int32_t nrows,
                         int32_t ncols, uint8_t* out, hipStream_t s);
hipError_t launch_pack_rows(const uint8_t* in, const Geometry& g, int32_t r0, int32_t nrows, uint64_t* W,
                            hipStream_t s);

// ---- batches --------------------------------------------------------------

// Tiled half-sweep over a wave table covering many lattices.  off32: every
// listed lattice is smaller than 4 GiB (32-bit word offsets).  partials
// (colour 1 of a measured sweep): each wavefront stores its sums there.
// fin_partials: before its own work, the launch finalizes every tiled
// lattice's measured sweep fin_off from those partials (written by an
// earlier launch on the same stream).  Lattices whose sweep_limit is <= an
// offset took no part in that sweep and are skipped.
hipError_t launch_halfsweep_multi(int wpt, int block, const LatticeDesc* descs, LatticeState* states,
                                  const WaveItem* waves, int64_t n_waves, int colour, uint32_t sweep_off,
                                  Partial* partials, const Partial* fin_partials, uint32_t fin_off, bool off32,
                                  hipStream_t s);
inline bool fits_off32(const Geometry& g) { return (uint64_t)g.N * (uint64_t)g.L * 8u < (1ull << 32); }
// End of a chunk of k sweeps: finalize the tiled lattices' measured sweep
// fin_off (fin_partials non-null) and advance every lattice's sweep counter
// by min(k, sweep_limit).
hipError_t launch_chunk_end(const LatticeDesc* descs, LatticeState* states, int32_t n_lat,
                            const Partial* fin_partials, uint32_t fin_off, uint32_t k, hipStream_t s);
// One workgroup per listed lattice, K sweeps per launch; samples after local
// sweeps s with (s + 1) % every == 0 (every > 0).  lds_bytes > 0 keeps the
// lattice in LDS (it must fit; call set_resident_lds first, outside any
// graph capture).
hipError_t set_resident_lds(int wpt, size_t lds_bytes);
hipError_t launch_resident(int wpt, int block, const LatticeDesc* descs, LatticeState* states, const int32_t* ids,
                           int32_t n_ids, int32_t K, int32_t every, size_t lds_bytes, hipStream_t s);
// Current E and M into states[i].last_E / last_M for the lattices ids[0..n)
// (ids null: lattices 0..n), and into out_EM[2k], out_EM[2k+1] for the k-th
// listed lattice when out_EM is non-null.
hipError_t launch_observe_multi(const LatticeDesc* descs, LatticeState* states, const int32_t* ids, int32_t n_lat,
                                int64_t* out_EM, hipStream_t s);
// Zero the sample accumulators of every lattice; start a call (series_idx = 0).
hipError_t launch_reset_sums(LatticeState* states, int32_t n_lat, hipStream_t s);
hipError_t launch_begin_call(LatticeState* states, int32_t n_lat, hipStream_t s);

// ---- multi-sweep LDS tiles --------------------------------------------------

// Dynamic LDS of one tile of interior width w (w >= L: the whole lattice)
// for a launch of K sweeps.  A tile fits if its bytes are at most
// tile_lds_limit(device); allow_tile_lds(device) must have run once before
// the first launch_tiles (outside any graph capture).
size_t tile_lds_bytes(int32_t L, int32_t N, int32_t w, int32_t K);
size_t tile_lds_limit(int device);
hipError_t allow_tile_lds(int device);
// Words per tile of the halo copy for tiles of N word rows and launches of
// up to K sweeps.
int64_t tile_halo_stride(int32_t N, int32_t K);
// A launch of the tiles a.tiles[0 .. n_tiles_launched): the halo columns of
// the tiles narrower than their lattice are first copied into `halo`
// (n_tiles_launched x halo_stride words, halo_stride at least
// tile_halo_stride(N, a.K) for every such tile; 0 and null when every tile
// holds a whole lattice), then the tiles run.
hipError_t launch_tiles(const TileLaunch& a, int32_t n_tiles_launched, int block, size_t lds_bytes, uint64_t* halo,
                        int64_t halo_stride, hipStream_t s);
// The n_samples samples of one resident-tile launch of a batch (partials
// [sample][tile], a lattice's tiles at part_begin .. + part_count) for the
// listed lattices: series entries, moment sums, last E and M, in order.
hipError_t launch_finalize_resident(const LatticeDesc* descs, LatticeState* states, const int32_t* ids,
                                    int32_t n_lat, const Partial* partials, int32_t n_tiles, int32_t n_samples,
                                    hipStream_t s);
// E, M of n_samples samples of one lattice from its tiles' partials, in
// order: series entries idx0 .. idx0 + n_samples - 1, moment sums, and the
// last sample into out_EM[0..1] (each optional).
hipError_t launch_finalize_samples(const Partial* partials, int32_t n_tiles, int32_t n_samples, int32_t L,
                                   int64_t* series_E, int64_t* series_M, int64_t idx0, Moments* mom, int64_t* out_EM,
                                   hipStream_t s);

// The samples of one tile launch (sample_mask, first sweep sweep_off of the
// chunk) for the listed lattices of a batch: series entries, moment sums,
// last E and M, in order.
hipError_t launch_finalize_tiles(const LatticeDesc* descs, LatticeState* states, const int32_t* ids, int32_t n_lat,
                                 const Partial* partials, int32_t n_tiles, uint32_t sample_mask, uint32_t sweep_off,
                                 hipStream_t s);

// ---- resident LDS tiles with boundary exchange -------------------------------

// Dynamic LDS of the resident tiles of a lattice cut into bands of w word
// columns (w >= L: the whole lattice) for workgroups of `block` threads;
// the limit and the one-time attribute as for the tiles above.
size_t persist_lds_bytes(int32_t L, int32_t N, int32_t w, int32_t block);
size_t persist_lds_limit(int device);
hipError_t allow_persist_lds(int device);
// How many resident tiles of `block` threads and lds_bytes of LDS the device
// holds at once (a launch must not exceed it).
hipError_t persist_capacity(int block, size_t lds_bytes, int device, int64_t* tiles);
hipError_t launch_persist(const PersistLaunch& a, int32_t n_tiles, int block, size_t lds_bytes, hipStream_t s);
// Runs launch(), which enqueues work holding resident tiles on stream s of
// `device`, ordered after the previous such work of this process on that
// device (a stream wait on its completion event), and makes it the previous
// one.  Inside a graph capture of s, or with another device current,
// launch() runs unordered.
hipError_t resident_gate(int device, hipStream_t s, const std::function<hipError_t()>& launch);
// The n_samples samples of one resident-tile launch of a batch (partials
// [sample][tile], a lattice's tiles at part_begin .. + part_count) for the
// listed lattices: series entries, moment sums, last E and M, in order.
hipError_t launch_finalize_resident(const LatticeDesc* descs, LatticeState* states, const int32_t* ids,
                                    int32_t n_lat, const Partial* partials, int32_t n_tiles, int32_t n_samples,
                                    hipStream_t s);
// E, M of n_samples samples of one lattice from its tiles' partials
// (sample k in partials[k n_tiles ...]) into out_E[k], out_M[k], then, with
// mom, added to the moment sums in order.
hipError_t launch_samples(const Partial* partials, int32_t n_tiles, int32_t n_samples, int32_t L, int64_t* out_E,
                          int64_t* out_M, Moments* mom, hipStream_t s);

// ---- small lattices with their draws taken ahead ----------------------------

// One workgroup per listed lattice, the lattice and the acceptance codes of
// `batch` sweeps (2..64) in LDS (small_lds_bytes), K sweeps, samples as
// launch_resident.  launch_resident uses it for LDS-resident lattices whose
// codes of two or more sweeps fit beside them.
size_t small_lds_bytes(int32_t L, int32_t N, int32_t batch);
size_t small_lds_limit(int device);
hipError_t allow_small_lds(int device);
hipError_t launch_small(int block, const LatticeDesc* descs, LatticeState* states, const int32_t* ids, int32_t n_ids,
                        int32_t K, int32_t every, int32_t batch, size_t lds_bytes, hipStream_t s);

// ---- small lattices with their draws spread over the chip --------------------

// Draw pass: the acceptance codes of sweeps [sweep_off, sweep_off + S) of
// the current chunk of each listed lattice into codes (DrawLat layout);
// max_n_draw = the largest n_draw of the list.
hipError_t launch_draw_codes(const LatticeDesc* descs, const LatticeState* states, const DrawLat* lats, int32_t n_lats,
                             int32_t max_n_draw, uint64_t* codes, int32_t sweep_off, int32_t S, hipStream_t s);
// Apply pass over the same sweeps: one workgroup of `block` threads (64,
// 128 or 256) per listed lattice, wmax (1, 2 or 4:
// wave_apply_words_per_thread) words of a colour per thread, codes loaded
// from the buffer into registers ahead of use; lds_bytes =
// wave_apply_lds_bytes(largest N L, S).  Samples as launch_resident.
hipError_t launch_wave_apply(int wmax, int block, const LatticeDesc* descs, LatticeState* states, const DrawLat* lats,
                             int32_t n_lats, const uint64_t* codes, int32_t sweep_off, int32_t S, int32_t every,
                             size_t lds_bytes, hipStream_t s);
size_t wave_apply_lds_bytes(int32_t NL, int32_t max_samples);
// Words of one colour per thread of a `block`-thread apply workgroup (0:
// more than 4).
int32_t wave_apply_words_per_thread(int32_t L, int32_t N, int32_t block);
hipError_t allow_wave_apply_lds(int device);

// Largest dynamic LDS a resident workgroup may use on this device.
size_t resident_lds_limit(int device);

}  // namespace ising
