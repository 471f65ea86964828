/*
 * ising.h -- C ABI of the MI355X (gfx950) multi-spin-coded Ising library.
 *
 * The library runs the checkerboard Metropolis sweep of the 2D square-lattice
 * Ising model with periodic boundaries, J = 1, h = 0, k_B = 1
 * (Hamiltonian: Section 2, Eq. 1; acceptance rule: Section 2, steps 1-3),
 * on lattices stored with the paper's multi-spin coding: 21 spins of 3 bits
 * in each 64-bit word, bit 63 always 0, "001" = up and "000" = down
 * (Section 3), word row I of column J holding the spins of rows
 * I, I+N, ..., I+20N (Section 3, Fig. 1), with the periodic wrap between the
 * first and last word rows made by 3-bit shifts (Section 3, Fig. 2).  The
 * neighbour count is the XOR sum of Eq. 3 and its meaning is Table 1 of
 * Section 3.1.  Energies are computed from right and down bonds, each bond
 * once (Section 5.3, Listing 1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - L: linear size, even, 4 <= L <= 262144 (2^18).  The lattice has L*L
 *    spins.  The word lattice has N(L) rows and L columns, N(L) the smallest
 *    even integer >= L/21; rows r >= L of the 21*N(L) coded rows are dead
 *    slots (always 0, never flipped, not counted).  For L = 21N with N even
 *    this is exactly the paper's layout.
 *  - Word layout in device memory: uint64 W[N][L], row major (column index
 *    fastest); the spin of row r, column c is bit 3*(20 - r/N) of W[r%N][c].
 *  - T: temperature in units of J/k_B, finite and > 0.  The acceptance
 *    thresholds t4 = floor(exp(-4/T) 2^32) and t8 = floor(exp(-8/T) 2^32)
 *    (clamped to 2^32-1) are computed on the host in IEEE double; a move with
 *    dE = +4J (+8J) is accepted iff its 32-bit uniform u < t4 (u < t8), moves
 *    with dE <= 0 always.
 *  - Random numbers: Philox4x32-10 keyed by the 64-bit seed
 *    (key = (seed mod 2^32, seed div 2^32)).  Site (r, c) at absolute sweep t
 *    uses counter (t mod 2^32, I*L + c', t div 2^32, g + 8*stream) and output
 *    word q, with I = r mod N, p = r div N and
 *      p < 20:  g = p div 4, q = p mod 4, c' = c;
 *      p = 20:  g = 5, q = (c div 2) mod 4, c' = 8*(c div 8) + (c mod 2);
 *    stream 0 is the hot-start draw (t = 0), stream 1 the Metropolis sweeps.
 *    A hot start sets a site up iff its draw is < 2^31; a cold start sets all
 *    spins up.
 *  - Sweep t: all sites with (r + c) even are updated, then all with
 *    (r + c) odd.  Sweep indices are absolute per lattice: sweeping a then b
 *    equals sweeping a + b, and the temperature may change between calls.
 *  - E = -sum over bonds of s_i s_j (each bond once), M = sum of s_i, both
 *    exact int64 in units of J (resp. spins).
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls that only enqueue device work return before it runs;
 *    only the calls documented as synchronising wait for the stream.
 *  - Memory: "device pointer" means memory the GPU can address (hipMalloc or
 *    a torch CUDA tensor); "host pointer" means ordinary process memory.
 *    The library never frees memory it did not allocate.
 *  - Errors: every int-returning call returns ISING_OK (0) or a negative
 *    ISING_E* code and then leaves a message for ising_last_error() in
 *    thread-local storage.  No C++ exception crosses this interface.
 *  - Threading: one handle must not be used by two threads at once; distinct
 *    handles are independent.
 */
#ifndef ISING_H
#define ISING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ISING_OK = 0,
    ISING_EINVAL = -1, /* argument out of range (L, T, sweeps, pointers, sizes)      */
    ISING_ENOMEM = -2, /* device allocation failed or a memory budget is exceeded    */
    ISING_EHIP = -3,   /* a HIP runtime call failed (message names it)               */
    ISING_EBUSY = -4,  /* the object is in a state that forbids the call             */
    ISING_EAGAIN = -5  /* nothing available yet (server queue)                       */
};
enum { ISING_COLD = 0, ISING_HOT = 1 };

/* Exact sums over sampled states (E_k, M_k), k = 1..n_samples.  The wide
   sums are unsigned little-endian 64-bit limbs (value = sum_j limb[j] 2^(64j)).
   Exact for every L <= 2^18 while n_samples < 2^26 (sum_E, sum_absM) and
   n_samples < 2^48 (the wide sums). */
typedef struct {
    int64_t n_samples;
    int64_t sum_E;       /* sum of E                  */
    uint64_t sum_E2[2];  /* sum of E^2, 128 bits      */
    int64_t sum_absM;    /* sum of |M|                */
    uint64_t sum_M2[2];  /* sum of M^2, 128 bits      */
    uint64_t sum_M4[3];  /* sum of M^4, 192 bits      */
} ising_moments;

/* Per-spin thermodynamics of one set of moments at temperature T on L x L
   spins (k_B = J = 1), <x> = sum x / n_samples:
     e      = <E> / L^2                          (the paper's average energy,
                                                  Section 2, Eq. 2, per spin)
     c      = (<E^2> - <E>^2) / (T^2 L^2)        specific heat
     abs_m  = <|M|> / L^2
     chi    = (<M^2> - <|M|>^2) / (T L^2)        susceptibility
     binder = 1 - <M^4> / (3 <M^2>^2)            Binder cumulant
   The fluctuation formulas are the standard canonical-ensemble ones; the
   paper itself reports only e. */
typedef struct {
    double e, c, abs_m, chi, binder;
} ising_thermo;

/* ising_thermodynamics: host arithmetic only (long double), no device work.
   EINVAL for NULL pointers, n_samples < 1, invalid L or T.  binder is NaN
   when <M^2> = 0. */
int ising_thermodynamics(const ising_moments* m, int32_t L, double T, ising_thermo* out);

typedef struct ising_lattice ising_lattice; /* one lattice (opaque)                 */
typedef struct ising_batch ising_batch;     /* many lattices, one launch per phase  */
typedef struct ising_server ising_server;   /* continuous-batching request server   */
typedef struct ising_replicas ising_replicas; /* 21 replicas sharing one word lattice */

/* ------------------------------------------------------------------ */
/* Geometry and thresholds (host only, no GPU needed)                   */
/* ------------------------------------------------------------------ */

/* N(L), the number of word rows (Section 3 with the even-N reading for
   L not a multiple of 21); 0 if L is invalid. */
int32_t ising_word_rows(int32_t L);

/* Bytes of the packed word lattice, 8 * N(L) * L; 0 if L is invalid. */
size_t ising_required_bytes(int32_t L);

/* Acceptance thresholds for temperature T (Section 2, step 3, with dE from
   Table 1).  EINVAL if T is not finite and > 0. */
int ising_thresholds(double T, uint32_t* t4, uint32_t* t8);

/* Library version string and the GPU architecture it was built for. */
const char* ising_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* ising_last_error(void);

/* ------------------------------------------------------------------ */
/* Single lattice: one lattice per kernel launch                        */
/* ------------------------------------------------------------------ */

/* Allocate (hipMalloc) and initialise a lattice: init = ISING_COLD or
   ISING_HOT (Section 5.1 initialises at random; the hot start is that).
   The initialisation kernel is enqueued on `stream`.  *out receives the
   handle; the library owns it and its device memory. */
int ising_create(int32_t L, uint64_t seed, int32_t init, void* stream, ising_lattice** out);

/* As ising_create, but the word lattice lives in a caller-owned device
   buffer `dev_words` of `bytes` >= ising_required_bytes(L) bytes, 8-byte
   aligned, which must outlive the handle (e.g. a torch CUDA tensor). */
int ising_create_in(int32_t L, uint64_t seed, int32_t init, void* dev_words, size_t bytes, void* stream,
                    ising_lattice** out);

/* Re-initialise the lattice in place (cold or hot start with `seed`, as
   ising_create) and set the sweep count to 0; enqueued on the handle's
   stream, no allocation.  The seed of later sweeps becomes `seed`. */
int ising_reset(ising_lattice* h, uint64_t seed, int32_t init);

/* Release the handle (and the device memory the library allocated).
   Waits for the handle's stream first.  NULL is accepted. */
int ising_destroy(ising_lattice* h);

/* Enqueue n_sweeps >= 0 checkerboard sweeps at temperature T. */
int ising_sweep(ising_lattice* h, double T, int64_t n_sweeps);

/* As ising_sweep, and after the k-th sweep of this call (k = every, 2 every,
   ...) store that state's E and M in dev_E[k/every - 1] and dev_M[k/every - 1]
   (device pointers to n_sweeps/every int64 each).  The reduction is fused
   into the second half of the sampled sweep.  every >= 1. */
int ising_sweep_measure(ising_lattice* h, double T, int64_t n_sweeps, int32_t every, int64_t* dev_E,
                        int64_t* dev_M);

/* As ising_sweep_measure, but every sampled (E, M) is added to the moment
   sums *dev_acc (a device pointer to one ising_moments, which the caller
   zeroes before the first call and may keep adding to) instead of a series. */
int ising_sweep_moments(ising_lattice* h, double T, int64_t n_sweeps, int32_t every, ising_moments* dev_acc);

/* Temperature scan with the lattice carried over from one temperature to
   the next, the paper's driver loop (Section 5: the program steps the
   temperature and keeps the lattice, averaging the energy of the iterations
   at each temperature): for i = 0..n_T-1, therm >= 0 sweeps at T[i] without
   sampling, then meas >= 0 sweeps at T[i] sampled after every every-th
   (every >= 1), whose moments are stored in out[i] (host array of n_T).  An
   ascending T is a heating scan, a descending one a cooling scan.  Advances
   the sweep counter by n_T (therm + meas).  Synchronises. */
int ising_scan(ising_lattice* h, int32_t n_T, const double* T, int64_t therm, int64_t meas, int32_t every,
               ising_moments* out);

/* The paper's own dynamics instead of the checkerboard: random word
   selection inside vertical strips (Sections 4 and 5.2).  The word lattice
   is cut into L/strip_cols strips of strip_cols word columns (one process's
   sub-lattice each; 2 <= strip_cols <= L, strip_cols divides L).  One
   iteration is two phases: in phase 0 every strip updates
   10 N floor(strip_cols/2) words of its left floor(strip_cols/2) columns,
   in phase 1 10 N (strip_cols - floor(strip_cols/2)) words of its right
   columns, each word chosen uniformly with replacement and updated from the
   current state (ten updates per word on average, Table 2).  Strips are
   independent inside a phase (their border words are never updated in the
   same phase, Section 4) and run in parallel.  Random numbers, with h the
   phase, t the absolute iteration index (the handle's sweep counter) and
   key = seed: pick k of strip p uses Philox counter
   (t mod 2^32, p, k div 2, 8 (2 + h) + 256 (t div 2^32)), outputs (x, y) for
   even k and (z, w) for odd k, word row floor(x N / 2^32) and column
   p strip_cols + (h ? floor(strip_cols/2) : 0) + floor(y width / 2^32); the
   uniform of position q of pick k is output q mod 4 (q = 20: output 0) of
   counter (t mod 2^32, p, k, g + 8 (4 + h) + 256 (t div 2^32)),
   g = min(q div 4, 5).  Acceptance as for the checkerboard.
   After the k-th iteration of this call with k % every == 0, E and M are
   stored at dev_E[k/every - 1], dev_M[k/every - 1] and added to *dev_acc
   (device pointers; each may be NULL; every >= 1 when any is given,
   every = 0 takes no samples).  Advances the sweep counter by n_iterations.
   EINVAL if a strip would apply more than 2^22 picks in one phase. */
int ising_random_iterations(ising_lattice* h, double T, int32_t strip_cols, int64_t n_iterations, int32_t every,
                            int64_t* dev_E, int64_t* dev_M, ising_moments* dev_acc);

/* For callers that cannot allocate device memory (code under graph
   capture, tight serving loops, harnesses that forbid it): the sweeps of
   ising_sweep_measure on a caller-owned word lattice, with no handle and no
   allocation.  dev_words: device buffer of bytes >= ising_required_bytes(L)
   bytes (8-byte aligned) holding the lattice in the layout above (for
   example the words of a handle, ising_words); it is advanced by n_sweeps
   >= 0 sweeps at T with key `seed`, the first being absolute sweep t0; after
   the k-th sweep with k % every == 0 (every >= 1) E and M go to
   dev_E[k/every - 1], dev_M[k/every - 1] (device pointers).  The launch
   shape is ising_create's default one-launch-per-half-sweep plan.  Its
   scratch (the partial sums of a sampled half-sweep and their reduction
   state) is a fixed 2 MiB device array, per GPU, held until the process
   ends: EINVAL for a lattice whose partial sums would not fit (L above
   32768).  Enqueued on `stream`; allocates nothing.  Calls that overlap on
   one GPU (different streams, threads) share that scratch and race; calls
   ordered on one stream do not.  The scratch keeps the last call's
   contents; each call clears what must start at zero itself (with a kernel,
   so it may be captured into a graph). */
int ising_sweep_measure_static(void* dev_words, size_t bytes, int32_t L, uint64_t seed, uint64_t t0, double T,
                               int64_t n_sweeps, int32_t every, int64_t* dev_E, int64_t* dev_M, void* stream);

/* E and M of the current state (host pointers).  Synchronises the stream. */
int ising_observables(ising_lattice* h, int64_t* E, int64_t* M);

/* Copy the spins to a host array of L*L bytes, row major, 1 = up, 0 = down.
   Synchronises the stream. */
int ising_get_spins(ising_lattice* h, uint8_t* host_spins);

/* Spins of the h x w window with top-left site (r0, c0), indices taken
   modulo L, into a host array of h*w bytes.  1 <= h, w <= L.  Synchronises. */
int ising_get_spins_region(ising_lattice* h, int32_t r0, int32_t c0, int32_t nrows, int32_t ncols,
                           uint8_t* host_spins);

/* Replace the state by a host array of L*L bytes (nonzero = up).  The sweep
   counter is unchanged.  Synchronises the stream. */
int ising_set_spins(ising_lattice* h, const uint8_t* host_spins);

/* Number of sweeps done (the absolute index of the next sweep).  Together
   with the spins this is the complete state: set_spins + set_sweep_count
   restore a checkpoint exactly. */
int ising_get_sweep_count(ising_lattice* h, uint64_t* t);
int ising_set_sweep_count(ising_lattice* h, uint64_t t);

/* Device pointer to the word lattice and its size in bytes (read-only view
   for callers that move or inspect words themselves). */
int ising_words(ising_lattice* h, void** dev_words, size_t* bytes);

/* Kernel variant used by ising_sweep*: words_per_thread in {1, 2, 4} (same-
   colour words of one row handled by one thread; 4 lets one Philox call serve
   position 20 of four words) and block a multiple of 64 in [64, 256].
   Results never depend on the choice. */
int ising_set_plan(ising_lattice* h, int32_t words_per_thread, int32_t block);
int ising_get_plan(ising_lattice* h, int32_t* words_per_thread, int32_t* block);

/* Several sweeps per launch on LDS tiles (the paper's sub-lattices with
   ghost columns, Sections 4 and 5.2, Figs. 3 and 5, as redundant halos):
   with sweeps_per_launch = K in [1, 16], ising_sweep* runs K sweeps per
   launch, each workgroup on one tile -- every word row of tile_cols interior
   word columns (even) plus 2K halo columns on each side, all in LDS -- and
   K = 0 goes back to one launch per half-sweep.  tile_cols >= L keeps the
   whole lattice in one workgroup; otherwise tile_cols + 4K <= L.  block:
   threads per workgroup, a multiple of 64 in [64, 1024].  EINVAL if a tile
   does not fit in LDS.  Synchronises the stream.  Results never depend on
   it.  Setting it switches resident tiles off.  ising_get_tiling returns
   K = 0 (and zeros) when tiling is off. */
int ising_set_tiling(ising_lattice* h, int32_t sweeps_per_launch, int32_t tile_cols, int32_t block);
int ising_get_tiling(ising_lattice* h, int32_t* sweeps_per_launch, int32_t* tile_cols, int32_t* block);

/* Resident tiles (the paper's decomposition into vertical strips with
   ghost columns, Sections 4 and 5.2, Figs. 3 and 5, on the workgroups of one
   GPU): with tile_cols > 0, ising_sweep* keeps every word row of tile_cols
   word columns (even) in one workgroup's LDS, for up to max_sweeps
   (1..4096) sweeps per launch, and each half-sweep trades the tiles'
   boundary words with the neighbouring tiles through global memory;
   tile_cols >= L keeps the whole lattice in one workgroup.  block: threads
   per workgroup, a multiple of 64 in [64, 1024].  tile_cols = 0 switches it
   off; either this or ising_set_tiling is in effect, the last one set.
   EINVAL if a tile does not fit in LDS or the tiles do not all fit on the
   device at once.  A launch whose tiles wait for a neighbour longer than
   about a second is abandoned: the next call on the handle returns
   ISING_EHIP, and the lattice state is undefined.  Launches of resident
   tiles on different streams of one device (of this or other handles and
   batches) run one after another.  Synchronises.  Results never depend on
   it.  ising_get_resident_tiles returns zeros when off.
   ising_create and ising_create_in switch it on for L <= 7680 (up to
   L = 192 the whole lattice in one workgroup of one thread per word of a
   colour, a power of two from 64 to 1024; below L = 1024 bands of 8
   columns, 512 threads; from there bands of 2 ceil(L / 512) columns, 1024
   threads; 1000 sweeps per launch) when those fit. */
int ising_set_resident_tiles(ising_lattice* h, int32_t tile_cols, int32_t block, int32_t max_sweeps);
/* Bound of every wait of the resident-tile launches for their neighbour
   tiles, in ticks of the GPU's 100 MHz constant clock; 0 restores the
   default of 100,000,000 (one second), at most one minute (EINVAL beyond).
   A launch whose wait runs past it sets an error word and every tile of the
   launch stops at once, so the launch always ends; the next call on the
   handle that checks (a sweep, ising_observables, ising_synchronize)
   returns ISING_EHIP and clears it, and the lattice state is undefined until
   ising_reset or ising_set_spins.  A small bound is how a caller (a test)
   can exercise that path without a fault. */
int ising_set_resident_wait(ising_lattice* h, uint64_t ticks);
int ising_get_resident_tiles(ising_lattice* h, int32_t* tile_cols, int32_t* block, int32_t* max_sweeps);

/* Time every plan on this lattice's shape (on a scratch copy, the state is
   not touched) and keep the fastest.  Synchronises.  best_ms (host, may be
   NULL) receives the time per sweep of the chosen plan. */
int ising_autotune(ising_lattice* h, double T, double* best_ms_per_sweep);

/* Wait for all work enqueued on the handle's stream. */
int ising_synchronize(ising_lattice* h);

/* ------------------------------------------------------------------ */
/* Batch: many independent lattices of mixed L and T advanced together  */
/* ------------------------------------------------------------------ */

/* n >= 1 lattices; L[i], seed[i], init[i] as for ising_create (host arrays).
   All words live in one library-owned device arena. */
int ising_batch_create(int32_t n, const int32_t* L, const uint64_t* seed, const int32_t* init, void* stream,
                       ising_batch** out);
int ising_batch_destroy(ising_batch* b);

/* Advance every lattice i by n_sweeps at temperature T[i] (host array).
   every = 0: no measurement.  every >= 1: after each every-th sweep of this
   call, every lattice's E and M are added to its running sums (see
   ising_batch_results) and, if dev_E / dev_M are non-NULL, stored at
   dev_E[i * (n_sweeps/every) + k] (device pointers, int64).  The work is
   enqueued as hipGraph replays of one chunk of sweeps. */
int ising_batch_sweep(ising_batch* b, const double* T, int64_t n_sweeps, int32_t every, int64_t* dev_E,
                      int64_t* dev_M);

/* Per-lattice results into host arrays of n int64 (any may be NULL): the
   current E and M, and sum_E, sum_absM, n_samples accumulated by every
   measuring ising_batch_sweep since creation or the last reset.
   Synchronises. */
int ising_batch_results(ising_batch* b, int64_t* E, int64_t* M, int64_t* sum_E, int64_t* sum_absM,
                        int64_t* n_samples);
int ising_batch_reset_sums(ising_batch* b);

/* Per-lattice moment sums over the same samples as ising_batch_results
   (host array of n).  Synchronises. */
int ising_batch_moments(ising_batch* b, ising_moments* out);

/* Temperature scan of every lattice of the batch at once, each carried over
   from one temperature to the next: for step j = 0..n_T-1 every lattice i
   takes therm sweeps at T[j*n + i] without sampling, then meas sweeps sampled
   after every every-th (every >= 1), whose moments go to out[j*n + i] (host
   arrays of n_T*n).  The running sums of ising_batch_results are reset at
   each step and hold the last step's samples afterwards.  Synchronises. */
int ising_batch_scan(ising_batch* b, int32_t n_T, const double* T, int64_t therm, int64_t meas, int32_t every,
                     ising_moments* out);

/* Spins of lattice i (host array of L[i]^2 bytes); sweep counter of i. */
int ising_batch_get_spins(ising_batch* b, int32_t i, uint8_t* host_spins);
/* Spins of the nrows x ncols window of lattice i with top-left site
   (r0, c0), indices taken modulo L[i], into a host array of nrows*ncols
   bytes, row major, 1 = up.  1 <= nrows, ncols <= L[i]; EINVAL otherwise or
   for i out of range.  Synchronises the batch's stream. */
int ising_batch_get_spins_region(ising_batch* b, int32_t i, int32_t r0, int32_t c0, int32_t nrows, int32_t ncols,
                                 uint8_t* host);
int ising_batch_get_sweep_count(ising_batch* b, int32_t i, uint64_t* t);

/* Execution plan.  Lattices with L <= resident_max_L are advanced by one
   workgroup each, all their sweeps of a chunk inside one launch, the lattice
   held in LDS when it fits; lattices with resident_max_L < L <= tile_max_L
   by LDS tiles of tile_cols word columns: with tile_exchange = 0,
   tile_sweeps sweeps per launch on tiles with redundant halos (as
   ising_set_tiling); with tile_exchange = 1, resident tiles that keep their
   words in LDS for a whole chunk and trade boundary words every half-sweep
   (as ising_set_resident_tiles; the lattices whose tiles would exceed what
   the device holds at once, in index order, go to the next path); a lattice
   whose tile would not fit in LDS goes to the next path; the others
   by per-half-sweep launches over a table of (lattice, row segment) work
   items with words_per_thread words per thread.  sweeps_per_graph sweeps are
   captured in one hipGraph (rounded to a multiple of `every`).  With
   draw_sweeps > 0, resident lattices with at most 4 x min(resident_block,
   256) words of a colour (L up to 128 with 256 threads) instead have their
   acceptance codes (which do not depend on the spins, Table 1) drawn by a
   launch spread over the whole chip, draw_sweeps sweeps at a time (a
   device buffer of draw_sweeps x 8 x their words bytes, capped at
   256 MiB), and applied by one workgroup of min(resident_block, 256)
   threads per lattice.  Results never depend on the plan. */
typedef struct {
    int32_t resident_max_L;   /* 0 = no resident lattices                    */
    int32_t resident_block;   /* threads per resident workgroup (64..1024)   */
    int32_t words_per_thread; /* 1, 2 or 4 (half-sweep path)                 */
    int32_t tiled_block;      /* threads per half-sweep workgroup (64..256)  */
    int32_t sweeps_per_graph; /* >= 1                                        */
    int32_t tile_max_L;       /* 0 = no multi-sweep tiles                    */
    int32_t tile_sweeps;      /* sweeps per tile launch, 1..16               */
    int32_t tile_cols;        /* interior word columns per tile (even)       */
    int32_t tile_block;       /* threads per tile workgroup (64..1024)       */
    int32_t tile_exchange;    /* 1: resident tiles trading boundary words    */
    int32_t draw_sweeps;      /* 0, or sweeps per chip-wide draw (1..4096)   */
} ising_batch_plan;

/* Validate a plan without a batch (host only, no GPU needed): ISING_OK or
   EINVAL with the reason.  resident_max_L must be in [0, 4096]: one
   workgroup per lattice is only sensible for lattices that fit, or nearly
   fit, in one workgroup's LDS.  With tile_max_L > 0, tile_sweeps must be in
   [1, 16], tile_cols even and >= 2, tile_block a multiple of 64 in
   [64, 1024], tile_exchange 0 or 1.  draw_sweeps must be in [0, 4096].
   ising_batch_set_plan applies the same checks. */
int ising_batch_check_plan(const ising_batch_plan* plan);
int ising_batch_set_plan(ising_batch* b, const ising_batch_plan* plan);
int ising_batch_get_plan(ising_batch* b, ising_batch_plan* plan);

/* Autotuner: time candidate plans on a scratch batch of the same shapes
   (this batch's state is untouched), keep the fastest, and record it in the
   JSON file cache_path (may be NULL) keyed by GPU architecture and the
   multiset of L.  If the file already holds an entry for that key, it is
   used without timing.  Synchronises. */
int ising_batch_autotune(ising_batch* b, const double* T, const char* cache_path, ising_batch_plan* chosen);

/* ------------------------------------------------------------------ */
/* Server: continuous batching of simulation requests                   */
/* ------------------------------------------------------------------ */

typedef struct {
    uint64_t req_id;
    int32_t L;
    int32_t status;       /* ISING_OK, or a negative code if the request failed */
    double T;
    int64_t sweeps;
    int64_t E, M;         /* observables of the final state                     */
    double t_submit_s;    /* host clock (seconds, CLOCK_MONOTONIC) at submit    */
    double t_admit_s;     /* when its lattice was created on the device         */
    double t_done_s;      /* when its result was read back                      */
} ising_result;

/* A server holding at most max_slots resident lattices whose packed words
   (ising_required_bytes) sum to at most hbm_budget bytes.  Work proceeds in
   quanta of `quantum_sweeps` sweeps over all resident lattices; requests are
   admitted in arrival order as slots and budget free up and leave as soon as
   their sweeps are done. */
int ising_server_create(size_t hbm_budget, int32_t max_slots, int32_t quantum_sweeps, void* stream,
                        ising_server** out);

/* Queue a request (host-side, never blocks on the GPU).  EINVAL for bad
   arguments or a lattice larger than the whole budget. */
int ising_server_submit(ising_server* s, uint64_t req_id, int32_t L, double T, int64_t sweeps, uint64_t seed,
                        int32_t init);

/* Run one scheduling quantum: retire finished lattices (reading E, M),
   admit queued requests that fit, and launch one quantum of sweeps for all
   resident lattices.  *active (may be NULL) receives the number of resident
   lattices after the call.  Synchronises the previous quantum. */
int ising_server_step(ising_server* s, int32_t* active);

/* Move up to cap finished results into out (host array); *n receives how
   many.  Returns ISING_OK even when *n == 0. */
int ising_server_poll(ising_server* s, ising_result* out, int32_t cap, int32_t* n);

/* Counts of queued, resident and finished-but-unpolled requests, and the
   bytes of resident lattices. */
int ising_server_stats(ising_server* s, int32_t* queued, int32_t* resident, int32_t* finished, size_t* bytes_in_use);

int ising_server_destroy(ising_server* s);

/* ------------------------------------------------------------------ */
/* Replica multi-spin coding: 21 independent lattices in one word lattice */
/* ------------------------------------------------------------------ */

/* The other packing of the multi-spin-coding family the paper builds on
   (Section 3 and its references): word (r, c), r, c < L, holds site (r, c)
   of replica k = 0..20 in field 20 - k (bit 3 (20 - k)).  Replicas never
   interact: replica k runs the checkerboard Metropolis chain of the single
   lattice (same Table 1 rule, same integer thresholds) at its own
   temperature T[k], with its own draws: Philox key = seed, counter
   (t mod 2^32, r L + c', t div 2^32, g + 8 stream), output q, where
   k < 20: g = k div 4, q = k mod 4, c' = c; k = 20: g = 5,
   q = (c div 2) mod 4, c' = 8 (c div 8) + (c mod 2); stream 6 for sweeps,
   7 for the hot start (t = 0; up iff the draw is < 2^31).  The word lattice
   is uint64 W[L][L], 8 L^2 bytes for 21 L^2 spins.  4 <= L <= 65536, even
   (r L + c' must fit 32 bits).  E, M arrays hold the 21 replicas in order. */
int ising_replicas_create(int32_t L, uint64_t seed, int32_t init, void* stream, ising_replicas** out);
int ising_replicas_destroy(ising_replicas* h);

/* n_sweeps sweeps of every replica, replica k at T[k] (host array of 21). */
int ising_replicas_sweep(ising_replicas* h, const double* T, int64_t n_sweeps);

/* As ising_replicas_sweep; after the k-th sweep of the call with
   k % every == 0 the replicas' E and M go to dev_E[(k/every - 1) 21 + i],
   dev_M[...] (device pointers to (n_sweeps/every) 21 int64 each). */
int ising_replicas_sweep_measure(ising_replicas* h, const double* T, int64_t n_sweeps, int32_t every, int64_t* dev_E,
                                 int64_t* dev_M);

/* As ising_replicas_sweep_measure, but the samples are added to the moment
   sums dev_acc[0..20] (device pointer to 21 ising_moments, zeroed by the
   caller before the first call). */
int ising_replicas_sweep_moments(ising_replicas* h, const double* T, int64_t n_sweeps, int32_t every,
                                 ising_moments* dev_acc);

/* E[21], M[21] of the current state (host arrays).  Synchronises. */
int ising_replicas_observables(ising_replicas* h, int64_t* E, int64_t* M);

/* Spins of replica k as L*L host bytes (1 = up).  Synchronises. */
int ising_replicas_get_spins(ising_replicas* h, int32_t k, uint8_t* host_spins);

/* Sweeps done (the absolute index of the next sweep). */
int ising_replicas_get_sweep_count(ising_replicas* h, uint64_t* t);

/* Words per thread of the half-sweep kernel, 1, 2 or 4 (default 2).
   Results never depend on it. */
int ising_replicas_set_plan(ising_replicas* h, int32_t words_per_thread);

#ifdef __cplusplus
}
#endif

#endif /* ISING_H */
