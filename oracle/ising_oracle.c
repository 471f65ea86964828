/*
 * CPU ORACLE for the checkerboard Metropolis sweep of the 2D periodic Ising
 * model (J = 1, h = 0, k_B = 1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is compared against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the product path never
 * links, imports or calls it, and it shares no code, header, table or constant
 * generator with the HIP library.
 *
 * Representation: one byte per spin, s[r*L + c] in {0, 1} (1 = up = +1,
 * 0 = down = -1), following the paper's "001 = up, 000 = down" convention of
 * Section 3 (multi-spin coding).  There is no packing here at all: every step
 * below is the definition of the method written out site by site.
 *
 * What is computed, and where it comes from:
 *   - Hamiltonian H = -J sum_<m,n> s_m s_n on the periodic square lattice
 *     (Section 2, Eq. 1).
 *   - Metropolis rule: a flip with dE <= 0 is accepted, otherwise accepted
 *     with probability exp(-dE / kT) (Section 2, step 3).  With n = number of
 *     antiparallel nearest neighbours, dE = 8 - 4n in units of J, which is
 *     Table 1 of Section 3.1 (n is the value of the 3-bit group of Eq. 3).
 *   - Energy of a configuration from right and down bonds only, each bond
 *     counted once (Section 5.3, Listing 1).
 *
 * Readings of the paper adopted here (the paper's own driver picks words at
 * random with replacement and reseeds a non-deterministic generator; a
 * reproducible chain needs fixed choices):
 *   - Update order: checkerboard.  Sweep t = every site of colour
 *     (r + c) & 1 == 0, then every site of colour 1; same-colour sites do not
 *     interact, so the order inside a colour is irrelevant.
 *   - Acceptance: integer thresholds t_k = floor(exp(-4k/T) * 2^32) for
 *     k = 1 (dE = +4) and k = 2 (dE = +8), evaluated once on the host in IEEE
 *     double with the C library exp, clamped to 2^32 - 1; a flip with dE > 0
 *     is accepted iff u < t_k for a 32-bit uniform u (strict <).
 *   - Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11,
 *     "Parallel random numbers: as easy as 1, 2, 3"), keyed by the lattice
 *     seed, with the counter built from (sweep, site) as in site_uniform().
 *     One 32-bit output per site per sweep, drawn whether or not it is used.
 *   - Hot start: site is up iff its draw of the initialisation stream is
 *     below 2^31; cold start: every site up.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_API __attribute__((visibility("default")))

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, written from the SC'11 definition.                         */
/* One round maps (c0, c1, c2, c3) with key (k0, k1) to                      */
/*   (hi(B*c2) ^ c1 ^ k0, lo(B*c2), hi(A*c0) ^ c3 ^ k1, lo(A*c0))            */
/* with A = 0xD2511F53, B = 0xCD9E8D57; between rounds the key is advanced   */
/* by the Weyl constants (0x9E3779B9, 0xBB67AE85).                           */
/* ------------------------------------------------------------------------ */
ORACLE_API void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2],
                                     uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ------------------------------------------------------------------------ */
/* Geometry used only to name random numbers.                                */
/* The paper stores column j of a 21N x 21N lattice in N words, word row I   */
/* holding rows I, I+N, ..., I+20N (Section 3, Fig. 1).  For general even L  */
/* take N = the smallest even integer >= L/21; site (r, c) then sits in word */
/* row I = r mod N at position p = r div N (0..20), word column J = c.       */
/* ------------------------------------------------------------------------ */
ORACLE_API int32_t oracle_word_rows(int32_t L)
{
    /* smallest even N with 21 N >= L */
    int32_t n = (L + 20) / 21;
    if (n & 1) n += 1;
    return n;
}

/*
 * The 32-bit uniform drawn for site (r, c) at sweep t of stream `stream`
 * (0 = hot-start initialisation, used with t = 0; 1 = Metropolis sweeps).
 *
 * Counter (c0, c1, c2, c3) = (t mod 2^32, w, t div 2^32, g + 8*stream),
 * key = (seed mod 2^32, seed div 2^32), u = output[q], where
 *   positions p = 0..19: g = p div 4, q = p mod 4, w = I*L + c
 *     (one call serves four positions of the same word);
 *   position p = 20:     g = 5, q = (c div 2) mod 4,
 *                         w = I*L + c0 with c0 = 8*(c div 8) + (c mod 2)
 *     (one call serves position 20 of the four same-colour words
 *      c0, c0+2, c0+4, c0+6 of word row I).
 * Every (t, stream, site) therefore owns a distinct output word.
 */
ORACLE_API uint32_t oracle_site_uniform(uint64_t seed, uint32_t stream, uint64_t t,
                                        int32_t L, int32_t r, int32_t c)
{
    int32_t N = oracle_word_rows(L);
    int32_t I = r % N;
    int32_t p = r / N;
    uint32_t g, q, col;
    if (p < 20) {
        g = (uint32_t)(p >> 2);
        q = (uint32_t)(p & 3);
        col = (uint32_t)c;
    } else {
        g = 5u;
        q = (uint32_t)((c >> 1) & 3);
        col = (uint32_t)((c & ~7) | (c & 1));
    }
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)t;
    ctr[1] = (uint32_t)I * (uint32_t)L + col;
    ctr[2] = (uint32_t)(t >> 32);
    ctr[3] = g | (stream << 3);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
    return out[q];
}

/* ------------------------------------------------------------------------ */
/* Acceptance thresholds: t4 for dE = +4J, t8 for dE = +8J (Section 2 step 3 */
/* with the energies of Table 1).                                            */
/* ------------------------------------------------------------------------ */
static uint32_t threshold_of(double x)
{
    double v = floor(exp(x) * 4294967296.0);
    if (v >= 4294967295.0) return 4294967295u;
    if (v <= 0.0) return 0u;
    return (uint32_t)v;
}

ORACLE_API void oracle_thresholds(double T, uint32_t* t4, uint32_t* t8)
{
    *t4 = threshold_of(-4.0 / T);
    *t8 = threshold_of(-8.0 / T);
}

/*
 * Metropolis decision for a spin with n_anti antiparallel neighbours
 * (0..4): dE = 8 - 4 n_anti (Table 1).  dE <= 0 is always accepted; dE = 4
 * needs u < t4, dE = 8 needs u < t8.
 */
ORACLE_API int oracle_accept(int n_anti, uint32_t u, uint32_t t4, uint32_t t8)
{
    int dE = 8 - 4 * n_anti;
    if (dE <= 0) return 1;
    if (dE == 4) return u < t4;
    return u < t8;
}

/* ------------------------------------------------------------------------ */
/* Lattice state                                                             */
/* ------------------------------------------------------------------------ */
static int valid_L(int32_t L) { return L >= 4 && L <= (1 << 18) && (L % 2) == 0; }

ORACLE_API int oracle_init(int32_t L, uint64_t seed, int32_t hot, uint8_t* s)
{
    if (!valid_L(L)) return -1;
    /* every site's draw is independent of the others: rows in any order */
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < L; ++r)
        for (int32_t c = 0; c < L; ++c)
            s[(int64_t)r * L + c] = hot ? (uint8_t)(oracle_site_uniform(seed, 0, 0, L, r, c) < 0x80000000u)
                                        : (uint8_t)1;
    return 0;
}

/* number of nearest neighbours (periodic) antiparallel to site (r, c) */
static int count_anti(int32_t L, const uint8_t* s, int32_t r, int32_t c)
{
    uint8_t me = s[(int64_t)r * L + c];
    int32_t ru = (r + L - 1) % L, rd = (r + 1) % L;
    int32_t cl = (c + L - 1) % L, cr = (c + 1) % L;
    return (s[(int64_t)ru * L + c] != me) + (s[(int64_t)rd * L + c] != me) +
           (s[(int64_t)r * L + cl] != me) + (s[(int64_t)r * L + cr] != me);
}

static void half_sweep(int32_t L, uint64_t seed, uint64_t t, uint32_t t4, uint32_t t8,
                       uint8_t* s, int colour)
{
    /* sites of one colour never neighbour each other, so any visiting order
       (and any split over threads) gives the same result */
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < L; ++r) {
        for (int32_t c = (r + colour) & 1; c < L; c += 2) {
            int n = count_anti(L, s, r, c);
            uint32_t u = oracle_site_uniform(seed, 1, t, L, r, c);
            if (oracle_accept(n, u, t4, t8)) s[(int64_t)r * L + c] ^= 1u;
        }
    }
}

/* Energy and magnetisation in units of J: E = -sum over right and down
   bonds of sigma sigma' (Section 5.3), M = sum sigma. */
ORACLE_API void oracle_observables(int32_t L, const uint8_t* s, int64_t* E, int64_t* M)
{
    int64_t e = 0, m = 0;
#pragma omp parallel for reduction(+ : e, m) schedule(static)
    for (int32_t r = 0; r < L; ++r) {
        for (int32_t c = 0; c < L; ++c) {
            int sig = s[(int64_t)r * L + c] ? 1 : -1;
            int right = s[(int64_t)r * L + (c + 1) % L] ? 1 : -1;
            int down = s[(int64_t)((r + 1) % L) * L + c] ? 1 : -1;
            e -= sig * (right + down);
            m += sig;
        }
    }
    *E = e;
    *M = m;
}

/* nthreads > 0 uses that many threads; 0 restores the count the process
   started with (a call with an explicit count must not leak into later
   calls). */
static void set_threads(int32_t nthreads)
{
#ifdef _OPENMP
    static int initial = 0;
    if (initial == 0) initial = omp_get_max_threads();
    omp_set_num_threads(nthreads > 0 ? nthreads : initial);
#else
    (void)nthreads;
#endif
}

ORACLE_API int32_t oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * n_sweeps sweeps at temperature T starting at absolute sweep index t0;
 * after sweep number k (1-based within this call) with k % every == 0 the
 * observables are written to E_series[k/every - 1], M_series[...] (skip
 * with every <= 0 or null arrays).  Returns 0, or -1 on bad arguments.
 */
ORACLE_API int oracle_sweep_measure(int32_t L, uint64_t seed, uint64_t t0, int64_t n_sweeps,
                                    double T, uint8_t* s, int32_t every, int64_t* E_series,
                                    int64_t* M_series, int32_t nthreads)
{
    if (!valid_L(L) || n_sweeps < 0 || !(T > 0.0) || isinf(T)) return -1;
    set_threads(nthreads);
    uint32_t t4, t8;
    oracle_thresholds(T, &t4, &t8);
    for (int64_t k = 1; k <= n_sweeps; ++k) {
        uint64_t t = t0 + (uint64_t)(k - 1);
        half_sweep(L, seed, t, t4, t8, s, 0);
        half_sweep(L, seed, t, t4, t8, s, 1);
        if (every > 0 && E_series && M_series && k % every == 0)
            oracle_observables(L, s, &E_series[k / every - 1], &M_series[k / every - 1]);
    }
    return 0;
}

ORACLE_API int oracle_sweep(int32_t L, uint64_t seed, uint64_t t0, int64_t n_sweeps, double T,
                            uint8_t* s, int32_t nthreads)
{
    return oracle_sweep_measure(L, seed, t0, n_sweeps, T, s, 0, NULL, NULL, nthreads);
}

/* ------------------------------------------------------------------------ */
/* Windows: exact evolution of a sub-rectangle of a large lattice.           */
/* A site's state after one half-sweep depends only on itself and its four  */
/* neighbours, and every random number depends only on (seed, t, global     */
/* site), so a window of h x w sites with global origin (r0, c0) evolved in */
/* isolation is exact on rows [k, h-k) x cols [k, w-k) after k half-sweeps.  */
/* ------------------------------------------------------------------------ */
ORACLE_API int oracle_init_window(int32_t L, uint64_t seed, int32_t hot, int32_t r0, int32_t c0,
                                  int32_t h, int32_t w, uint8_t* win)
{
    if (!valid_L(L) || h <= 0 || w <= 0) return -1;
    for (int32_t i = 0; i < h; ++i)
        for (int32_t j = 0; j < w; ++j) {
            int32_t r = (int32_t)(((int64_t)r0 + i) % L), c = (int32_t)(((int64_t)c0 + j) % L);
            win[(int64_t)i * w + j] =
                hot ? (uint8_t)(oracle_site_uniform(seed, 0, 0, L, r, c) < 0x80000000u) : (uint8_t)1;
        }
    return 0;
}

ORACLE_API int oracle_sweep_window(int32_t L, uint64_t seed, uint64_t t0, int64_t n_sweeps,
                                   double T, int32_t r0, int32_t c0, int32_t h, int32_t w,
                                   uint8_t* win, int32_t nthreads)
{
    if (!valid_L(L) || h < 3 || w < 3 || n_sweeps < 0 || !(T > 0.0) || isinf(T)) return -1;
    set_threads(nthreads);
    uint32_t t4, t8;
    oracle_thresholds(T, &t4, &t8);
    for (int64_t k = 0; k < n_sweeps; ++k) {
        uint64_t t = t0 + (uint64_t)k;
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (int32_t i = 1; i < h - 1; ++i) {
                int32_t r = (int32_t)(((int64_t)r0 + i) % L);
                for (int32_t j = 1; j < w - 1; ++j) {
                    int32_t c = (int32_t)(((int64_t)c0 + j) % L);
                    if (((r + c) & 1) != colour) continue;
                    uint8_t me = win[(int64_t)i * w + j];
                    int n = (win[(int64_t)(i - 1) * w + j] != me) + (win[(int64_t)(i + 1) * w + j] != me) +
                            (win[(int64_t)i * w + j - 1] != me) + (win[(int64_t)i * w + j + 1] != me);
                    uint32_t u = oracle_site_uniform(seed, 1, t, L, r, c);
                    if (oracle_accept(n, u, t4, t8)) win[(int64_t)i * w + j] ^= 1u;
                }
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The paper's own dynamics: random word selection inside strips, two       */
/* phases per iteration (Sections 4 and 5.2, Table 2).                      */
/*                                                                           */
/* The word lattice (N word rows x L columns) is cut into L / S vertical     */
/* strips of S word columns; strip p owns columns [pS, pS + S) (one          */
/* process's sub-lattice, Section 4).  One iteration is two phases.  In      */
/* phase 0 every strip updates 10 N h0 words of its left h0 = floor(S/2)     */
/* columns, in phase 1 10 N h1 words of its right h1 = S - h0 columns, each  */
/* word chosen uniformly at random with replacement (ten updates per word on */
/* average, Table 2).  A strip's picks are applied one after another, each   */
/* to the current state.  The columns a strip updates in a phase border only */
/* columns that no strip updates in that phase (Section 4: the border words  */
/* of neighbouring processes are never updated at the same time), so strips  */
/* are independent inside a phase and their order does not matter.          */
/*                                                                           */
/* Updating a word applies the Metropolis rule to each of its live spins     */
/* given the current neighbours.  The spins of one word (rows I + qN) never  */
/* neighbour each other for even N >= 2, so visiting them one by one equals  */
/* the simultaneous word update of Section 3.1.                              */
/*                                                                           */
/* Reproducible random numbers replace the paper's reseeded generator; with */
/* h the phase, t the iteration and key = seed:                              */
/*   pick k of strip p:  counter (t mod 2^32, p, k div 2,                    */
/*                                8 (2 + h) + 256 (t div 2^32))              */
/*     -> (x, y, z, w); pick k uses (x, y) for even k, (z, w) for odd k:     */
/*     word row I = floor(x N / 2^32) and column                             */
/*     J = pS + o_h + floor(y w_h / 2^32), with o_0 = 0, o_1 = h0 and w_h    */
/*     the phase's width;                                                    */
/*   uniform of position q (0..20) in pick k:  counter (t mod 2^32, p, k,    */
/*     g + 8 (4 + h) + 256 (t div 2^32)), g = q div 4, output q mod 4 (for   */
/*     q = 20: g = 5, output 0).                                             */
/* ------------------------------------------------------------------------ */
#define PICK_LIMIT (1u << 22) /* picks of one strip in one phase */

static int32_t phase_width(int32_t S, int32_t h) { return h == 0 ? S / 2 : S - S / 2; }

ORACLE_API int64_t oracle_picks_per_phase(int32_t L, int32_t S, int32_t h)
{
    return 10 * (int64_t)oracle_word_rows(L) * phase_width(S, h);
}

ORACLE_API void oracle_pick(uint64_t seed, uint64_t t, int32_t L, int32_t S, int32_t h, int32_t p,
                            uint32_t k, int32_t* I, int32_t* J)
{
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)t;
    ctr[1] = (uint32_t)p;
    ctr[2] = k >> 1;
    ctr[3] = 8u * (uint32_t)(2 + h) + ((uint32_t)(t >> 32) << 8);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
    uint32_t x = (k & 1) ? out[2] : out[0];
    uint32_t y = (k & 1) ? out[3] : out[1];
    int32_t N = oracle_word_rows(L);
    *I = (int32_t)(((uint64_t)x * (uint64_t)N) >> 32);
    *J = p * S + (h == 0 ? 0 : S / 2) + (int32_t)(((uint64_t)y * (uint64_t)phase_width(S, h)) >> 32);
}

ORACLE_API uint32_t oracle_pick_uniform(uint64_t seed, uint64_t t, int32_t h, int32_t p, uint32_t k,
                                        int32_t q)
{
    uint32_t g = q < 20 ? (uint32_t)(q >> 2) : 5u;
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)t;
    ctr[1] = (uint32_t)p;
    ctr[2] = k;
    ctr[3] = g + 8u * (uint32_t)(4 + h) + ((uint32_t)(t >> 32) << 8);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
    return q < 20 ? out[q & 3] : out[0];
}

static void strip_phase(int32_t L, int32_t S, uint64_t seed, uint64_t t, int32_t h, int32_t p,
                        uint32_t t4, uint32_t t8, uint8_t* s)
{
    int32_t N = oracle_word_rows(L);
    int64_t picks = oracle_picks_per_phase(L, S, h);
    for (int64_t k = 0; k < picks; ++k) {
        int32_t I, J;
        oracle_pick(seed, t, L, S, h, p, (uint32_t)k, &I, &J);
        for (int32_t q = 0; q < 21; ++q) {
            int32_t r = I + q * N;
            if (r >= L) break; /* dead slot */
            int n = count_anti(L, s, r, J);
            uint32_t u = oracle_pick_uniform(seed, t, h, p, (uint32_t)k, q);
            if (oracle_accept(n, u, t4, t8)) s[(int64_t)r * L + J] ^= 1u;
        }
    }
}

ORACLE_API int oracle_random_valid(int32_t L, int32_t S)
{
    if (!valid_L(L) || S < 2 || S > L || L % S != 0) return 0;
    return oracle_picks_per_phase(L, S, 1) <= (int64_t)PICK_LIMIT;
}

/*
 * n_iter iterations of the strip dynamics at temperature T starting at the
 * absolute iteration index t0; after iteration k (1-based in this call) with
 * k % every == 0 the observables go to E_series[k/every - 1], M_series[...].
 * order 0: strips in parallel (OpenMP), 1: strips one by one, last first.
 * Returns 0, or -1 on bad arguments.
 */
ORACLE_API int oracle_random_iterations(int32_t L, uint64_t seed, uint64_t t0, int64_t n_iter, double T,
                                        int32_t S, uint8_t* s, int32_t every, int64_t* E_series,
                                        int64_t* M_series, int32_t order, int32_t nthreads)
{
    if (!oracle_random_valid(L, S) || n_iter < 0 || !(T > 0.0) || isinf(T)) return -1;
    if ((t0 + (uint64_t)n_iter) >> 56) return -1;
    set_threads(nthreads);
    uint32_t t4, t8;
    oracle_thresholds(T, &t4, &t8);
    const int32_t P = L / S;
    for (int64_t k = 1; k <= n_iter; ++k) {
        uint64_t t = t0 + (uint64_t)(k - 1);
        for (int32_t h = 0; h < 2; ++h) {
            if (order == 0) {
#pragma omp parallel for schedule(dynamic, 1)
                for (int32_t p = 0; p < P; ++p) strip_phase(L, S, seed, t, h, p, t4, t8, s);
            } else {
                for (int32_t p = P - 1; p >= 0; --p) strip_phase(L, S, seed, t, h, p, t4, t8, s);
            }
        }
        if (every > 0 && E_series && M_series && k % every == 0)
            oracle_observables(L, s, &E_series[k / every - 1], &M_series[k / every - 1]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Replica multi-spin coding: 21 independent L x L lattices (replicas) in    */
/* one word lattice, the variant of multi-spin coding that packs the same    */
/* site of different systems into one word (the coding family the paper     */
/* builds on, Section 3 and its references).  Word (r, c) holds site (r, c) */
/* of replica k in field 20 - k.  Replicas never interact: each runs the    */
/* checkerboard Metropolis chain of the sections above at its own           */
/* temperature T_k, with its own draws.  Here each replica is one byte      */
/* lattice, s[k L^2 + r L + c].                                              */
/*                                                                           */
/* Draw of replica k at site (r, c), sweep t, stream `stream` (6 = sweeps,  */
/* 7 = hot start at t = 0): Philox key = seed, counter                      */
/* (t mod 2^32, r L + c', t div 2^32, g + 8 stream) and output q with        */
/*   k < 20:  g = k div 4, q = k mod 4, c' = c;                             */
/*   k = 20:  g = 5, q = (c div 2) mod 4, c' = 8 (c div 8) + (c mod 2).      */
/* r L + c' < 2^32 needs L <= 2^16.                                          */
/* ------------------------------------------------------------------------ */
#define REPLICAS 21

static int valid_replica_L(int32_t L) { return L >= 4 && L <= (1 << 16) && (L % 2) == 0; }

ORACLE_API uint32_t oracle_replica_uniform(uint64_t seed, uint32_t stream, uint64_t t, int32_t L, int32_t k,
                                           int32_t r, int32_t c)
{
    uint32_t g, q, col;
    if (k < 20) {
        g = (uint32_t)(k >> 2);
        q = (uint32_t)(k & 3);
        col = (uint32_t)c;
    } else {
        g = 5u;
        q = (uint32_t)((c >> 1) & 3);
        col = (uint32_t)((c & ~7) | (c & 1));
    }
    uint32_t ctr[4], key[2], out[4];
    ctr[0] = (uint32_t)t;
    ctr[1] = (uint32_t)r * (uint32_t)L + col;
    ctr[2] = (uint32_t)(t >> 32);
    ctr[3] = g + 8u * stream;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    oracle_philox4x32_10(ctr, key, out);
    return out[q];
}

ORACLE_API int oracle_replica_init(int32_t L, uint64_t seed, int32_t hot, uint8_t* s)
{
    if (!valid_replica_L(L)) return -1;
    const int64_t n = (int64_t)L * L;
#pragma omp parallel for schedule(static)
    for (int32_t r = 0; r < L; ++r)
        for (int32_t k = 0; k < REPLICAS; ++k)
            for (int32_t c = 0; c < L; ++c)
                s[k * n + (int64_t)r * L + c] =
                    hot ? (uint8_t)(oracle_replica_uniform(seed, 7, 0, L, k, r, c) < 0x80000000u) : (uint8_t)1;
    return 0;
}

/*
 * n_sweeps sweeps of every replica, replica k at temperature T[k], starting
 * at absolute sweep t0; after sweep k (1-based in this call) with
 * k % every == 0 the 21 replicas' E and M go to E_series[(k/every - 1) 21 +
 * replica], M_series[...].  Returns 0, or -1 on bad arguments.
 */
ORACLE_API int oracle_replica_sweep(int32_t L, uint64_t seed, uint64_t t0, int64_t n_sweeps, const double* T,
                                    uint8_t* s, int32_t every, int64_t* E_series, int64_t* M_series,
                                    int32_t nthreads)
{
    if (!valid_replica_L(L) || n_sweeps < 0) return -1;
    for (int32_t k = 0; k < REPLICAS; ++k)
        if (!(T[k] > 0.0) || isinf(T[k])) return -1;
    set_threads(nthreads);
    uint32_t t4[REPLICAS], t8[REPLICAS];
    for (int32_t k = 0; k < REPLICAS; ++k) oracle_thresholds(T[k], &t4[k], &t8[k]);
    const int64_t n = (int64_t)L * L;
    for (int64_t i = 1; i <= n_sweeps; ++i) {
        uint64_t t = t0 + (uint64_t)(i - 1);
        for (int colour = 0; colour < 2; ++colour) {
#pragma omp parallel for schedule(static)
            for (int32_t r = 0; r < L; ++r)
                for (int32_t k = 0; k < REPLICAS; ++k)
                    for (int32_t c = (r + colour) & 1; c < L; c += 2) {
                        uint8_t* sk = s + k * n;
                        int na = count_anti(L, sk, r, c);
                        uint32_t u = oracle_replica_uniform(seed, 6, t, L, k, r, c);
                        if (oracle_accept(na, u, t4[k], t8[k])) sk[(int64_t)r * L + c] ^= 1u;
                    }
        }
        if (every > 0 && E_series && M_series && i % every == 0)
            for (int32_t k = 0; k < REPLICAS; ++k)
                oracle_observables(L, s + k * n, &E_series[(i / every - 1) * REPLICAS + k],
                                   &M_series[(i / every - 1) * REPLICAS + k]);
    }
    return 0;
}
