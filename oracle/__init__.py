"""CPU oracle for the checkerboard Metropolis Ising sweep -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  The GPU library never imports it.  It wraps the plain C
implementation in ``ising_oracle.c`` (one byte per spin, its own
Philox4x32-10) with numpy arrays; see that file for the definitions and the
passages of the paper each function follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libising_oracle.so")
_lib = None

COLD = 0
HOT = 1


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build  # build only if nothing is built yet
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32, u32, u64, i64, dbl = ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
    lib.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
    lib.oracle_philox4x32_10.restype = None
    lib.oracle_word_rows.argtypes = [i32]
    lib.oracle_word_rows.restype = i32
    lib.oracle_site_uniform.argtypes = [u64, u32, u64, i32, i32, i32]
    lib.oracle_site_uniform.restype = u32
    lib.oracle_thresholds.argtypes = [dbl, u32p, u32p]
    lib.oracle_thresholds.restype = None
    lib.oracle_accept.argtypes = [ctypes.c_int, u32, u32, u32]
    lib.oracle_accept.restype = ctypes.c_int
    lib.oracle_init.argtypes = [i32, u64, i32, u8p]
    lib.oracle_init.restype = ctypes.c_int
    lib.oracle_observables.argtypes = [i32, u8p, i64p, i64p]
    lib.oracle_observables.restype = None
    lib.oracle_sweep_measure.argtypes = [i32, u64, u64, i64, dbl, u8p, i32, i64p, i64p, i32]
    lib.oracle_sweep_measure.restype = ctypes.c_int
    lib.oracle_sweep.argtypes = [i32, u64, u64, i64, dbl, u8p, i32]
    lib.oracle_sweep.restype = ctypes.c_int
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = i32
    lib.oracle_init_window.argtypes = [i32, u64, i32, i32, i32, i32, i32, u8p]
    lib.oracle_init_window.restype = ctypes.c_int
    lib.oracle_sweep_window.argtypes = [i32, u64, u64, i64, dbl, i32, i32, i32, i32, u8p, i32]
    lib.oracle_sweep_window.restype = ctypes.c_int
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.oracle_picks_per_phase.argtypes = [i32, i32, i32]
    lib.oracle_picks_per_phase.restype = i64
    lib.oracle_pick.argtypes = [u64, u64, i32, i32, i32, i32, u32, i32p, i32p]
    lib.oracle_pick.restype = None
    lib.oracle_pick_uniform.argtypes = [u64, u64, i32, i32, u32, i32]
    lib.oracle_pick_uniform.restype = u32
    lib.oracle_random_valid.argtypes = [i32, i32]
    lib.oracle_random_valid.restype = ctypes.c_int
    lib.oracle_random_iterations.argtypes = [i32, u64, u64, i64, dbl, i32, u8p, i32, i64p, i64p, i32, i32]
    lib.oracle_random_iterations.restype = ctypes.c_int
    dblp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_replica_uniform.argtypes = [u64, u32, u64, i32, i32, i32, i32]
    lib.oracle_replica_uniform.restype = u32
    lib.oracle_replica_init.argtypes = [i32, u64, i32, u8p]
    lib.oracle_replica_init.restype = ctypes.c_int
    lib.oracle_replica_sweep.argtypes = [i32, u64, u64, i64, dblp, u8p, i32, i64p, i64p, i32]
    lib.oracle_replica_sweep.restype = ctypes.c_int
    _lib = lib
    return lib


def _u8(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def library_path():
    return _LIB_PATH


def philox4x32_10(ctr, key):
    """Philox4x32-10 block: 4 counter words, 2 key words -> 4 output words."""
    lib = _load()
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib.oracle_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def word_rows(L):
    return int(_load().oracle_word_rows(int(L)))


def site_uniform(seed, stream, t, L, r, c):
    return int(_load().oracle_site_uniform(int(seed), int(stream), int(t), int(L), int(r), int(c)))


def thresholds(T):
    """(t4, t8) = floor(exp(-4/T) 2^32), floor(exp(-8/T) 2^32), clamped."""
    t4 = ctypes.c_uint32()
    t8 = ctypes.c_uint32()
    _load().oracle_thresholds(float(T), ctypes.byref(t4), ctypes.byref(t8))
    return int(t4.value), int(t8.value)


def accept(n_anti, u, t4, t8):
    return bool(_load().oracle_accept(int(n_anti), int(u), int(t4), int(t8)))


def max_threads():
    return int(_load().oracle_max_threads())


def init(L, seed, hot):
    """Initial state, uint8 array (L, L): 1 = up, 0 = down."""
    s = np.empty((L, L), dtype=np.uint8)
    if _load().oracle_init(int(L), int(seed), int(bool(hot)), _u8(s)) != 0:
        raise ValueError(f"invalid lattice size L={L}")
    return s


def observables(s):
    """Exact (E, M) of a uint8 (L, L) state: E = -sum of right+down bonds."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    E = ctypes.c_int64()
    M = ctypes.c_int64()
    _load().oracle_observables(int(s.shape[0]), _u8(s), ctypes.byref(E), ctypes.byref(M))
    return int(E.value), int(M.value)


def sweep(s, seed, t0, n_sweeps, T, every=0, threads=0):
    """Advance state ``s`` (modified in place) by n_sweeps sweeps at T.

    Sweep indices are absolute: the first sweep performed is t0.  With
    ``every > 0`` returns (E_series, M_series) sampled after every
    ``every``-th sweep of this call; otherwise returns None.
    """
    assert s.dtype == np.uint8 and s.flags.c_contiguous and s.shape[0] == s.shape[1]
    L = s.shape[0]
    n = int(n_sweeps)
    if every > 0:
        k = n // every
        Es = np.zeros(k, dtype=np.int64)
        Ms = np.zeros(k, dtype=np.int64)
        rc = _load().oracle_sweep_measure(L, int(seed), int(t0), n, float(T), _u8(s), int(every),
                                          _i64(Es), _i64(Ms), int(threads))
        if rc != 0:
            raise ValueError("bad sweep arguments")
        return Es, Ms
    rc = _load().oracle_sweep(L, int(seed), int(t0), n, float(T), _u8(s), int(threads))
    if rc != 0:
        raise ValueError("bad sweep arguments")
    return None


def moments(Es, Ms):
    """Exact sums over a sample series, as Python ints: the number of samples,
    sum E, sum E^2, sum |M|, sum M^2, sum M^4."""
    Es = [int(e) for e in Es]
    Ms = [int(m) for m in Ms]
    return {"n_samples": len(Es), "sum_E": sum(Es), "sum_E2": sum(e * e for e in Es),
            "sum_absM": sum(abs(m) for m in Ms), "sum_M2": sum(m * m for m in Ms),
            "sum_M4": sum(m ** 4 for m in Ms)}


def scan(L, seed, hot, Ts, therm, meas, every=1, threads=0, state=None, t0=0):
    """Temperature scan with the lattice carried over, the paper's driver
    loop (Section 5: the temperature is stepped while the lattice is kept,
    and the energies of the iterations at each temperature are averaged,
    Section 2, Eq. 2): at each T in order, ``therm`` sweeps without samples,
    then ``meas`` sweeps sampled after every ``every``-th.

    Returns (list of moments dicts, final state, next sweep index)."""
    s = init(L, seed, hot) if state is None else state
    t = int(t0)
    out = []
    for T in Ts:
        sweep(s, seed, t, therm, T, threads=threads)
        t += int(therm)
        Es, Ms = sweep(s, seed, t, meas, T, every, threads=threads)
        t += int(meas)
        out.append(moments(Es, Ms))
    return out, s, t


def thermodynamics(m, L, T):
    """Per-spin canonical averages from exact moment sums (k_B = J = 1), in
    exact rational arithmetic rounded once: e = <E>/L^2 (Eq. 2 per spin),
    c = (<E^2> - <E>^2)/(T^2 L^2), |m| = <|M|>/L^2,
    chi = (<M^2> - <|M|>^2)/(T L^2), binder = 1 - <M^4>/(3 <M^2>^2)."""
    from fractions import Fraction

    n = m["n_samples"]
    if n < 1:
        raise ValueError("no samples")
    N = Fraction(L * L)
    T = Fraction(float(T))
    E1, E2 = Fraction(m["sum_E"], n), Fraction(m["sum_E2"], n)
    A1, M2, M4 = Fraction(m["sum_absM"], n), Fraction(m["sum_M2"], n), Fraction(m["sum_M4"], n)
    return {"e": float(E1 / N), "c": float((E2 - E1 * E1) / (T * T * N)), "abs_m": float(A1 / N),
            "chi": float((M2 - A1 * A1) / (T * N)),
            "binder": float(1 - M4 / (3 * M2 * M2)) if M2 else float("nan")}


def init_window(L, seed, hot, r0, c0, h, w):
    win = np.empty((h, w), dtype=np.uint8)
    if _load().oracle_init_window(int(L), int(seed), int(bool(hot)), int(r0), int(c0), int(h), int(w),
                                  _u8(win)) != 0:
        raise ValueError("bad window")
    return win


def sweep_window(win, L, seed, t0, n_sweeps, T, r0, c0, threads=0):
    """Evolve a window in place; exact on [2n, h-2n) x [2n, w-2n) afterwards."""
    assert win.dtype == np.uint8 and win.flags.c_contiguous
    h, w = win.shape
    rc = _load().oracle_sweep_window(int(L), int(seed), int(t0), int(n_sweeps), float(T), int(r0), int(c0),
                                     int(h), int(w), _u8(win), int(threads))
    if rc != 0:
        raise ValueError("bad window sweep")


def picks_per_phase(L, S, phase):
    """Words a strip of S columns updates in one phase: 10 N floor(S/2) for
    phase 0, 10 N (S - floor(S/2)) for phase 1."""
    return int(_load().oracle_picks_per_phase(int(L), int(S), int(phase)))


def pick(seed, t, L, S, phase, p, k):
    """(word row I, word column J) of pick k of strip p in a phase of iteration t."""
    I, J = ctypes.c_int32(), ctypes.c_int32()
    _load().oracle_pick(int(seed), int(t), int(L), int(S), int(phase), int(p), int(k), ctypes.byref(I),
                        ctypes.byref(J))
    return int(I.value), int(J.value)


def pick_uniform(seed, t, phase, p, k, q):
    return int(_load().oracle_pick_uniform(int(seed), int(t), int(phase), int(p), int(k), int(q)))


def random_valid(L, S):
    return bool(_load().oracle_random_valid(int(L), int(S)))


def random_iterations(s, seed, t0, n_iter, T, S, every=0, order=0, threads=0):
    """The paper's strip dynamics (random word picks, two phases per
    iteration) on state ``s`` in place, starting at absolute iteration t0.
    With every > 0 returns (E_series, M_series) sampled after every
    every-th iteration of this call."""
    assert s.dtype == np.uint8 and s.flags.c_contiguous and s.shape[0] == s.shape[1]
    L = s.shape[0]
    n = int(n_iter)
    k = n // every if every > 0 else 0
    Es = np.zeros(max(k, 1), dtype=np.int64)
    Ms = np.zeros(max(k, 1), dtype=np.int64)
    rc = _load().oracle_random_iterations(L, int(seed), int(t0), n, float(T), int(S), _u8(s), int(every),
                                          _i64(Es), _i64(Ms), int(order), int(threads))
    if rc != 0:
        raise ValueError("bad strip-dynamics arguments")
    return (Es[:k], Ms[:k]) if every > 0 else None


REPLICAS = 21


def replica_uniform(seed, stream, t, L, k, r, c):
    """Draw of replica k at site (r, c), sweep t (stream 6 sweeps, 7 hot start)."""
    return int(_load().oracle_replica_uniform(int(seed), int(stream), int(t), int(L), int(k), int(r), int(c)))


def replica_init(L, seed, hot):
    """21 replicas, uint8 array (21, L, L): 1 = up."""
    s = np.empty((REPLICAS, L, L), dtype=np.uint8)
    if _load().oracle_replica_init(int(L), int(seed), int(bool(hot)), _u8(s)) != 0:
        raise ValueError(f"invalid replica lattice size L={L}")
    return s


def replica_sweep(s, seed, t0, n_sweeps, T, every=0, threads=0):
    """Advance 21 replicas (array (21, L, L), in place), replica k at T[k].
    With every > 0 returns (E, M) arrays of shape (n // every, 21)."""
    assert s.dtype == np.uint8 and s.flags.c_contiguous and s.shape[0] == REPLICAS
    L = s.shape[1]
    T = np.ascontiguousarray(np.broadcast_to(np.asarray(T, dtype=np.float64), (REPLICAS,)))
    n = int(n_sweeps)
    k = n // every if every > 0 else 0
    Es = np.zeros((max(k, 1), REPLICAS), dtype=np.int64)
    Ms = np.zeros((max(k, 1), REPLICAS), dtype=np.int64)
    rc = _load().oracle_replica_sweep(L, int(seed), int(t0), n, T.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                      _u8(s), int(every), _i64(Es), _i64(Ms), int(threads))
    if rc != 0:
        raise ValueError("bad replica sweep arguments")
    return (Es[:k], Ms[:k]) if every > 0 else None
