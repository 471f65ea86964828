"""GPU parity of the single-lattice path against the CPU oracle.

Bit-exact: the spin state after every call and the exact int64 E, M series
must equal the oracle's on the same seeds (integer work, no tolerance).
Sizes: tiny and ragged lattices (L = 4, 6, 42, 84: not multiples of the
8-column segments, position 20 present or absent), the paper's lattices
L = 21 N (1008, 2016), powers of two (64 ... 4096), and the full-size
L = 32768 lattice in the launch configuration the benchmark times, checked
on windows the oracle evolves exactly.
"""
import sys

import numpy as np
import pytest

import oracle
import paper_1811_04384_amd as ising

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ising.load()
    yield
    torch.cuda.synchronize()


def _oracle_run(L, seed, hot, T_calls):
    """Oracle state and E/M series after each (T, n, every) call."""
    s = oracle.init(L, seed, hot)
    t = 0
    out = []
    for T, n, every in T_calls:
        if every:
            Es, Ms = oracle.sweep(s, seed, t, n, T, every=every)
        else:
            oracle.sweep(s, seed, t, n, T)
            Es = Ms = None
        t += n
        out.append((s.copy(), Es, Ms))
    return out


CASES = [
    (4, 3, True), (6, 5, False), (42, 7, True), (64, 1234, False), (84, 9, True), (128, 2, True),
    (256, 13, True), (1008, 21, True), (2016, 22, False),
]


@pytest.mark.parametrize("L,seed,hot", CASES)
def test_state_and_series_match_oracle(L, seed, hot):
    calls = [(2.269, 3, 1), (1.5, 2, 2), (3.5, 4, 0), (2.0, 3, 3)]
    _log(f"single L={L} seed={seed} hot={hot}")
    ref = _oracle_run(L, seed, hot, calls)
    lat = ising.Lattice(L, seed, hot=hot)
    try:
        assert (lat.spins() == oracle.init(L, seed, hot)).all(), "initial state"
        for (T, n, every), (s_ref, E_ref, M_ref) in zip(calls, ref):
            if every:
                E, M = lat.sweep_measure(T, n, every)
                assert E.cpu().numpy().tolist() == E_ref.tolist()
                assert M.cpu().numpy().tolist() == M_ref.tolist()
            else:
                lat.sweep(T, n)
            got = lat.spins()
            assert (got == s_ref).all(), f"state differs at {np.argwhere(got != s_ref)[:5].tolist()}"
            assert lat.observables() == oracle.observables(s_ref)
        assert lat.t == sum(c[1] for c in calls)
    finally:
        lat.close()


@pytest.mark.parametrize("L", [42, 64, 130, 1008])
def test_every_plan_gives_identical_results(L):
    """Words per thread 1/2/4 and block sizes 64..256: same state (the plan
    changes the thread <-> word mapping and which thread draws the shared
    position-20 block, so this also detects races between threads)."""
    seed, T, n = 77, 2.269, 6
    s_ref = oracle.init(L, seed, True)
    oracle.sweep(s_ref, seed, 0, n, T)
    for wpt in (1, 2, 4):
        for block in (64, 128, 256):
            lat = ising.Lattice(L, seed, hot=True)
            try:
                lat.set_resident_tiles(0)  # the half-sweep launches, whatever the default for L
                lat.set_plan(wpt, block)
                lat.sweep(T, n)
                assert (lat.spins() == s_ref).all(), (wpt, block)
            finally:
                lat.close()


def test_l4096_hot_seed7_matches_oracle():
    """The single-lattice workload's lattice (L = 4096, hot start, seed 7,
    T = 2.269) for a 4-sweep prefix, E/M sampled every 2 sweeps."""
    L, seed, T = 4096, 7, 2.269
    _log("L=4096 oracle prefix")
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 4, T, every=2)
    lat = ising.Lattice(L, seed, hot=True)
    try:
        E, M = lat.sweep_measure(T, 4, 2)
        assert E.cpu().tolist() == Es.tolist() and M.cpu().tolist() == Ms.tolist()
        assert (lat.spins() == s).all()
    finally:
        lat.close()


def test_checkpoint_restore_is_exact():
    L, seed, T = 84, 3, 2.1
    a = ising.Lattice(L, seed, hot=True)
    b = ising.Lattice(L, 999, hot=False)
    try:
        a.sweep(T, 5)
        snap, t = a.spins(), a.t
        a.sweep(T, 7)
        b.set_spins(snap)
        b.t = t
        assert (b.spins() == snap).all()
        # the seed is part of the state: restore into a lattice with the same seed
        c = ising.Lattice(L, seed, hot=False)
        c.set_spins(snap)
        c.t = t
        c.sweep(T, 7)
        assert (c.spins() == a.spins()).all()
        c.close()
    finally:
        a.close()
        b.close()


def test_region_matches_full_state():
    L = 128
    lat = ising.Lattice(L, 5, hot=True)
    try:
        lat.sweep(2.4, 3)
        full = lat.spins()
        for r0, c0, h, w in ((0, 0, 5, 7), (120, 125, 16, 9), (64, 3, 1, 128), (127, 127, 128, 128)):
            rows = [(r0 + i) % L for i in range(h)]
            cols = [(c0 + j) % L for j in range(w)]
            assert (lat.region(r0, c0, h, w) == full[np.ix_(rows, cols)]).all()
    finally:
        lat.close()


def test_set_spins_arbitrary_state_then_sweep():
    L, seed, T = 64, 17, 2.6
    rng = np.random.default_rng(1)
    s0 = rng.integers(0, 2, (L, L)).astype(np.uint8)
    lat = ising.Lattice(L, seed, hot=False)
    try:
        lat.set_spins(s0)
        assert lat.observables() == oracle.observables(s0)
        lat.sweep(T, 4)
        ref = s0.copy()
        oracle.sweep(ref, seed, 0, 4, T)
        assert (lat.spins() == ref).all()
    finally:
        lat.close()


def test_ground_state_and_zero_sweeps():
    L = 96
    lat = ising.Lattice(L, 1, hot=False)
    try:
        lat.sweep(0.1, 0)
        assert lat.t == 0
        E, M = lat.sweep_measure(0.1, 10, 5)
        assert E.cpu().tolist() == [-2 * L * L] * 2 and M.cpu().tolist() == [L * L] * 2
        assert (lat.spins() == 1).all()
    finally:
        lat.close()


def test_invalid_arguments_are_rejected():
    lat = ising.Lattice(16, 1)
    try:
        for bad in (0.0, -1.0, float("inf"), float("nan")):
            with pytest.raises(ising.IsingError):
                lat.sweep(bad, 1)
        with pytest.raises(ising.IsingError):
            lat.sweep(2.0, -1)
        with pytest.raises(ising.IsingError):
            lat.set_plan(3, 256)
        with pytest.raises(ising.IsingError):
            lat.region(0, 0, 17, 1)
    finally:
        lat.close()


def test_l32768_windows_match_oracle():
    """Full-size lattice of the benchmark (L = 32768, hot start, seed 11) in
    the benchmark's launch configuration, 3 sweeps at T = 2.269: windows at
    the corners (periodic wrap in both directions), the word-row seams
    (rows N-1|N, and rows 20N-1..20N around the last position) and the
    interior equal the oracle's exact window evolution; the fused and the
    standalone E/M reductions agree."""
    L, seed, T, n = 32768, 11, 2.269, 3
    N = oracle.word_rows(L)
    lat = ising.Lattice(L, seed, hot=True)
    try:
        _log("L=32768 plan", lat.plan())
        E, M = lat.sweep_measure(T, n, n)
        E2, M2 = lat.observables()
        assert (int(E[0]), int(M[0])) == (E2, M2)
        assert E2 % 4 == 0 and M2 % 2 == 0
        k = 2 * n + 1
        h = w = 24
        spots = [(L - 12, L - 12), (N - 12, 1000), (20 * N - 12, 7), (L - 12, 16000), (12345, L - 5), (777, 20001)]
        for (r, c) in spots:
            r0, c0 = (r - k) % L, (c - k) % L
            win = oracle.init_window(L, seed, True, r0, c0, h + 2 * k, w + 2 * k)
            oracle.sweep_window(win, L, seed, 0, n, T, r0, c0)
            want = win[k:k + h, k:k + w]
            got = lat.region(r0 + k, c0 + k, h, w)
            assert (got == want).all(), (r, c)
    finally:
        lat.close()


def test_largest_lattice_matches_oracle():
    """The largest lattice the library accepts, L = 2^18 (N = 12484 word
    rows, 26 GB of words, beyond 4 GiB so the kernels use 64-bit word
    offsets; I·L + c of the random-number counter still fits 32 bits), in its
    default launch configuration, 2 sweeps at T = 2.5 from a hot start:
    windows at the corners (periodic wrap), the last word row and the seam
    between position 19 and 20, and the interior equal the oracle's exact
    window evolution; E and M are consistent."""
    L, seed, T, n = 1 << 18, 5, 2.5, 2
    N = oracle.word_rows(L)
    assert N * L < 1 << 32 and 8 * N * L > 1 << 32
    lat = ising.Lattice(L, seed, hot=True)
    try:
        _log("L=2^18 plan", lat.plan())
        E, M = lat.sweep_measure(T, n, n)
        E2, M2 = lat.observables()
        assert (int(E[0]), int(M[0])) == (E2, M2)
        assert E2 % 4 == 0 and M2 % 2 == 0 and abs(E2) <= 2 * L * L and abs(M2) <= L * L
        k = 2 * n + 1
        h = w = 20
        spots = [(L - 10, L - 10), (N - 10, 131072), (20 * N - 10, 5), (L - 10, 200000), (100000, L - 4), (4321, 77777)]
        for (r, c) in spots:
            r0, c0 = (r - k) % L, (c - k) % L
            win = oracle.init_window(L, seed, True, r0, c0, h + 2 * k, w + 2 * k)
            oracle.sweep_window(win, L, seed, 0, n, T, r0, c0)
            want = win[k:k + h, k:k + w]
            got = lat.region(r0 + k, c0 + k, h, w)
            assert (got == want).all(), (r, c)
    finally:
        lat.close()


def test_outputs_on_a_non_default_stream_are_ordered():
    """A lattice on a stream of its own: the series tensors (allocated on
    torch's stream, written by the library on the lattice's) read at once on
    torch's stream, and an accumulator zeroed on torch's stream and filled on
    the lattice's, both equal the oracle -- the binding orders the two
    streams around each call."""
    import torch

    L, seed, T = 1008, 3, 2.4
    side = torch.cuda.Stream()
    lat = ising.Lattice(L, seed, hot=True, stream=side)
    try:
        E, M = lat.sweep_measure(T, 40, 4)
        got_E, got_M = E.cpu().numpy().tolist(), M.cpu().numpy().tolist()
        acc = lat.sweep_moments(T, 20, 2)
        got_m = ising.moments_of(acc)
        got_s = lat.spins()
    finally:
        lat.close()
    ref = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(ref, seed, 0, 40, T, every=4)
    Es2, Ms2 = oracle.sweep(ref, seed, 40, 20, T, every=2)
    assert got_E == Es.tolist() and got_M == Ms.tolist()
    assert got_m == oracle.moments(Es2, Ms2)
    assert (got_s == ref).all()


def test_spin_io_in_pieces_through_the_staging_buffer():
    """Spin reads and writes move through a fixed 16 MiB staging buffer:
    at L = 8192 (64 MiB of bytes) a full read, a window that wraps in both
    directions and a full write all take several pieces and stay exact."""
    L, seed = 8192, 17
    lat = ising.Lattice(L, seed, hot=True)
    try:
        ref = oracle.init(L, seed, True)
        assert (lat.spins() == ref).all()
        win = lat.region(L - 3000, L - 5, 5000, 11)
        want = np.roll(np.roll(ref, 3000, axis=0), 5, axis=1)[:5000, :11]
        assert (win == want).all()
        rng = np.random.default_rng(5)
        s = (rng.random((L, L)) < 0.3).astype(np.uint8)
        lat.set_spins(s)
        assert (lat.spins() == s).all()
        assert lat.observables() == oracle.observables(s)
    finally:
        lat.close()
