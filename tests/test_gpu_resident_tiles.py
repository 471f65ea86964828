"""GPU parity of resident LDS tiles that trade boundary columns (every word
row of a band of word columns kept in one workgroup's LDS for many sweeps,
the neighbouring bands' boundary words exchanged through global memory
every half-sweep) against the CPU oracle.

Bit-exact: the spin state after every call and every sampled E, M equal the
oracle's.  Cases: the whole lattice in one workgroup (no exchange), many
bands, two bands (each the other's left and right neighbour), ragged last
bands down to two columns, L not a multiple of 8 or of 21, the paper's
L = 21 N lattices, samples spanning launches (calls longer than one launch),
workgroups of 64 to 1024 threads, both ways of drawing the codes (per
word item in its half-sweep, or a half-sweep ahead into LDS code tables),
and the library's default shapes from L = 4 to 7680.
"""
import pytest

import oracle
import paper_1811_04384_amd as ising

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ising.load()


CALLS = [(2.269, 7, 0), (1.5, 10, 3), (3.5, 5, 1), (2.6, 9, 2)]

# (L, seed, hot, tile columns, block, sweeps per launch)
CASES = [
    (4, 3, True, 4, 64, 5),
    (6, 5, False, 6, 64, 3),
    (42, 7, True, 8, 128, 4),
    (64, 1234, False, 64, 256, 1000),
    (84, 9, True, 14, 128, 2),
    (128, 2, True, 20, 192, 7),
    (130, 11, True, 16, 256, 3),
    (252, 12, True, 126, 512, 4),
    (256, 13, True, 256, 1024, 16),
    (1006, 4, True, 48, 512, 5),
    (1008, 21, True, 48, 512, 9),
    (2016, 22, True, 96, 1024, 4),
    # at most two words of a colour per thread: items formed once per launch
    # and codes drawn a half-sweep ahead (two rounds on two wavefronts; the
    # heating scan's bands, 24 even rounds)
    (168, 3, False, 40, 128, 6),
    (1008, 25, True, 64, 1024, 5),
    # wide bands with more words per thread and a narrow last band with at
    # most two (its code tables must fit the LDS reserved for the wide ones)
    (1008, 23, True, 22, 256, 3),
    (1010, 24, False, 32, 256, 4),
    # a partial last round of second items (more words of a colour than
    # threads, not a multiple of 64 more) with 256 and 512 threads
    (200, 31, True, 60, 256, 5),
    (500, 32, False, 50, 512, 6),
]


@pytest.mark.parametrize("L,seed,hot,cols,block,K", CASES)
def test_resident_tiles_match_oracle(L, seed, hot, cols, block, K):
    print(f"resident tiles L={L} cols={cols} block={block} K={K}", flush=True)
    lat = ising.Lattice(L, seed, hot=hot)
    try:
        lat.set_resident_tiles(cols, block, K)
        assert lat.resident_tiles() == (min(cols, L), block, K)
        s = oracle.init(L, seed, hot)
        t = 0
        for T, n, every in CALLS:
            if every:
                E, M = lat.sweep_measure(T, n, every)
                Es, Ms = oracle.sweep(s, seed, t, n, T, every=every)
                assert E.cpu().numpy().tolist() == Es.tolist(), (T, n, every)
                assert M.cpu().numpy().tolist() == Ms.tolist(), (T, n, every)
            else:
                lat.sweep(T, n)
                oracle.sweep(s, seed, t, n, T)
            t += n
            assert (lat.spins() == s).all(), (T, n, every)
        assert lat.observables() == oracle.observables(s)
    finally:
        lat.close()


def test_resident_tiles_moments_and_other_paths():
    """Resident tiles, half-sweep launches and halo tiles on one sweep
    counter; moment sums across all three."""
    L, seed, T = 1008, 31, 2.4
    lat = ising.Lattice(L, seed, hot=True)
    try:
        lat.set_resident_tiles(64, 512, 4)
        acc = lat.sweep_moments(T, 6, 1)
        lat.set_tiling(2, 64, 512)
        assert lat.resident_tiles() == (0, 0, 0)
        lat.sweep_moments(T, 5, 1, acc)
        lat.set_tiling(0)
        lat.sweep_moments(T, 3, 1, acc)
        lat.set_resident_tiles(32, 256, 1000)
        assert lat.tiling() == (0, 0, 0)
        lat.sweep_moments(T, 7, 1, acc)
        m = ising.moments_of(acc)
        spins = lat.spins()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 21, T, every=1)
    assert m == oracle.moments(Es, Ms)
    assert (spins == s).all()


def test_resident_tiles_l4096_prefix_matches_oracle():
    """The plain workload's lattice (L = 4096, hot start seed 7, T = 2.269)
    in 256 bands of 16 columns, E/M every 10 sweeps, 30 sweeps in launches
    of 20: series and state equal the oracle's."""
    L, seed, T = 4096, 7, 2.269
    lat = ising.Lattice(L, seed, hot=True)
    try:
        lat.set_resident_tiles(16, 512, 20)
        E, M = lat.sweep_measure(T, 30, 10)
        got = lat.spins()
        got_E, got_M = E.cpu().numpy().tolist(), M.cpu().numpy().tolist()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 30, T, every=10)
    assert got_E == Es.tolist() and got_M == Ms.tolist()
    assert (got == s).all()


@pytest.mark.parametrize("L,tiles", [(4, (4, 64, 1000)), (64, (64, 128, 1000)), (130, (130, 1024, 1000)),
                                     (192, (192, 1024, 1000)), (194, (8, 512, 1000)), (512, (8, 512, 1000)),
                                     (770, (8, 512, 1000)), (1024, (4, 1024, 1000)), (2304, (10, 1024, 1000)),
                                     (5000, (20, 1024, 1000)), (7680, (30, 1024, 1000))])
def test_default_resident_tiles_match_oracle(L, tiles):
    """The library's default up to L = 7680 (the whole lattice in one
    workgroup up to L = 192, then bands of 8 columns, then bands of about
    L/256 columns, all resident at once): the default is taken, and series
    and state equal the oracle's (ragged last bands at L = 194 and 770, the
    largest band that fits at L = 7680)."""
    seed, T = 3 + L, 2.269
    lat = ising.Lattice(L, seed, hot=True)
    try:
        assert lat.resident_tiles() == tiles
        print(f"default resident tiles L={L} {tiles}", flush=True)
        E, M = lat.sweep_measure(T, 7, 2)
        got = lat.spins()
        got_E, got_M = E.cpu().numpy().tolist(), M.cpu().numpy().tolist()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 7, T, every=2)
    assert got_E == Es.tolist() and got_M == Ms.tolist()
    assert (got == s).all()


def test_resident_launches_on_two_streams():
    """Two lattices in the default resident tiles (256 bands of 1024 threads
    each, one per compute unit) on two streams, every call made with its own
    stream current so that nothing but the library orders them: each
    launch runs after the device's previous resident launch, so neither
    waits out its bound on tiles the other holds, and both equal the
    oracle."""
    import torch

    L, T = 2048, 2.269
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    lats = [ising.Lattice(L, 50 + k, hot=True, stream=streams[k]) for k in range(2)]
    try:
        assert all(lat.resident_tiles() == (8, 1024, 1000) for lat in lats)
        print("resident tiles on two streams", flush=True)
        for _ in range(3):
            for k in range(2):
                with torch.cuda.stream(streams[k]):
                    lats[k].sweep(T, 40)
        series = []
        for k in range(2):
            with torch.cuda.stream(streams[k]):
                series.append(lats[k].sweep_measure(T, 20, 5))
        torch.cuda.synchronize()
        for k in range(2):
            lats[k].synchronize()
            s = oracle.init(L, 50 + k, True)
            oracle.sweep(s, 50 + k, 0, 120, T)
            Es, Ms = oracle.sweep(s, 50 + k, 120, 20, T, every=5)
            E, M = series[k]
            assert E.cpu().numpy().tolist() == Es.tolist() and M.cpu().numpy().tolist() == Ms.tolist(), k
            assert (lats[k].spins() == s).all(), k
    finally:
        for lat in lats:
            lat.close()


def test_default_plan_outside_the_resident_range():
    """Above 7680 columns the default stays one launch per half-sweep."""
    for L in (7682, 8192):
        lat = ising.Lattice(L, 1, hot=False)
        try:
            assert lat.resident_tiles() == (0, 0, 0), L
        finally:
            lat.close()


def test_default_resident_tiles_l4096_full_launch_matches_oracle():
    """The single-lattice workload in the launch configuration the benchmark
    times: L = 4096, hot start seed 7, T = 2.269, the default plan (256
    bands of 16 columns, 1024 threads, 1000 sweeps per launch), one whole
    launch of 1000 sweeps with E/M every 10 sweeps: all 100 samples and the
    final state equal the oracle's (about 20 s of oracle work)."""
    L, seed, T = 4096, 7, 2.269
    lat = ising.Lattice(L, seed, hot=True)
    try:
        assert lat.resident_tiles() == (16, 1024, 1000)
        print("L=4096 default plan, one 1000-sweep launch", flush=True)
        E, M = lat.sweep_measure(T, 1000, 10)
        got = lat.spins()
        got_E, got_M = E.cpu().numpy().tolist(), M.cpu().numpy().tolist()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 1000, T, every=10)
    assert got_E == Es.tolist() and got_M == Ms.tolist()
    assert (got == s).all()


def test_invalid_resident_tiles_are_rejected():
    lat = ising.Lattice(4096, 1, hot=True)
    try:
        default = lat.resident_tiles()
        assert default == (16, 1024, 1000)  # the library's default for this size
        for bad in ((7, 256, 10), (-2, 256, 10), (16, 96, 10), (16, 2048, 10), (16, 256, 0), (16, 256, 5000),
                    (2, 1024, 10)):  # the last: 2048 bands of 1024 threads exceed what the device holds at once
            with pytest.raises(ising.IsingError) as e:
                lat.set_resident_tiles(*bad)
            assert e.value.code == ising.ISING_EINVAL
        assert lat.resident_tiles() == default  # a refused setting leaves the plan as it was
        lat.set_resident_tiles(0)
        assert lat.resident_tiles() == (0, 0, 0)
    finally:
        lat.close()
    big = ising.Lattice(32768, 1, hot=False)
    try:
        with pytest.raises(ising.IsingError):
            big.set_resident_tiles(64, 256, 10)  # 1562 word rows: a band does not fit in LDS
    finally:
        big.close()


def test_resident_tiles_after_reset_and_counter_set_back():
    """The tiles' flags follow the sweep counter: after ising_reset and a
    checkpoint restore to an earlier sweep the runs still equal the oracle."""
    L, seed, T = 1008, 41, 2.3
    lat = ising.Lattice(L, seed, hot=True)
    try:
        lat.set_resident_tiles(48, 512, 3)
        lat.sweep(T, 8)
        lat.reset(seed, hot=True)
        lat.sweep(T, 5)
        s = oracle.init(L, seed, True)
        oracle.sweep(s, seed, 0, 5, T)
        assert (lat.spins() == s).all()
        check = lat.spins(), lat.t
        lat.sweep(T, 7)
        lat.set_spins(check[0])
        lat.t = check[1]
        lat.sweep(T, 4)
        oracle.sweep(s, seed, 5, 4, T)
        assert (lat.spins() == s).all() and lat.t == 9
    finally:
        lat.close()


def test_resident_tiles_expired_wait_is_reported_and_recoverable():
    """Failure path forced from the host: with the bound of every wait set to
    one tick (10 ns) the tiles' waits for their neighbours expire, the
    launches stop early (every wait is bounded, so they end), the error is
    reported once as ISING_EHIP, and after ising_reset with the default bound
    the lattice runs as the oracle again."""
    L, seed, T = 4096, 7, 2.269
    lat = ising.Lattice(L, seed, hot=True)
    try:
        assert lat.resident_tiles()[0] > 0
        lat.set_resident_wait(1)
        print("resident tiles with a one-tick wait bound", flush=True)
        lat.sweep(T, 40)
        with pytest.raises(ising.IsingError) as e:
            lat.synchronize()
        assert e.value.code == ising.ISING_EHIP and "waited too long" in ising.ising_last_error()
        lat.synchronize()  # reported once
        lat.set_resident_wait(0)
        lat.reset(seed, hot=True)
        E, M = lat.sweep_measure(T, 20, 10)
        got = lat.spins()
        got_E, got_M = E.cpu().numpy().tolist(), M.cpu().numpy().tolist()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 20, T, every=10)
    assert got_E == Es.tolist() and got_M == Ms.tolist()
    assert (got == s).all()
