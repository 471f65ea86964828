"""GPU parity of the batched form: every lattice of a mixed batch equals the
oracle (and therefore the same lattice run alone), for every execution plan
(resident in LDS, resident in global memory, half-sweep launches with 1/2/4
words per thread, multi-sweep LDS tiles, resident tiles, codes drawn
chip-wide, several chunk lengths), including sample series and sums."""
import numpy as np
import pytest

import oracle
import paper_1811_04384_amd as ising

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ising.load()


LS = [64, 42, 128, 256, 84, 512, 6, 1008]
SEEDS = [1234, 5, 6, 7, 8, 9, 10, 11]
HOT = [False, True, True, True, False, True, True, True]
TS = [1.5, 1.8, 2.1, 2.269, 2.5, 2.8, 3.1, 3.5]


def _reference(n1, n2, every):
    out = []
    for L, seed, hot, T in zip(LS, SEEDS, HOT, TS):
        s = oracle.init(L, seed, hot)
        oracle.sweep(s, seed, 0, n1, T)
        Es, Ms = oracle.sweep(s, seed, n1, n2, T, every=every)
        out.append((s, Es, Ms))
    return out


PLANS = [
    dict(resident_max_L=0, resident_block=256, words_per_thread=4, tiled_block=256, sweeps_per_graph=4),
    dict(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=3),
    dict(resident_max_L=256, resident_block=256, words_per_thread=2, tiled_block=128, sweeps_per_graph=5),
    dict(resident_max_L=1008, resident_block=1024, words_per_thread=4, tiled_block=256, sweeps_per_graph=2),
    dict(resident_max_L=128, resident_block=64, words_per_thread=1, tiled_block=256, sweeps_per_graph=50),
    # multi-sweep LDS tiles: every lattice (L = 6 whole, the others halo tiles)
    dict(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=4,
         tile_max_L=1008, tile_sweeps=2, tile_cols=16, tile_block=256),
    # resident, tiles and half-sweep launches in one chunk; chunks of 3 + 3
    dict(resident_max_L=64, resident_block=256, words_per_thread=2, tiled_block=128, sweeps_per_graph=7,
         tile_max_L=512, tile_sweeps=3, tile_cols=32, tile_block=512),
    # four sweeps per launch, whole-lattice tiles up to L = 64
    dict(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=8,
         tile_max_L=4096, tile_sweeps=4, tile_cols=64, tile_block=1024),
    # resident tiles trading boundary words: every lattice (L = 6, 42 whole)
    dict(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=4,
         tile_max_L=1008, tile_sweeps=1, tile_cols=48, tile_block=512, tile_exchange=1),
    # resident lattices, resident tiles (two-column bands) and half-sweep launches in one chunk
    dict(resident_max_L=64, resident_block=256, words_per_thread=2, tiled_block=128, sweeps_per_graph=6,
         tile_max_L=512, tile_sweeps=1, tile_cols=2, tile_block=64, tile_exchange=1),
    # codes drawn chip-wide for L <= 128 (draw passes of 4 + 3 sweeps), one
    # wavefront per apply workgroup (up to 8 words of a colour per thread
    # is too many for L = 128: it stays on k_small); the rest on half-sweep
    # launches
    dict(resident_max_L=128, resident_block=64, words_per_thread=1, tiled_block=64, sweeps_per_graph=7,
         draw_sweeps=4),
    # the same with four wavefronts per apply workgroup, beside k_small
    # (L = 256), resident tiles and half-sweep launches
    dict(resident_max_L=256, resident_block=256, words_per_thread=2, tiled_block=128, sweeps_per_graph=6,
         tile_max_L=512, tile_sweeps=1, tile_cols=32, tile_block=256, tile_exchange=1, draw_sweeps=3),
]


@pytest.mark.parametrize("plan", PLANS, ids=[f"plan{i}" for i in range(len(PLANS))])
def test_batch_matches_oracle(plan):
    n1, n2, every = 5, 6, 2
    ref = _reference(n1, n2, every)
    b = ising.Batch(LS, SEEDS, hot=HOT)
    try:
        b.set_plan(**plan)
        b.sweep(TS, n1)
        E, M = b.sweep(TS, n2, every=every, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        res = b.results()
        for i, (s, Es, Ms) in enumerate(ref):
            assert (b.spins(i) == s).all(), (i, LS[i])
            assert E[i].tolist() == Es.tolist() and M[i].tolist() == Ms.tolist(), i
            assert (res["E"][i], res["M"][i]) == oracle.observables(s)
            assert res["n_samples"][i] == n2 // every
            assert res["sum_E"][i] == Es.sum() and res["sum_absM"][i] == np.abs(Ms).sum()
            assert b.sweep_count(i) == n1 + n2
    finally:
        b.close()


@pytest.mark.parametrize("block", [64, 128, 256])
def test_drawn_codes_across_passes(block):
    """Codes drawn chip-wide: 40 sweeps per chunk in draw passes of 30 + 10
    (the apply kernel's codes run several sweeps ahead of their use, across
    its unrolled steps and the pass ends), samples every third sweep; then a
    second call that starts mid-way through the counter, sampling every
    sweep.  With 64 threads L = 128 has too many words per thread and stays
    on the in-workgroup path."""
    Ls, seeds, Ts = [128, 64, 84, 6, 4], [21, 22, 23, 24, 25], [2.0, 2.3, 2.6, 3.0, 1.7]
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=128, resident_block=block, words_per_thread=1, tiled_block=64, sweeps_per_graph=40,
                   draw_sweeps=30)
        E1, M1 = b.sweep(Ts, 40, every=3, series=True)
        E2, M2 = b.sweep(Ts, 17, every=1, series=True)
        E1, M1, E2, M2 = (x.cpu().numpy() for x in (E1, M1, E2, M2))
        for i, (L, seed, T) in enumerate(zip(Ls, seeds, Ts)):
            s = oracle.init(L, seed, True)
            Es1, Ms1 = oracle.sweep(s, seed, 0, 40, T, every=3)
            Es2, Ms2 = oracle.sweep(s, seed, 40, 17, T, every=1)
            assert E1[i].tolist() == Es1.tolist() and M1[i].tolist() == Ms1.tolist(), (i, L)
            assert E2[i].tolist() == Es2.tolist() and M2[i].tolist() == Ms2.tolist(), (i, L)
            assert (b.spins(i) == s).all(), (i, L)
    finally:
        b.close()


def test_drawn_codes_small_shapes():
    """Codes drawn chip-wide for the small shapes: two and four word rows,
    the row-(L-1) patch in either word row, L = 4 ... 84 in one batch;
    samples every second sweep over a pass boundary, then every sweep."""
    Ls = [4, 6, 20, 22, 42, 44, 62, 64, 84]
    seeds = list(range(60, 60 + len(Ls)))
    Ts = [1.6 + 0.2 * i for i in range(len(Ls))]
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=84, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=30,
                   draw_sweeps=12)
        E1, M1 = b.sweep(Ts, 30, every=2, series=True)
        E2, M2 = b.sweep(Ts, 11, every=1, series=True)
        E1, M1, E2, M2 = (x.cpu().numpy() for x in (E1, M1, E2, M2))
        res = b.results()
        for i, (L, seed, T) in enumerate(zip(Ls, seeds, Ts)):
            s = oracle.init(L, seed, True)
            Es1, Ms1 = oracle.sweep(s, seed, 0, 30, T, every=2)
            Es2, Ms2 = oracle.sweep(s, seed, 30, 11, T, every=1)
            assert E1[i].tolist() == Es1.tolist() and M1[i].tolist() == Ms1.tolist(), (i, L)
            assert E2[i].tolist() == Es2.tolist() and M2[i].tolist() == Ms2.tolist(), (i, L)
            assert (b.spins(i) == s).all(), (i, L)
            assert (res["E"][i], res["M"][i]) == oracle.observables(s)
    finally:
        b.close()


def test_drawn_codes_many_lattices():
    """More lattices than compute units: the apply workgroups share compute
    units with smaller LDS code buffers."""
    n = 300
    Ls = [(4, 6, 8, 10)[i % 4] for i in range(n)]
    seeds = list(range(100, 100 + n))
    Ts = [1.5 + 2.0 * (i % 11) / 10 for i in range(n)]
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=10, resident_block=64, words_per_thread=1, tiled_block=64, sweeps_per_graph=25,
                   draw_sweeps=25)
        E, M = b.sweep(Ts, 25, every=5, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        for i in range(0, n, 7):
            s = oracle.init(Ls[i], seeds[i], True)
            Es, Ms = oracle.sweep(s, seeds[i], 0, 25, Ts[i], every=5)
            assert E[i].tolist() == Es.tolist() and M[i].tolist() == Ms.tolist(), i
            assert (b.spins(i) == s).all(), i
    finally:
        b.close()


def test_batch_equals_lattices_alone():
    """Each lattice of a batch equals the plain single-lattice path."""
    Ls = [256, 512, 1024, 2048] * 2
    seeds = list(range(8))
    Ts = [1.5 + 2 * k / 7 for k in range(8)]
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.sweep(Ts, 9)
        for i, (L, seed, T) in enumerate(zip(Ls, seeds, Ts)):
            lat = ising.Lattice(L, seed, hot=True)
            lat.sweep(T, 9)
            assert (lat.spins() == b.spins(i)).all(), i
            lat.close()
    finally:
        b.close()


def test_graph_replays_and_reset_sums():
    """Replaying the same captured chunk many times (with eager work and
    synchronisation in between) keeps matching the oracle."""
    import torch

    Ls, seeds, Ts = [64, 128], [3, 4], [2.2, 2.7]
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=64, resident_block=128, words_per_thread=4, tiled_block=256, sweeps_per_graph=2)
        refs = [oracle.init(L, s, True) for L, s in zip(Ls, seeds)]
        t = 0
        for rep in range(6):
            b.sweep(Ts, 2, every=1)
            for r, s, T in zip(refs, seeds, Ts):
                oracle.sweep(r, s, t, 2, T)
            t += 2
            x = torch.ones(1000, device="cuda").sum()  # unrelated eager work between replays
            torch.cuda.synchronize()
            assert float(x) == 1000.0
            for i, r in enumerate(refs):
                assert (b.spins(i) == r).all(), (rep, i)
        res = b.results()
        assert res["n_samples"].tolist() == [12, 12]
        b.reset_sums()
        res = b.results()
        assert res["n_samples"].tolist() == [0, 0] and res["sum_E"].tolist() == [0, 0]
    finally:
        b.close()


def test_autotune_picks_a_plan_and_keeps_state(tmp_path):
    Ls = [64] * 8 + [256] * 4
    seeds = list(range(12))
    Ts = [2.0] * 12
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.sweep(Ts, 3)
        before = [b.spins(i) for i in range(len(Ls))]
        cache = str(tmp_path / "tune.json")
        plan = b.autotune(Ts, cache)
        assert plan["words_per_thread"] in (1, 2, 4)
        after = [b.spins(i) for i in range(len(Ls))]
        assert all((x == y).all() for x, y in zip(before, after))
        assert b.plan() == plan
        b.sweep(Ts, 4)
        for i, (L, seed) in enumerate(zip(Ls, seeds)):
            s = oracle.init(L, seed, True)
            oracle.sweep(s, seed, 0, 7, 2.0)
            assert (b.spins(i) == s).all()
        # the cached entry is used without timing
        b2 = ising.Batch(Ls, seeds, hot=True)
        assert b2.autotune(Ts, cache) == plan
        b2.close()
    finally:
        b.close()


def test_lattice_beyond_4gib_in_a_batch():
    """A batch holding a lattice larger than 4 GiB (L = 110000, N = 5240,
    4.6 GB, so the tiled kernel takes 64-bit word offsets) beside a small one,
    tiled, 2 sweeps with a sample: windows of the large lattice at its
    corners and seams (read with ising_batch_get_spins_region) and all of the
    small one equal the oracle; the window reader checks its arguments."""
    Ls, seeds, Ts, n = [110000, 130], [3, 4], [2.5, 2.0], 2
    N = oracle.word_rows(Ls[0])
    assert 8 * N * Ls[0] > 1 << 32
    print("batch with L=110000", flush=True)
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=2)
        b.sweep(Ts, n, every=n)
        res = b.results()
        L, seed, T = Ls[0], seeds[0], Ts[0]
        k, h, w = 2 * n + 1, 16, 16
        for (r, c) in [(L - 8, L - 8), (N - 8, 55000), (20 * N - 8, 3), (12345, 67890)]:
            r0, c0 = (r - k) % L, (c - k) % L
            win = oracle.init_window(L, seed, True, r0, c0, h + 2 * k, w + 2 * k)
            oracle.sweep_window(win, L, seed, 0, n, T, r0, c0)
            assert (b.region(0, r0 + k, c0 + k, h, w) == win[k:k + h, k:k + w]).all(), (r, c)
        s = oracle.init(Ls[1], seeds[1], True)
        oracle.sweep(s, seeds[1], 0, n, Ts[1])
        assert (b.spins(1) == s).all()
        assert (b.region(1, 0, 0, 130, 130) == s).all()
        assert (b.region(1, -3, 127, 5, 7) == np.roll(np.roll(s, 3, 0), -127, 1)[:5, :7]).all()
        assert (int(res["E"][1]), int(res["M"][1])) == oracle.observables(s)
        assert int(res["E"][0]) % 4 == 0 and int(res["M"][0]) % 2 == 0
        for bad in [(2, 0, 0, 1, 1), (0, 0, 0, 0, 4), (1, 0, 0, 131, 1)]:
            with pytest.raises(ising.IsingError):
                b.region(*bad)
    finally:
        b.close()


def test_batch_tiles_sample_every_sweep():
    """Multi-sweep tiles with a sample after every sweep (several samples per
    launch, in order) and chunks that are not a multiple of the sweeps per
    launch: series, sums and states equal the oracle's."""
    Ls = [1008, 1008, 130, 42, 2016]
    seeds = [3, 4, 5, 6, 7]
    Ts = [2.2, 2.4, 2.6, 1.9, 2.269]
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=10,
                   tile_max_L=2016, tile_sweeps=4, tile_cols=32, tile_block=512)
        E, M = b.sweep(Ts, 13, every=1, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        res = b.results()
        for i, (L, seed, T) in enumerate(zip(Ls, seeds, Ts)):
            s = oracle.init(L, seed, True)
            Es, Ms = oracle.sweep(s, seed, 0, 13, T, every=1)
            assert E[i].tolist() == Es.tolist() and M[i].tolist() == Ms.tolist(), i
            assert (b.spins(i) == s).all(), i
            assert res["n_samples"][i] == 13 and res["sum_E"][i] == Es.sum()
    finally:
        b.close()


def test_batch_resident_tiles_sample_every_sweep():
    """Resident tiles with a sample after every sweep (many samples per
    launch, in order): series, sums and states equal the oracle's."""
    Ls = [1008, 1008, 130, 42, 2016]
    seeds = [3, 4, 5, 6, 7]
    Ts = [2.2, 2.4, 2.6, 1.9, 2.269]
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=10,
                   tile_max_L=2016, tile_sweeps=1, tile_cols=32, tile_block=512, tile_exchange=1)
        E, M = b.sweep(Ts, 13, every=1, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        res = b.results()
        for i, (L, seed, T) in enumerate(zip(Ls, seeds, Ts)):
            s = oracle.init(L, seed, True)
            Es, Ms = oracle.sweep(s, seed, 0, 13, T, every=1)
            assert E[i].tolist() == Es.tolist() and M[i].tolist() == Ms.tolist(), i
            assert (b.spins(i) == s).all(), i
            assert res["n_samples"][i] == 13 and res["sum_E"][i] == Es.sum()
    finally:
        b.close()
