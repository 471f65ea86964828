"""GPU parity of the multi-sweep LDS tile path (several sweeps per launch on
tiles of word columns with redundant halos, or the whole lattice in one
workgroup) against the CPU oracle.

Bit-exact: the spin state after every call and every sampled E, M equal
the oracle's on the same seeds.  The cases cover: the whole lattice in one
workgroup (tiny and LDS-sized lattices, up to 16 sweeps and 16 samples per
launch), halo tiles with 1 to 8 sweeps per launch, ragged last tiles, L not
a multiple of 8 (position-20 groups split where the tile wraps past the
lattice's end) or of 21 (the row-(L-1) patch), the paper's L = 21 N
lattices, dead slots, sample counts that do not divide the sweeps per
launch, workgroups of 64 to 1024 threads, and more tiles in one launch than
the chip runs at once.
"""
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


CALLS = [(2.269, 7, 0), (1.5, 10, 3), (3.5, 5, 1), (2.6, 9, 2)]

# (L, seed, hot, sweeps per launch, tile columns, block)
CASES = [
    (4, 3, True, 2, 4, 64),
    (6, 5, False, 3, 6, 64),
    (42, 7, True, 1, 8, 128),
    (42, 8, True, 4, 10, 256),
    (64, 1234, False, 16, 64, 256),
    (84, 9, True, 2, 14, 128),
    (128, 2, True, 3, 20, 192),
    (130, 11, True, 2, 16, 256),
    (256, 13, True, 8, 256, 1024),
    (1006, 4, True, 2, 48, 512),
    (1008, 21, True, 2, 48, 512),
    (1008, 23, False, 4, 64, 1024),
    (2016, 22, True, 3, 96, 1024),
]


def _check(L, seed, hot, lat):
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


@pytest.mark.parametrize("L,seed,hot,K,cols,block", CASES)
def test_tiles_match_oracle(L, seed, hot, K, cols, block):
    print(f"tiles L={L} K={K} cols={cols} block={block}", flush=True)
    lat = ising.Lattice(L, seed, hot=hot)
    try:
        lat.set_tiling(K, cols, block)
        assert lat.tiling() == (K, min(cols, L) if cols < L else L, block)
        _check(L, seed, hot, lat)
    finally:
        lat.close()


def test_tiles_moments_and_mixed_with_half_sweep_launches():
    """Tile launches and half-sweep launches on one sweep counter: moments
    accumulate across both paths."""
    L, seed, T = 1008, 31, 2.4
    lat = ising.Lattice(L, seed, hot=True)
    try:
        lat.set_tiling(2, 64, 512)
        acc = lat.sweep_moments(T, 6, 1)
        lat.set_tiling(0)
        lat.sweep_moments(T, 5, 1, acc)
        lat.set_tiling(3, 96, 1024)
        lat.sweep_moments(T, 7, 1, acc)
        m = ising.moments_of(acc)
        spins = lat.spins()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 18, T, every=1)
    assert m == oracle.moments(Es, Ms)
    assert (spins == s).all()


def test_tiles_l4096_prefix_matches_oracle():
    """The plain workload's lattice (L = 4096, hot start seed 7, T = 2.269)
    with 16-column tiles, two sweeps per launch, E/M every 10 sweeps, over
    30 sweeps: the series and the state equal the oracle's."""
    L, seed, T = 4096, 7, 2.269
    lat = ising.Lattice(L, seed, hot=True)
    try:
        lat.set_tiling(2, 16, 1024)
        E, M = lat.sweep_measure(T, 30, 10)
        got = lat.spins()
        got_E, got_M = E.cpu().numpy().tolist(), M.cpu().numpy().tolist()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 30, T, every=10)
    assert got_E == Es.tolist() and got_M == Ms.tolist()
    assert (got == s).all()


def test_tiles_more_than_fit_at_once_match_oracle():
    """2048 two-column tiles of L = 4096 in one launch: more workgroups than
    the chip holds at once, so tiles of a later round load their halos after
    their neighbours have stored their interiors (the halos come from the
    copy taken ahead of the launch)."""
    L, seed, T = 4096, 19, 2.269
    lat = ising.Lattice(L, seed, hot=True)
    try:
        lat.set_tiling(1, 2, 64)
        E, M = lat.sweep_measure(T, 6, 2)
        got = lat.spins()
        got_E, got_M = E.cpu().numpy().tolist(), M.cpu().numpy().tolist()
    finally:
        lat.close()
    s = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(s, seed, 0, 6, T, every=2)
    assert got_E == Es.tolist() and got_M == Ms.tolist()
    assert (got == s).all()


def test_invalid_tilings_are_rejected():
    lat = ising.Lattice(64, 1, hot=True)
    try:
        for bad in ((17, 8, 256), (-1, 8, 256), (2, 7, 256), (2, 0, 256), (2, 60, 256), (2, 8, 96), (2, 8, 2048)):
            with pytest.raises(ising.IsingError) as e:
                lat.set_tiling(*bad)
            assert e.value.code == ising.ISING_EINVAL
        assert lat.tiling() == (0, 0, 0)
    finally:
        lat.close()
    big = ising.Lattice(32768, 1, hot=False)
    try:
        with pytest.raises(ising.IsingError):
            big.set_tiling(2, 64, 256)  # 1562 word rows: a tile does not fit in LDS
    finally:
        big.close()
