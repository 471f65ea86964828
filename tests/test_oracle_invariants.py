"""Invariants and special cases of the oracle: energy closed forms, the
energy change of a single flip (Table 1), global spin-flip symmetry,
splitting sweeps, thread-count independence and exact windows."""
import numpy as np
import pytest

import oracle


@pytest.mark.parametrize("L", [4, 6, 42, 64])
def test_energy_closed_forms(L):
    n = L * L
    up = np.ones((L, L), np.uint8)
    assert oracle.observables(up) == (-2 * n, n)
    assert oracle.observables(1 - up) == (-2 * n, -n)
    rr, cc = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    neel = ((rr + cc) % 2).astype(np.uint8)
    assert oracle.observables(neel) == (2 * n, 0)
    # vertical stripes of width 1: every horizontal bond antiparallel, every vertical one aligned
    stripes = (cc % 2).astype(np.uint8)
    assert oracle.observables(stripes) == (0, 0)
    # one flipped spin in the aligned state raises E by 8 (Table 1, dE = +8J)
    one = up.copy()
    one[L // 2, 1] = 0
    assert oracle.observables(one) == (-2 * n + 8, n - 2)


def test_energy_parity_and_single_flip_changes():
    rng = np.random.default_rng(3)
    for L in (4, 10, 64):
        s = rng.integers(0, 2, (L, L)).astype(np.uint8)
        E, M = oracle.observables(s)
        assert E % 4 == 0 and M % 2 == 0
        for _ in range(20):
            r, c = rng.integers(0, L, 2)
            sig = 1 if s[r, c] else -1
            nb = sum(1 if s[(r + dr) % L, (c + dc) % L] else -1 for dr, dc in ((1, 0), (-1, 0), (0, 1), (0, -1)))
            s2 = s.copy()
            s2[r, c] ^= 1
            E2, M2 = oracle.observables(s2)
            assert E2 - E == 2 * sig * nb  # dE of Table 1
            assert M2 - M == -2 * sig


def test_global_flip_symmetry():
    """Counts of antiparallel neighbours are invariant under flipping every
    spin, and the draws do not depend on the state: the complemented start
    follows exactly the complemented trajectory."""
    L, seed, T = 64, 31, 2.3
    a = oracle.init(L, seed, hot=True)
    b = (1 - a).astype(np.uint8)
    Ea, Ma = oracle.sweep(a, seed, 0, 30, T, every=3, threads=2)
    Eb, Mb = oracle.sweep(b, seed, 0, 30, T, every=3, threads=3)
    assert (a == 1 - b).all()
    assert (Ea == Eb).all() and (Ma == -Mb).all()


def test_sweep_split_and_temperature_change():
    L, seed = 42, 8
    a = oracle.init(L, seed, hot=True)
    b = a.copy()
    oracle.sweep(a, seed, 0, 25, 2.4)
    oracle.sweep(b, seed, 0, 10, 2.4)
    oracle.sweep(b, seed, 10, 15, 2.4)
    assert (a == b).all()
    oracle.sweep(a, seed, 25, 5, 1.7)
    c = b.copy()
    oracle.sweep(b, seed, 25, 5, 1.7)
    assert (a == b).all()
    oracle.sweep(c, seed, 26, 5, 1.7)  # a different sweep index gives a different chain
    assert not (c == b).all()


def test_thread_count_does_not_change_results():
    L, seed = 128, 4
    ref = oracle.init(L, seed, hot=True)
    oracle.sweep(ref, seed, 0, 12, 2.269, threads=1)
    for th in (2, 5, 8):
        s = oracle.init(L, seed, hot=True)
        oracle.sweep(s, seed, 0, 12, 2.269, threads=th)
        assert (s == ref).all()


def test_hot_start_statistics():
    s = oracle.init(1008, 7, hot=True)
    frac = s.mean()
    assert abs(frac - 0.5) < 5 * 0.5 / 1008
    assert oracle.init(64, 7, hot=True).tolist() == oracle.init(64, 7, hot=True).tolist()
    assert not (oracle.init(64, 7, hot=True) == oracle.init(64, 8, hot=True)).all()


@pytest.mark.parametrize("L,r0,c0,h,w,n", [(64, 10, 20, 30, 26, 3), (42, 35, 30, 24, 30, 4), (128, 120, 3, 40, 40, 5)])
def test_window_evolution_is_exact(L, r0, c0, h, w, n):
    seed, T = 12, 2.2
    full = oracle.init(L, seed, hot=True)
    win = oracle.init_window(L, seed, True, r0, c0, h, w)
    rows = [(r0 + i) % L for i in range(h)]
    cols = [(c0 + j) % L for j in range(w)]
    assert (win == full[np.ix_(rows, cols)]).all()
    oracle.sweep(full, seed, 5, n, T)
    oracle.sweep_window(win, L, seed, 5, n, T, r0, c0)
    k = 2 * n
    sub = full[np.ix_(rows, cols)]
    assert (win[k:h - k, k:w - k] == sub[k:h - k, k:w - k]).all()


def test_invalid_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.init(5, 1, True)
    with pytest.raises(ValueError):
        oracle.init(2, 1, True)
    s = oracle.init(8, 1, True)
    with pytest.raises(ValueError):
        oracle.sweep(s, 1, 0, 1, 0.0)
    with pytest.raises(ValueError):
        oracle.sweep(s, 1, 0, 1, float("inf"))
