"""GPU parity of replica multi-spin coding: the 21 replicas' states, E/M
series, observables and moment sums equal the oracle's bit for bit for
several sizes (incl. the smallest, ragged segments and the bench size),
temperature sets and start kinds, for every kernel plan; argument checks."""
import numpy as np
import pytest

import oracle
import paper_1811_04384_amd as ising

pytestmark = pytest.mark.gpu

TS = [1.5 + 0.1 * k for k in range(21)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ising.load()


@pytest.mark.parametrize("L,seed,hot,n,every", [
    (4, 3, True, 7, 1),      # smallest lattice: one segment per row
    (6, 4, False, 5, 1),     # 3 same-colour words per row: ragged segments
    (64, 5, True, 9, 3),
    (130, 6, True, 6, 2),    # 65 same-colour words per row
    (1024, 7, False, 4, 2),
])
def test_replicas_match_oracle(L, seed, hot, n, every):
    print(f"replicas L={L} seed={seed}", flush=True)
    T = [TS[(k * 7) % 21] for k in range(21)]  # not monotone in k
    rep = ising.Replicas(L, seed, hot=hot)
    rep.sweep(T, 2)
    E, M = rep.sweep_measure(T, n, every)
    s = oracle.replica_init(L, seed, hot)
    oracle.replica_sweep(s, seed, 0, 2, T)
    Es, Ms = oracle.replica_sweep(s, seed, 2, n, T, every=every)
    assert np.array_equal(E.cpu().numpy(), Es) and np.array_equal(M.cpu().numpy(), Ms)
    for k in range(21):
        assert np.array_equal(rep.spins(k), s[k]), k
    Eo, Mo = rep.observables()
    assert list(Eo) == [oracle.observables(s[k])[0] for k in range(21)]
    assert list(Mo) == [oracle.observables(s[k])[1] for k in range(21)]
    assert rep.t == 2 + n
    rep.close()


@pytest.mark.parametrize("wpt", [1, 2, 4])
def test_every_plan_gives_identical_results(wpt):
    L, seed = 90, 11
    rep = ising.Replicas(L, seed, hot=True)
    rep.set_plan(wpt)
    rep.sweep(TS, 6)
    s = oracle.replica_init(L, seed, True)
    oracle.replica_sweep(s, seed, 0, 6, TS)
    for k in (0, 5, 19, 20):
        assert np.array_equal(rep.spins(k), s[k]), (wpt, k)
    rep.close()


def test_replica_moments_and_bench_size():
    L, seed = 8192, 21
    rep = ising.Replicas(L, seed, hot=True)
    acc = rep.sweep_moments(TS, 2, 1)
    got = rep.moments(acc)
    print("oracle: 21 replicas of L=8192, 2 sweeps", flush=True)
    s = oracle.replica_init(L, seed, True)
    Es, Ms = oracle.replica_sweep(s, seed, 0, 2, TS, every=1)
    for k in range(21):
        assert got[k] == oracle.moments(Es[:, k], Ms[:, k]), k
    for k in (0, 20):
        assert np.array_equal(rep.spins(k), s[k]), k
    rep.close()


def test_invalid_replica_arguments():
    for L in (2, 5, 65538):
        with pytest.raises(ising.IsingError):
            ising.Replicas(L, 1)
    rep = ising.Replicas(16, 1)
    bad = list(TS)
    bad[4] = float("inf")
    with pytest.raises(ising.IsingError):
        rep.sweep(bad, 1)
    with pytest.raises(ising.IsingError):
        rep.set_plan(3)
    with pytest.raises(ising.IsingError):
        ising.ising_replicas_get_spins(rep.handle, 21, 16)
    assert rep.t == 0
    rep.close()
