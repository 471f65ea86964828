"""GPU parity of the batched form: every lattice of a mixed batch equals the
oracle (and therefore the same lattice run alone), for every execution plan
(resident in LDS, resident in global memory, tiled with 1/2/4 words per
thread, several chunk lengths), including sample series and sums."""
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
