"""Seeded random mixes of lattices and execution plans (32 cases), each lattice's series,
state and sums against the oracle: every plan kind of the batch engine (half-
sweep launches, one workgroup per lattice, halo tiles, resident tiles, codes
drawn chip-wide) combined at random with lattice sizes (L not a multiple of
21, one or several word rows of each colour), chunk lengths, draw-pass
lengths and sampling intervals, over two calls that continue one counter."""
import random

import numpy as np
import pytest

import oracle
import paper_1811_04384_amd as ising

pytestmark = pytest.mark.gpu

SIZES = [4, 6, 8, 14, 20, 22, 30, 42, 44, 62, 64, 84, 86, 100, 126, 128, 130, 168, 200, 256, 512, 1010]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ising.load()


def _random_plan(rng, Ls):
    Lmax = max(Ls)
    p = dict(resident_max_L=rng.choice([0, 16, 64, 130, Lmax]), resident_block=rng.choice([64, 128, 256, 512]),
             words_per_thread=rng.choice([1, 2, 4]), tiled_block=rng.choice([64, 128, 256]),
             sweeps_per_graph=rng.randint(1, 9), draw_sweeps=rng.choice([0, 0, 1, 3, 8]))
    kind = rng.choice(["none", "halo", "resident"])
    if kind != "none":
        p.update(tile_max_L=rng.choice([Lmax, 128]), tile_cols=rng.choice([2, 8, 16, 22, 32, 64]),
                 tile_block=rng.choice([64, 128, 256, 512, 1024]))
        if kind == "halo":
            p.update(tile_sweeps=rng.randint(1, 4), tile_exchange=0)
        else:
            p.update(tile_sweeps=1, tile_exchange=1)
    return p


@pytest.mark.parametrize("case", range(32))
def test_random_plan_mix_matches_oracle(case):
    rng = random.Random(1000 + case)
    n = rng.randint(2, 6)
    Ls = [rng.choice(SIZES) for _ in range(n)]
    seeds = [rng.randint(0, 2 ** 40) for _ in range(n)]
    hot = [rng.random() < 0.7 for _ in range(n)]
    Ts = [round(rng.uniform(1.2, 4.0), 3) for _ in range(n)]
    plan = _random_plan(rng, Ls)
    n1, n2 = rng.randint(1, 9), rng.randint(1, 9)
    every = rng.randint(1, 3)
    n2 = max(n2, every)
    print(f"case {case}: L={Ls} plan={plan} n1={n1} n2={n2} every={every}", flush=True)
    b = ising.Batch(Ls, seeds, hot=hot)
    try:
        b.set_plan(**plan)
        b.sweep(Ts, n1)
        E, M = b.sweep(Ts, n2, every=every, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        res = b.results()
        for i, (L, seed, h, T) in enumerate(zip(Ls, seeds, hot, Ts)):
            s = oracle.init(L, seed, h)
            oracle.sweep(s, seed, 0, n1, T)
            Es, Ms = oracle.sweep(s, seed, n1, n2, T, every=every)
            assert E[i].tolist() == Es.tolist() and M[i].tolist() == Ms.tolist(), (i, L)
            assert (b.spins(i) == s).all(), (i, L)
            assert (res["E"][i], res["M"][i]) == oracle.observables(s), (i, L)
            assert res["n_samples"][i] == n2 // every, (i, L)
            assert res["sum_E"][i] == Es.sum() and res["sum_absM"][i] == np.abs(Ms).sum(), (i, L)
            assert b.sweep_count(i) == n1 + n2
    finally:
        b.close()
