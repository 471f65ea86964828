"""GPU parity of the temperature scan and the moment sums: heating and
cooling scans of one lattice (plain path), moments accumulated across calls,
and scans of a whole batch under every kind of plan, all bit-exact against
the oracle's scan (the sums are exact integers on both sides); plus the
specific heat of a GPU heating scan against Kaufman's exact values."""
import math

import numpy as np
import pytest

import oracle
import paper_1811_04384_amd as ising
from exact_ising import kaufman_energy, kaufman_specific_heat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ising.load()


@pytest.mark.parametrize("L,seed,hot,Ts,therm,meas,every", [
    (64, 5, True, [1.5, 2.0, 2.269, 2.6, 3.5], 30, 120, 1),   # heating, 16 live rows per word
    (130, 9, False, [3.0, 2.4, 1.9], 7, 60, 3),               # cooling, ragged word rows, dead slots
    (1008, 21, True, [2.2, 2.35], 4, 10, 2),                  # L = 21 N: the paper's layout
])
def test_single_scan_matches_oracle(L, seed, hot, Ts, therm, meas, every):
    print(f"scan L={L} seed={seed} Ts={Ts}", flush=True)
    lat = ising.Lattice(L, seed, hot=hot)
    got = lat.scan(Ts, therm, meas, every)
    want, s, t = oracle.scan(L, seed, hot, Ts, therm, meas, every)
    assert got == want
    assert lat.t == t
    assert np.array_equal(lat.spins(), s)
    lat.close()


def test_scan_of_large_lattice_matches_oracle():
    L, seed, Ts = 4096, 7, [2.269, 2.4]
    print(f"scan L={L}", flush=True)
    lat = ising.Lattice(L, seed, hot=True)
    got = lat.scan(Ts, 3, 6, 2)
    want, s, t = oracle.scan(L, seed, True, Ts, 3, 6, 2)
    assert got == want and lat.t == t
    assert np.array_equal(lat.spins(), s)
    lat.close()


def test_sweep_moments_accumulates_across_calls():
    L, seed, T = 96, 3, 2.3
    lat = ising.Lattice(L, seed, hot=True)
    acc = lat.sweep_moments(T, 20, 4)
    lat.sweep(T, 5)
    lat.sweep_moments(T, 18, 3, acc)
    got = ising.moments_of(acc)
    s = oracle.init(L, seed, True)
    E1, M1 = oracle.sweep(s, seed, 0, 20, T, 4)
    oracle.sweep(s, seed, 20, 5, T)
    E2, M2 = oracle.sweep(s, seed, 25, 18, T, 3)
    assert got == oracle.moments(list(E1) + list(E2), list(M1) + list(M2))
    lat.close()


def test_scan_edge_cases():
    lat = ising.Lattice(20, 1, hot=True)
    assert lat.scan([], 5, 5, 1) == []
    got = lat.scan([2.0, 3.0], 4, 2, 3)  # fewer measurement sweeps than `every`: no samples
    assert all(m["n_samples"] == 0 for m in got) and lat.t == 12
    with pytest.raises(ising.IsingError):
        lat.scan([2.0, -1.0], 1, 1, 1)
    with pytest.raises(ising.IsingError):
        lat.scan([2.0], 1, 1, 0)
    assert lat.t == 12  # rejected calls did no work
    lat.close()


BATCH_LS = [64, 42, 128, 256, 84, 130, 6, 1008]
BATCH_SEEDS = [11, 12, 13, 14, 15, 16, 17, 18]
PLANS = [
    dict(resident_max_L=0, resident_block=256, words_per_thread=2, tiled_block=128, sweeps_per_graph=4),
    dict(resident_max_L=256, resident_block=256, words_per_thread=1, tiled_block=256, sweeps_per_graph=6),
    dict(resident_max_L=1008, resident_block=1024, words_per_thread=4, tiled_block=64, sweeps_per_graph=50),
    dict(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=6,
         tile_max_L=1008, tile_sweeps=2, tile_cols=16, tile_block=256),
    dict(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=6,
         tile_max_L=1008, tile_sweeps=1, tile_cols=16, tile_block=256, tile_exchange=1),
    dict(resident_max_L=130, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=6,
         draw_sweeps=4),
]


@pytest.mark.parametrize("plan", PLANS, ids=["tiled", "resident_lds", "resident_all", "lds_tiles", "resident_tiles",
                                             "drawn_codes"])
def test_batch_scan_matches_oracle(plan):
    print(f"batch scan plan={plan}", flush=True)
    n = len(BATCH_LS)
    Tmat = np.array([[1.6 + 0.1 * i + 0.4 * j for i in range(n)] for j in range(3)])  # heating per lattice
    b = ising.Batch(BATCH_LS, BATCH_SEEDS, hot=True)
    b.set_plan(**plan)
    got = b.scan(Tmat, 5, 12, 2)
    for i, (L, seed) in enumerate(zip(BATCH_LS, BATCH_SEEDS)):
        want, s, t = oracle.scan(L, seed, True, list(Tmat[:, i]), 5, 12, 2)
        assert [got[j][i] for j in range(3)] == want, (i, L)
        assert np.array_equal(b.spins(i), s) and b.sweep_count(i) == t
    # the running sums hold the last step's samples, as the moments do
    res = b.results()
    last = b.moments()
    for i in range(n):
        assert last[i] == got[2][i]
        assert res["sum_E"][i] == last[i]["sum_E"] and res["n_samples"][i] == last[i]["n_samples"]
    b.close()


def test_heating_workload_plan_matches_oracle():
    """The heating workload's shape and plan as the benchmark runs it: 16 x
    L = 1008, cold, seeds 0..15, resident tiles of 64 columns on 1024
    threads, 200 sweeps per chunk, carried over two temperatures with 40
    unsampled and 220 sampled sweeps each (so a chunk boundary falls inside
    the sampled run): every lattice's moment sums, state and sweep count
    equal the oracle's (about 10 s of oracle work)."""
    Ts = [1.5, 2.3]
    n = 16
    b = ising.Batch([1008] * n, list(range(n)), hot=False)
    try:
        b.set_plan(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=200,
                   tile_max_L=1008, tile_sweeps=1, tile_cols=64, tile_block=1024, tile_exchange=1)
        print("heating workload plan, 16 x L=1008", flush=True)
        got = b.scan(Ts, 40, 220, 1)
        for i in range(n):
            want, s, t = oracle.scan(1008, i, False, Ts, 40, 220, 1)
            assert [got[j][i] for j in range(2)] == want, i
            assert np.array_equal(b.spins(i), s) and b.sweep_count(i) == t
    finally:
        b.close()


def test_gpu_heating_scan_specific_heat_matches_kaufman():
    """Eight replicas of a 32 x 32 torus heated through the transition on the
    GPU: the replica-averaged energy and specific heat per spin at each
    temperature against Kaufman's exact finite-lattice values (errors from
    the spread over replicas)."""
    L, R = 32, 8
    Ts = [1.8, 2.2, 2.35, 2.6, 3.2]
    b = ising.Batch([L] * R, list(range(100, 100 + R)), hot=False)
    out = b.scan(Ts, 3000, 40_000, 1)
    b.close()
    for j, T in enumerate(Ts):
        th = [ising.ising_thermodynamics(out[j][r], L, T) for r in range(R)]
        for key, exact in (("e", kaufman_energy(L, T)), ("c", kaufman_specific_heat(L, T))):
            vals = np.array([x[key] for x in th])
            err = vals.std(ddof=1) / math.sqrt(R)
            assert abs(vals.mean() - exact) < 5 * err + 1e-3 * abs(exact), (T, key, vals.mean(), exact, err)


def test_paper_scan_energy_matches_kaufman():
    """The paper's driver loop on its demonstration lattice (N = 4, L = 84):
    T = 0.001, 0.101, ..., 10.001 with the lattice carried over, at each T
    400 iterations of 10 updates per spin with the energy recorded after each
    iteration and every iteration averaged (nothing discarded).  Eight
    replicas from a cold start; the replica-mean energy per spin at each of
    the 101 temperatures against Kaufman's exact value for the 84 x 84 torus.
    Near T_c the 4000-sweep averages carry a larger error, which the spread
    over replicas measures."""
    L, R = 84, 8
    Ts = [0.001 + 0.1 * k for k in range(101)]
    b = ising.Batch([L] * R, list(range(R)), hot=False)
    out = b.scan(Ts, 0, 4000, 10)
    b.close()
    worst = 0.0
    for j, T in enumerate(Ts):
        assert all(out[j][r]["n_samples"] == 400 for r in range(R))
        e = np.array([out[j][r]["sum_E"] / 400 / L ** 2 for r in range(R)])
        err = e.std(ddof=1) / math.sqrt(R)
        exact = kaufman_energy(L, T)
        assert abs(e.mean() - exact) < 5 * err + 2e-3, (T, e.mean(), exact, err)
        worst = max(worst, abs(e.mean() - exact))
    print(f"largest |e - e_exact| over 101 temperatures: {worst:.2e}", flush=True)
