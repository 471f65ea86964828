"""GPU parity at the benchmark workloads' full shapes.

- The L = 64 temperature scan: 8 lattices, cold start, seed 1234, 2000 + 2000
  sweeps with a sample after every measured sweep -- every sample of every
  lattice and the final states equal the oracle's (the whole run).
- The 2048-lattice mixed batch: the E/M samples of every one of the 2048
  lattices after the first sweep and after 10 sweeps equal the oracle's, and
  64 sampled lattices (16 of each size) equal it site by site after 10
  sweeps, under two plans (all 2048 under one); over the full 5000 sweeps
  with a sample every 10, four lattices of each size are followed: L = 256
  and 512 over all 500 samples and the final state, L = 1024 and 2048 over
  the first 50 samples (their full oracle run would take minutes); four
  L = 256 lattices stay equal over 500 sweeps.
- The L = 32768 single lattice over 20 sweeps on oracle-evolved windows, and
  the whole L = 32768 lattice of the headline workload (hot start, seed 11,
  T = 2.269, the benchmark's launch configuration) after 2 sweeps: every
  sampled E and M (Section 5.3's bond energy) and every one of its 1.07e9
  spins equal a full oracle run.
"""
import time

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


@pytest.mark.parametrize("draw_sweeps", [0, 500], ids=["in_workgroup", "drawn_chip_wide"])
def test_scan_l64_full_run_matches_oracle(draw_sweeps):
    Ts = [1.5 + 2.0 * i / 7 for i in range(8)]
    b = ising.Batch([64] * 8, [1234] * 8, hot=False)
    try:
        b.set_plan(resident_max_L=64, resident_block=64 if draw_sweeps == 0 else 256, words_per_thread=1,
                   tiled_block=256, sweeps_per_graph=500, draw_sweeps=draw_sweeps)
        b.sweep(Ts, 2000)
        E, M = b.sweep(Ts, 2000, every=1, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        res = b.results()
        for i, T in enumerate(Ts):
            s = oracle.init(64, 1234, False)
            oracle.sweep(s, 1234, 0, 2000, T, threads=1)
            Es, Ms = oracle.sweep(s, 1234, 2000, 2000, T, every=1, threads=1)
            assert (E[i] == Es).all() and (M[i] == Ms).all(), T
            assert (b.spins(i) == s).all()
            assert res["sum_E"][i] == Es.sum() and res["sum_absM"][i] == np.abs(Ms).sum()
    finally:
        b.close()


def _batched_config():
    Ls = [(256, 512, 1024, 2048)[i % 4] for i in range(2048)]
    Ts = [1.5 + 2.0 * ((i // 4) % 32) / 31 for i in range(2048)]
    return Ls, Ts, list(range(2048))


@pytest.mark.parametrize("plan", [
    dict(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=128, sweeps_per_graph=10),
    dict(resident_max_L=512, resident_block=512, words_per_thread=2, tiled_block=256, sweeps_per_graph=5),
], ids=["tiled", "mixed"])
def test_batched_config_sampled_lattices(plan):
    Ls, Ts, seeds = _batched_config()
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(**plan)
        E1, M1 = b.sweep(Ts, 1, every=1, series=True)
        E1, M1 = E1.cpu().numpy(), M1.cpu().numpy()
        E, M = b.sweep(Ts, 9, every=9, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        rng = np.random.default_rng(4)
        picks = []
        for size_class in range(4):
            idx = [i for i in range(2048) if i % 4 == size_class]
            picks += list(rng.choice(idx, 16, replace=False))
        for i in picks:
            s = oracle.init(Ls[i], seeds[i], True)
            Es, Ms = oracle.sweep(s, seeds[i], 0, 1, Ts[i], every=1)
            assert E1[i, 0] == Es[0] and M1[i, 0] == Ms[0]
            Es, Ms = oracle.sweep(s, seeds[i], 1, 9, Ts[i], every=9)
            assert (b.spins(int(i)) == s).all(), (i, Ls[i])
            assert E[i, 0] == Es[0] and M[i, 0] == Ms[0]
        if plan["resident_max_L"]:  # once: the samples of every lattice
            t0 = time.time()
            for i in range(2048):
                if i % 256 == 0:
                    print(f"oracle: all 2048 lattices, 10 sweeps: {i} done, {time.time() - t0:.0f} s", flush=True)
                s = oracle.init(Ls[i], seeds[i], True)
                Es, Ms = oracle.sweep(s, seeds[i], 0, 1, Ts[i], every=1)
                assert E1[i, 0] == Es[0] and M1[i, 0] == Ms[0], (i, Ls[i])
                Es, Ms = oracle.sweep(s, seeds[i], 1, 9, Ts[i], every=9)
                assert E[i, 0] == Es[0] and M[i, 0] == Ms[0], (i, Ls[i])
    finally:
        b.close()


def test_batched_config_full_run_sampled_lattices():
    Ls, Ts, seeds = _batched_config()
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.set_plan(resident_max_L=512, resident_block=512, words_per_thread=1, tiled_block=128, sweeps_per_graph=50)
        E, M = b.sweep(Ts, 5000, every=10, series=True)
        E, M = E.cpu().numpy(), M.cpu().numpy()
        rng = np.random.default_rng(5)
        for size_class in range(4):
            idx = [i for i in range(2048) if i % 4 == size_class]
            for i in rng.choice(idx, 4, replace=False):
                i = int(i)
                L = Ls[i]
                n = 5000 if L <= 512 else 500
                print(f"oracle: lattice {i} L={L} {n} sweeps", flush=True)
                s = oracle.init(L, seeds[i], True)
                Es, Ms = oracle.sweep(s, seeds[i], 0, n, Ts[i], every=10)
                assert (E[i, : n // 10] == Es).all() and (M[i, : n // 10] == Ms).all(), (i, L)
                if n == 5000:
                    assert (b.spins(i) == s).all(), (i, L)
    finally:
        b.close()


def test_batched_l256_lattices_500_sweeps():
    Ls, Ts, seeds = _batched_config()
    b = ising.Batch(Ls, seeds, hot=True)
    try:
        b.sweep(Ts, 500, every=50)
        for i in (0, 4, 128, 2044):
            s = oracle.init(Ls[i], seeds[i], True)
            oracle.sweep(s, seeds[i], 0, 500, Ts[i])
            assert Ls[i] == 256
            assert (b.spins(i) == s).all(), i
    finally:
        b.close()


def test_l32768_twenty_sweeps_on_windows():
    L, seed, T, n = 32768, 11, 2.6, 20
    N = oracle.word_rows(L)
    lat = ising.Lattice(L, seed, hot=True)
    try:
        lat.sweep(T, n)
        k = 2 * n + 1
        h = w = 16
        for (r, c) in [(0, 0), (L - 8, 7), (N - 8, L - 8), (20 * N - 8, 16384), (31000, 123)]:
            r0, c0 = (r - k) % L, (c - k) % L
            win = oracle.init_window(L, seed, True, r0, c0, h + 2 * k, w + 2 * k)
            oracle.sweep_window(win, L, seed, 0, n, T, r0, c0)
            assert (lat.region(r0 + k, c0 + k, h, w) == win[k:k + h, k:k + w]).all(), (r, c)
    finally:
        lat.close()


def test_server_zero_sweep_and_cold_requests():
    srv = ising.Server(hbm_budget=1 << 24, max_slots=4, quantum_sweeps=3)
    try:
        srv.submit(1, 64, 2.0, 0)            # nothing to do: the initial state's E, M
        srv.submit(2, 42, 1.7, 5, hot=False)
        srv.submit(3, 128, 3.0, 7, seed=99)
        got = {}
        for _ in range(50):
            srv.step()
            for r in srv.poll():
                got[r["req_id"]] = (r["E"], r["M"])
            if len(got) == 3:
                break
        s1 = oracle.init(64, 1, True)
        assert got[1] == oracle.observables(s1)
        s2 = oracle.init(42, 2, False)
        oracle.sweep(s2, 2, 0, 5, 1.7)
        assert got[2] == oracle.observables(s2)
        s3 = oracle.init(128, 99, True)
        oracle.sweep(s3, 99, 0, 7, 3.0)
        assert got[3] == oracle.observables(s3)
        assert srv.stats() == {"queued": 0, "resident": 0, "finished": 0, "bytes_in_use": 0}
    finally:
        srv.close()


def test_l32768_full_lattice_matches_oracle():
    """The headline lattice end to end: E and M after each of 2 sweeps (the
    fused reduction), E and M of the final state (the standalone one), and
    the full final state, against a full oracle run of the same chain (about
    ten seconds on the host's cores, 1 GiB of bytes)."""
    import torch

    L, seed, T, n = 32768, 11, 2.269, 2
    print("L=32768 full oracle run", flush=True)
    ref = oracle.init(L, seed, True)
    Es, Ms = oracle.sweep(ref, seed, 0, n, T, every=1)
    lat = ising.Lattice(L, seed, hot=True)
    try:
        print("L=32768 GPU run, plan", lat.plan(), flush=True)
        E, M = lat.sweep_measure(T, n, 1)
        torch.cuda.synchronize()
        assert E.cpu().numpy().tolist() == Es.tolist() and M.cpu().numpy().tolist() == Ms.tolist()
        assert lat.observables() == oracle.observables(ref) == (int(Es[-1]), int(Ms[-1]))
        got = lat.spins()
        assert got.shape == ref.shape
        rows_got = got.sum(axis=1, dtype=np.int64)
        rows_want = ref.sum(axis=1, dtype=np.int64)
        bad_rows = np.nonzero(rows_got != rows_want)[0]
        assert bad_rows.size == 0, bad_rows[:10]
        assert np.array_equal(got, ref)
    finally:
        lat.close()
