"""GPU tests of the continuous-batching server: each served result equals the
same request run alone (plain single-lattice path, and the oracle for the
small ones), whatever else shares the GPU; admission respects the memory
budget and requests join and leave while others run."""
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


def _alone(L, T, sweeps, seed, hot=True):
    lat = ising.Lattice(L, seed, hot=hot)
    lat.sweep(T, sweeps)
    em = lat.observables()
    lat.close()
    return em


def test_served_results_equal_alone():
    rng = np.random.default_rng(2026)
    reqs = []
    for rid in range(24):
        L = int(2 ** rng.integers(4, 11))  # 16 .. 1024
        T = float(rng.uniform(1.5, 3.5))
        sweeps = int(rng.integers(0, 60))
        reqs.append((rid, L, T, sweeps))
    srv = ising.Server(hbm_budget=1 << 26, max_slots=8, quantum_sweeps=7)
    try:
        results = {}
        pending = list(reqs)
        steps = 0
        while len(results) < len(reqs):
            # requests arrive while others are running
            for _ in range(3):
                if pending:
                    rid, L, T, sw = pending.pop(0)
                    srv.submit(rid, L, T, sw)
            srv.step()
            for r in srv.poll():
                results[r["req_id"]] = r
            steps += 1
            assert steps < 10000
        for rid, L, T, sw in reqs:
            r = results[rid]
            assert r["status"] == 0
            assert (r["E"], r["M"]) == _alone(L, T, sw, rid), rid
            if L <= 128:
                s = oracle.init(L, rid, True)
                oracle.sweep(s, rid, 0, sw, T)
                assert (r["E"], r["M"]) == oracle.observables(s)
            assert r["t_submit_s"] <= r["t_admit_s"] <= r["t_done_s"]
    finally:
        srv.close()


def test_served_config5_shapes_equal_alone():
    """Requests of the served workload's shapes -- L = 2^U{7..12} (128 ..
    4096), T ~ U[1.5, 3.5], hot start, seed = request id -- with 1000 to 3000
    sweeps each, so that every request spans many 100-sweep quanta; 32
    requests share 8 slots and arrive two per quantum while others run.
    Every served E, M equals the request run alone on the single-lattice
    path, and the oracle's for L <= 256."""
    rng = np.random.default_rng(2026)
    reqs = []
    for rid in range(32):
        L = int(2 ** rng.integers(7, 13))
        T = float(rng.uniform(1.5, 3.5))
        sweeps = int(rng.integers(1000, 3001))
        reqs.append((rid, L, T, sweeps))
    assert {L for _, L, _, _ in reqs} == {128, 256, 512, 1024, 2048, 4096}
    srv = ising.Server(hbm_budget=1 << 30, max_slots=8, quantum_sweeps=100)
    try:
        results, pending, steps, max_resident = {}, list(reqs), 0, 0
        while len(results) < len(reqs):
            for _ in range(2):
                if pending:
                    rid, L, T, sw = pending.pop(0)
                    srv.submit(rid, L, T, sw)
            srv.step()
            max_resident = max(max_resident, srv.stats()["resident"])
            for r in srv.poll():
                results[r["req_id"]] = r
            steps += 1
            assert steps < 100000
        assert max_resident == 8
        for rid, L, T, sw in reqs:
            r = results[rid]
            assert r["status"] == 0 and r["L"] == L and r["sweeps"] == sw
            assert (r["E"], r["M"]) == _alone(L, T, sw, rid), rid
            if L <= 256:
                s = oracle.init(L, rid, True)
                oracle.sweep(s, rid, 0, sw, T)
                assert (r["E"], r["M"]) == oracle.observables(s), rid
    finally:
        srv.close()


def test_admission_by_memory_budget():
    L = 512
    per = ising.ising_required_bytes(L)  # 106496 bytes
    srv = ising.Server(hbm_budget=3 * per + 100, max_slots=64, quantum_sweeps=5)
    try:
        for rid in range(7):
            srv.submit(rid, L, 2.5, 10)
        srv.step()
        st = srv.stats()
        assert st["resident"] == 3 and st["queued"] == 4
        assert st["bytes_in_use"] <= 3 * per + 100
        done = []
        for _ in range(100):
            srv.step()
            done += srv.poll()
            if len(done) == 7:
                break
        assert sorted(r["req_id"] for r in done) == list(range(7))
        for r in done:
            assert (r["E"], r["M"]) == _alone(L, 2.5, 10, r["req_id"])
        with pytest.raises(ising.IsingError):
            srv.submit(99, 4096, 2.0, 10)  # larger than the whole budget
    finally:
        srv.close()
