"""The allocation-free entry point (ising_sweep_measure_static), called
through the C ABI, against the existing ising_sweep_measure on the same
lattice: the E/M series and the final words are equal bit for bit, on two
calls in a row, the second with a smaller lattice (the shared scratch keeps
the first call's contents); the smaller one also equals the oracle.  A
lattice too large for the fixed scratch is refused before any GPU work."""
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


def _static_run(L, seed, T, n, every):
    import torch

    init = ising.Lattice(L, seed, hot=True)  # the library's hot start, copied into a caller buffer
    buf = init.words.clone()
    init.close()
    k = n // every
    E = torch.empty(k, dtype=torch.int64, device="cuda")
    M = torch.empty(k, dtype=torch.int64, device="cuda")
    ising.ising_sweep_measure_static(buf, buf.numel() * 8, L, seed, 0, T, n, every, E, M)
    torch.cuda.synchronize()
    return buf, E.cpu().numpy(), M.cpu().numpy()


def test_static_entry_point_equals_sweep_measure():
    import torch

    for L, seed, T, n, every in ((1008, 5, 2.4, 12, 3), (130, 6, 1.9, 7, 2)):
        print(f"static entry point L={L} n={n} every={every}", flush=True)
        ref = ising.Lattice(L, seed, hot=True)
        try:
            ref.set_resident_tiles(0)  # the half-sweep launches the static entry point also runs
            assert ref.resident_tiles() == (0, 0, 0) and ref.tiling() == (0, 0, 0)
            E_ref, M_ref = ref.sweep_measure(T, n, every)
            torch.cuda.synchronize()
            words, E, M = _static_run(L, seed, T, n, every)
            assert E.tolist() == E_ref.cpu().numpy().tolist() and M.tolist() == M_ref.cpu().numpy().tolist()
            assert torch.equal(words, ref.words)
            if L <= 256:
                s = oracle.init(L, seed, True)
                Es, Ms = oracle.sweep(s, seed, 0, n, T, every=every)
                assert E.tolist() == Es.tolist() and M.tolist() == Ms.tolist()
                assert (ref.spins() == s).all()
        finally:
            ref.close()


def test_static_entry_point_refuses_large_lattices():
    import torch

    L = 40000  # its sampled half-sweep needs more partial sums than the fixed scratch holds
    buf = torch.empty(8, dtype=torch.int64, device="cuda")
    E = torch.empty(1, dtype=torch.int64, device="cuda")
    with pytest.raises(ising.IsingError) as e:
        ising.ising_sweep_measure_static(buf, ising.ising_required_bytes(L), L, 1, 0, 2.0, 1, 1, E, E)
    assert e.value.code == ising.ISING_EINVAL and "static scratch" in ising.ising_last_error()
    with pytest.raises(ising.IsingError):  # a buffer smaller than the lattice
        ising.ising_sweep_measure_static(buf, 64, 64, 1, 0, 2.0, 1, 1, E, E)
