"""GPU parity of the paper's own dynamics (random word picks inside vertical
strips, two phases per iteration): the state, E/M series and moment sums
equal the oracle's bit for bit for even and odd strip widths, one strip,
ragged word rows and the paper's lattices; mixing with checkerboard sweeps
on the shared counter; argument checks; and the energy against Kaufman."""

import numpy as np
import pytest

import oracle
import paper_1811_04384_amd as ising
from exact_ising import binned_mean, kaufman_energy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    ising.load()


@pytest.mark.parametrize("L,S,seed,hot,T,n,every", [
    (84, 2, 1, True, 2.2, 3, 1),      # the paper's N = 4 lattice, 42 strips of 2 columns
    (84, 12, 2, False, 2.6, 4, 2),    # 7 processes as in the paper's decomposition
    (84, 84, 3, True, 1.9, 2, 1),     # one strip: the whole lattice is one process
    (42, 3, 5, True, 2.0, 5, 1),      # odd width: 1 column in phase 0, 2 in phase 1
    (130, 10, 4, True, 2.4, 3, 1),    # ragged word rows (dead slots)
    (2016, 28, 6, True, 2.269, 2, 1), # Table 2's N = 96 lattice on 72 processes
    (2016, 2, 7, True, 2.5, 1, 1),    # 1008 strips
    (2016, 56, 8, True, 2.3, 1, 1),   # strip columns too large for LDS: one-kernel path
    (1008, 1008, 9, False, 2.6, 1, 1),  # one strip of the whole lattice, one-kernel path
    (5376, 2, 10, True, 2.4, 1, 1),   # 2688 strips: the picks of a phase are drawn in two chunks
])
def test_strip_dynamics_matches_oracle(L, S, seed, hot, T, n, every):
    print(f"strips L={L} S={S} seed={seed}", flush=True)
    lat = ising.Lattice(L, seed, hot=hot)
    E, M = lat.random_iterations(T, S, n, every)
    s = oracle.init(L, seed, hot)
    Es, Ms = oracle.random_iterations(s, seed, 0, n, T, S, every=every)
    assert np.array_equal(E.cpu().numpy(), Es) and np.array_equal(M.cpu().numpy(), Ms)
    assert np.array_equal(lat.spins(), s)
    assert lat.t == n
    lat.close()


def test_mixed_with_checkerboard_and_moments():
    """Checkerboard sweeps and strip iterations advance one counter; moments
    of the strip samples accumulate on the device."""
    import torch

    L, seed, T = 126, 12, 2.3
    lat = ising.Lattice(L, seed, hot=True)
    lat.sweep(T, 3)
    acc = torch.zeros(10, dtype=torch.int64, device="cuda")
    lat.random_iterations(T, 6, 4, 1, acc)
    lat.sweep(T, 2)
    lat.random_iterations(T, 6, 3, 3, acc)
    s = oracle.init(L, seed, True)
    oracle.sweep(s, seed, 0, 3, T)
    E1, M1 = oracle.random_iterations(s, seed, 3, 4, T, 6, every=1)
    oracle.sweep(s, seed, 7, 2, T)
    E2, M2 = oracle.random_iterations(s, seed, 9, 3, T, 6, every=3)
    assert np.array_equal(lat.spins(), s) and lat.t == 12
    assert ising.moments_of(acc) == oracle.moments(list(E1) + list(E2), list(M1) + list(M2))
    lat.close()


def test_invalid_strip_arguments_do_no_work():
    lat = ising.Lattice(84, 1, hot=True)
    before = lat.spins()
    for S in (0, 1, 5, 85, 168):
        with pytest.raises(ising.IsingError):
            lat.random_iterations(2.0, S, 1)
    with pytest.raises(ising.IsingError):
        lat.random_iterations(-2.0, 2, 1)
    with pytest.raises(ising.IsingError):
        ising.ising_random_iterations(lat.handle, 2.0, 2, -1)
    with pytest.raises(ising.IsingError):  # outputs without a sampling interval
        ising.ising_random_iterations(lat.handle, 2.0, 2, 1, 0, lat.words, lat.words)
    assert lat.t == 0 and np.array_equal(lat.spins(), before)
    lat.random_iterations(2.0, 2, 0)  # zero iterations: nothing happens
    assert lat.t == 0 and np.array_equal(lat.spins(), before)
    lat.close()
    big = ising.Lattice(32768, 1, hot=True)
    with pytest.raises(ising.IsingError):  # 10 N S/2 picks per strip and phase above the limit
        big.random_iterations(2.0, 32768, 1)
    big.close()


def test_strip_dynamics_energy_matches_kaufman():
    """A 256 x 256 torus (N = 14, ragged) under the strip dynamics with 2-column
    strips: the iteration-averaged energy per spin against Kaufman."""
    L, T = 256, 2.6
    lat = ising.Lattice(L, 77, hot=True)
    lat.random_iterations(T, 2, 200)
    E, _ = lat.random_iterations(T, 2, 1000, 1)
    e = E.cpu().numpy() / L ** 2
    e_mc, e_err = binned_mean(e, 20)
    exact = kaufman_energy(L, T)
    assert abs(e_mc - exact) < 5 * e_err + 5e-4, (e_mc, exact, e_err)
    lat.close()
