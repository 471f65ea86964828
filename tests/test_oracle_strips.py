"""Pins of the oracle's strip dynamics: the paper's own update scheme of
random word picks inside vertical strips, left half then right half of every
strip per iteration (Sections 4 and 5.2, Table 2).

What fixes it independently of the oracle: the chain samples the Boltzmann
distribution (exact enumeration of the 4 x 4 torus, Kaufman's exact energy
of the paper's 84 x 84 demonstration lattice); at infinite temperature
every pick flips its whole word, so the final state is the initial one
XOR the parity of each word's pick count, which fixes exactly which picks an
iteration applies; strips are independent inside a phase (any strip order
gives the same state); the pick stream is uniform over the phase's half of
the strip; the pick counts are the closed forms behind Table 2's ten updates
per word.  A wrong phase range, a pick count off by one, a pick applied to
the wrong strip, a frozen neighbour read from the wrong column or a missing
live-slot check fails one of these.
"""
import math

import numpy as np
import pytest

import oracle
from exact_ising import binned_mean, brute_force, kaufman_energy


def test_pick_counts_give_ten_updates_per_word():
    for L, S in ((84, 2), (84, 3), (84, 12), (84, 84), (2016, 28), (130, 10), (4, 2), (4, 4)):
        N = oracle.word_rows(L)
        h0, h1 = oracle.picks_per_phase(L, S, 0), oracle.picks_per_phase(L, S, 1)
        assert h0 == 10 * N * (S // 2) and h1 == 10 * N * (S - S // 2)
        assert (h0 + h1) * (L // S) == 10 * N * L  # every word ten times per iteration on average


@pytest.mark.parametrize("L,S,phase", [(84, 12, 0), (84, 12, 1), (84, 3, 0), (84, 3, 1), (130, 10, 1)])
def test_pick_stream_is_uniform_over_the_phase_half(L, S, phase):
    N = oracle.word_rows(L)
    lo = 0 if phase == 0 else S // 2
    width = S // 2 if phase == 0 else S - S // 2
    p, n = 3, 40_000
    rows = np.zeros(N, dtype=np.int64)
    cols = np.zeros(width, dtype=np.int64)
    for k in range(n):
        I, J = oracle.pick(99, 5, L, S, phase, p, k)
        assert 0 <= I < N and p * S + lo <= J < p * S + lo + width
        rows[I] += 1
        cols[J - p * S - lo] += 1
    for counts in (rows, cols):
        if len(counts) < 2:
            continue
        expect = n / len(counts)
        chi2 = float(((counts - expect) ** 2 / expect).sum())
        dof = len(counts) - 1
        assert chi2 < dof + 6 * math.sqrt(2 * dof), (chi2, dof)


@pytest.mark.parametrize("L,S", [(42, 2), (42, 3), (42, 6), (42, 42), (130, 10), (130, 26), (84, 12)])
def test_strips_are_independent_inside_a_phase(L, S):
    a = oracle.init(L, 17, True)
    b = a.copy()
    oracle.random_iterations(a, 17, 0, 3, 2.3, S, order=0)
    oracle.random_iterations(b, 17, 0, 3, 2.3, S, order=1)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("L,S", [(84, 2), (84, 7), (130, 10), (12, 12)])
def test_infinite_temperature_flips_each_picked_word(L, S):
    """At T -> infinity both thresholds are 2^32 - 1, so a pick flips every
    live spin of its word unless a draw equals 2^32 - 1 (checked not to
    happen here).  One iteration therefore leaves each spin flipped the
    number of times its word was picked."""
    seed, t = 2718, 9
    N = oracle.word_rows(L)
    assert oracle.thresholds(1e300) == (2 ** 32 - 1, 2 ** 32 - 1)
    count = np.zeros((N, L), dtype=np.int64)
    for h in (0, 1):
        for p in range(L // S):
            for k in range(oracle.picks_per_phase(L, S, h)):
                I, J = oracle.pick(seed, t, L, S, h, p, k)
                count[I, J] += 1
                assert all(oracle.pick_uniform(seed, t, h, p, k, q) != 2 ** 32 - 1 for q in (0, 7, 20))
    s0 = oracle.init(L, seed, True)
    s = s0.copy()
    oracle.random_iterations(s, seed, t, 1, 1e300, S)
    r = np.arange(L)
    expect = s0 ^ (count[r % N, :] & 1).astype(np.uint8)
    assert np.array_equal(s, expect)


@pytest.mark.parametrize("S,T", [(2, 1.8), (4, 1.8), (2, 3.0), (4, 3.0)])
def test_4x4_torus_matches_enumeration(S, T):
    e_ex, m_ex = brute_force(4, T)
    s = oracle.init(4, 31, True)
    oracle.random_iterations(s, 31, 0, 200, T, S, threads=1)
    Es, Ms = oracle.random_iterations(s, 31, 200, 100_000, T, S, every=1, threads=1)
    e_mc, e_err = binned_mean(Es / 16, 50)
    m_mc, m_err = binned_mean(np.abs(Ms) / 16, 50)
    assert abs(e_mc - e_ex) < 5 * e_err + 1e-4, (e_mc, e_ex, e_err)
    assert abs(m_mc - m_ex) < 5 * m_err + 1e-4, (m_mc, m_ex, m_err)


@pytest.mark.parametrize("S,T", [(2, 2.0), (12, 2.0), (2, 2.6), (28, 3.5)])
def test_paper_lattice_matches_kaufman(S, T):
    """The paper's demonstration lattice (N = 4, L = 84) with S columns per
    strip (84 / S processes): the energy per spin averaged over iterations
    against Kaufman's exact value."""
    L = 84
    s = oracle.init(L, 8, True)
    oracle.random_iterations(s, 8, 0, 300, T, S)
    Es, _ = oracle.random_iterations(s, 8, 300, 1500, T, S, every=1)
    e_mc, e_err = binned_mean(Es / L ** 2, 15)
    assert abs(e_mc - kaufman_energy(L, T)) < 5 * e_err + 1e-3, (e_mc, kaufman_energy(L, T), e_err)


def test_frozen_ground_state_and_counter():
    s = oracle.init(42, 1, False)
    Es, Ms = oracle.random_iterations(s, 1, 0, 6, 0.3, 6, every=2)
    assert s.all() and list(Es) == [-2 * 42 * 42] * 3 and list(Ms) == [42 * 42] * 3
    # iterations are absolute: 2 then 3 equals 5
    a = oracle.init(42, 4, True)
    b = a.copy()
    oracle.random_iterations(a, 4, 0, 5, 2.2, 6)
    oracle.random_iterations(b, 4, 0, 2, 2.2, 6)
    oracle.random_iterations(b, 4, 2, 3, 2.2, 6)
    assert np.array_equal(a, b)


def test_invalid_strip_arguments():
    s = oracle.init(84, 1, True)
    for S in (0, 1, 5, 85, 168):
        assert not oracle.random_valid(84, S)
        with pytest.raises(ValueError):
            oracle.random_iterations(s, 1, 0, 1, 2.0, S)
    assert not oracle.random_valid(32768, 32768)  # 10 N S/2 picks per phase exceeds the per-strip limit
    with pytest.raises(ValueError):
        oracle.random_iterations(s, 1, 0, 1, -1.0, 2)
