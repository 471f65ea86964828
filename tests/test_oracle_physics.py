"""Pins of the oracle's Markov chain against exact statistical mechanics.

A wrong neighbour (e.g. a missing periodic wrap), a wrong sign in dE, a
transposed threshold or a biased draw moves the sampled averages away from
the exact ones by far more than the statistical errors used here.
"""
import math

import numpy as np
import pytest

import oracle
from exact_ising import TC, binned_mean, brute_force, kaufman_energy, onsager_energy, yang_magnetisation


def _run(L, T, seed, hot, n_therm, n_meas, threads=0):
    s = oracle.init(L, seed, hot)
    oracle.sweep(s, seed, 0, n_therm, T, threads=threads)
    Es, Ms = oracle.sweep(s, seed, n_therm, n_meas, T, every=1, threads=threads)
    return Es / (L * L), np.abs(Ms) / (L * L)


@pytest.mark.parametrize("T", [1.5, 1.5 + 2 * 4 / 7 * 0.5, 3.5])
def test_4x4_torus_matches_enumeration(T):
    """All 2^16 states of the 4x4 torus enumerated exactly."""
    e_ex, m_ex = brute_force(4, T)
    e, m = _run(4, T, seed=2024, hot=True, n_therm=1000, n_meas=200_000, threads=1)
    e_mc, e_err = binned_mean(e, 50)
    m_mc, m_err = binned_mean(m, 50)
    assert abs(e_mc - e_ex) < 5 * e_err + 1e-4, (e_mc, e_ex, e_err)
    assert abs(m_mc - m_ex) < 5 * m_err + 1e-4, (m_mc, m_ex, m_err)


def test_kaufman_closed_form_matches_enumeration():
    # the finite-size exact energy is pinned before it is used as a pin
    for T in (1.2, 2.0, TC, 2.9, 5.0):
        assert abs(kaufman_energy(4, T) - brute_force(4, T)[0]) < 1e-10


def test_kaufman_tends_to_onsager():
    for T in (1.5, 2.0, 2.6, 3.5):
        assert abs(kaufman_energy(256, T) - onsager_energy(T)) < 2e-4
    assert abs(onsager_energy(TC * (1 + 1e-6)) + math.sqrt(2)) < 1e-4


def test_l64_eight_temperatures_match_kaufman():
    """The small scan workload: L = 64, cold start, 8 temperatures evenly
    spaced over [1.5, 3.5], 2000 thermalisation + 2000 measurement sweeps,
    seed 1234; the mean energy per spin at each T against the exact finite-L
    value.  Near T_c the 2000-sweep average carries a larger error, which the
    binned error estimate reflects."""
    Ts = [1.5 + 2.0 * i / 7 for i in range(8)]
    for T in Ts:
        e, _ = _run(64, T, seed=1234, hot=False, n_therm=2000, n_meas=2000)
        e_mc, e_err = binned_mean(e, 10)
        e_ex = kaufman_energy(64, T)
        assert abs(e_mc - e_ex) < 5 * e_err + 2e-3, (T, e_mc, e_ex, e_err)


@pytest.mark.parametrize("T,hot", [(1.5, False), (2.0, False), (2.6, True), (3.5, True)])
def test_l128_matches_onsager_and_yang(T, hot):
    L = 128
    e, m = _run(L, T, seed=77, hot=hot, n_therm=1000, n_meas=2000)
    e_mc, e_err = binned_mean(e, 10)
    assert abs(e_mc - onsager_energy(T)) < 5 * e_err + 2e-3, (e_mc, onsager_energy(T), e_err)
    if T < TC:
        m_mc, m_err = binned_mean(m, 10)
        assert abs(m_mc - yang_magnetisation(T)) < 5 * m_err + 3e-3, (m_mc, yang_magnetisation(T), m_err)


def test_ground_state_is_fixed_point():
    """T = 0.1 makes both thresholds 0: only dE <= 0 moves survive, and a
    fully aligned state has none, so it never changes."""
    for L in (4, 42, 64):
        s = oracle.init(L, 5, hot=False)
        Es, Ms = oracle.sweep(s, 5, 0, 20, 0.1, every=1, threads=1)
        assert (s == 1).all()
        assert (Es == -2 * L * L).all() and (Ms == L * L).all()


def test_zero_temperature_energy_never_rises():
    L = 64
    s = oracle.init(L, 9, hot=True)
    E0, _ = oracle.observables(s)
    Es, _ = oracle.sweep(s, 9, 0, 200, 0.1, every=1, threads=1)
    seq = np.concatenate([[E0], Es])
    assert (np.diff(seq) <= 0).all()
    assert seq[-1] < seq[0]
