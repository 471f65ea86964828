"""Pins of the oracle's temperature scan and moment sums.

The scan carries one lattice through a sequence of temperatures (the paper's
driver loop, Section 5) and sums E, E^2, |M|, M^2, M^4 over the samples at
each temperature.  What fixes the result independently of the oracle:
exact enumeration of the 4 x 4 torus (every moment), Kaufman's exact
finite-lattice energy and specific heat (pinned to the enumeration first),
and the frozen ground state below the temperature at which no uphill move
can be accepted.  A moment summed with the wrong power, a variance missing
the <E>^2 term, a wrong 1/T power in c or chi, or a scan that restarts the
lattice or the sweep counter at each temperature fails one of these.
"""
import math

import numpy as np
import pytest

import oracle
from exact_ising import binned_mean, brute_force_moments, kaufman_energy, kaufman_specific_heat


def _chain(L, seed, hot, Ts, therm, meas, every=1):
    """The scan's chain run sweep by sweep, keeping the series."""
    s = oracle.init(L, seed, hot)
    t = 0
    series = []
    for T in Ts:
        oracle.sweep(s, seed, t, therm, T)
        t += therm
        Es, Ms = oracle.sweep(s, seed, t, meas, T, every)
        t += meas
        series.append((Es.astype(np.float64), Ms.astype(np.float64)))
    return series, s, t


def _jackknife_c(E, T, n_spins, nbins):
    """Specific heat per spin and its jackknife error over contiguous bins."""
    nb = len(E) // nbins
    E = E[: nb * nbins].reshape(nbins, nb)
    s1, s2 = E.sum(axis=1), (E * E).sum(axis=1)
    tot1, tot2, n = s1.sum(), s2.sum(), nb * nbins

    def c_of(a1, a2, m):
        return (a2 / m - (a1 / m) ** 2) / (T * T * n_spins)

    full = c_of(tot1, tot2, n)
    loo = np.array([c_of(tot1 - s1[b], tot2 - s2[b], n - nb) for b in range(nbins)])
    err = math.sqrt((nbins - 1) / nbins * ((loo - loo.mean()) ** 2).sum())
    return float(full), err


def test_scan_carries_lattice_and_counter():
    """Heating then cooling: each temperature continues from the previous
    state at the next absolute sweep index (sweeping a then b equals a + b)."""
    Ts = [1.9, 2.4, 3.1, 2.2]
    ms, s, t = oracle.scan(24, 77, True, Ts, therm=5, meas=12, every=3)
    series, s_ref, t_ref = _chain(24, 77, True, Ts, 5, 12, 3)
    assert t == t_ref == len(Ts) * 17
    assert np.array_equal(s, s_ref)
    for m, (Es, Ms) in zip(ms, series):
        assert m["n_samples"] == 4
        assert m["sum_E"] == int(Es.sum()) and m["sum_absM"] == int(np.abs(Ms).sum())
    # one uninterrupted run of all sweeps reaches the same state
    s2 = oracle.init(24, 77, True)
    t2 = 0
    for T in Ts:
        oracle.sweep(s2, 77, t2, 17, T)
        t2 += 17
    assert np.array_equal(s2, s)


@pytest.mark.parametrize("T", [1.8, 2.5, 3.5])
def test_4x4_moments_match_enumeration(T):
    """Every moment of the 4 x 4 torus against the exact canonical average
    over all 2^16 states, and c from the moments against the exact c."""
    series, _, _ = _chain(4, 4242, True, [T], 1000, 200_000)
    Es, Ms = series[0]
    ex = brute_force_moments(4, T)
    ms, _, _ = oracle.scan(4, 4242, True, [T], 1000, 200_000)
    m = ms[0]
    n = m["n_samples"]
    assert n == 200_000
    for key, x, exact in (("sum_E", Es, ex["E"]), ("sum_E2", Es * Es, ex["E2"]), ("sum_absM", np.abs(Ms), ex["absM"]),
                          ("sum_M2", Ms * Ms, ex["M2"]), ("sum_M4", Ms ** 4, ex["M4"])):
        mean, err = binned_mean(x, 50)
        assert m[key] / n == pytest.approx(mean, rel=1e-12)
        assert abs(mean - exact) < 5 * err + 1e-9 * abs(exact), (key, mean, exact, err)
    c, c_err = _jackknife_c(Es, T, 16, 50)
    c_exact = (ex["E2"] - ex["E"] ** 2) / (T * T * 16)
    assert abs(c - c_exact) < 5 * c_err, (c, c_exact, c_err)
    th = oracle.thermodynamics(m, 4, T)
    assert th["c"] == pytest.approx(c, rel=1e-9)
    chi_exact = (ex["M2"] - ex["absM"] ** 2) / (T * 16)
    binder_exact = 1 - ex["M4"] / (3 * ex["M2"] ** 2)
    assert th["chi"] == pytest.approx(chi_exact, rel=0.05)
    assert th["binder"] == pytest.approx(binder_exact, abs=0.01)


def test_kaufman_specific_heat_matches_enumeration():
    # the exact finite-size specific heat is pinned before it is used as a pin
    for T in (1.3, 2.0, 2.27, 2.9, 4.0):
        ex = brute_force_moments(4, T)
        c_exact = (ex["E2"] - ex["E"] ** 2) / (T * T * 16)
        assert abs(kaufman_specific_heat(4, T) - c_exact) < 1e-10


def test_l16_heating_scan_matches_kaufman():
    """Heating scan of a 16 x 16 torus: energy and specific heat per spin at
    each temperature against Kaufman's exact finite-lattice values."""
    Ts = [1.8, 2.2, 2.4, 2.8, 3.5]
    series, _, _ = _chain(16, 99, False, Ts, 2000, 60_000)
    ms, _, _ = oracle.scan(16, 99, False, Ts, 2000, 60_000)
    for T, (Es, _), m in zip(Ts, series, ms):
        e_mc, e_err = binned_mean(Es / 256, 40)
        assert abs(e_mc - kaufman_energy(16, T)) < 5 * e_err + 1e-4, (T, e_mc, e_err)
        c, c_err = _jackknife_c(Es, T, 256, 40)
        c_exact = kaufman_specific_heat(16, T)
        assert abs(c - c_exact) < 5 * c_err + 1e-3, (T, c, c_exact, c_err)
        assert oracle.thermodynamics(m, 16, T)["c"] == pytest.approx(c, rel=1e-9)


def test_frozen_ground_state():
    """At T = 0.3, t8 = floor(exp(-8/T) 2^32) = 0, so from the all-up state
    (where every move has dE = +8) nothing is ever accepted: every sample is
    E = -2 L^2, M = L^2, and the moments and derived quantities are closed
    forms (c = chi = 0, Binder cumulant 2/3)."""
    L, T = 12, 0.3
    assert oracle.thresholds(T)[1] == 0
    ms, s, _ = oracle.scan(L, 5, False, [T, T], therm=3, meas=40, every=2)
    assert s.all()
    N = L * L
    for m in ms:
        n = m["n_samples"]
        assert n == 20
        assert m == {"n_samples": n, "sum_E": -2 * N * n, "sum_E2": 4 * N ** 2 * n, "sum_absM": N * n,
                     "sum_M2": N ** 2 * n, "sum_M4": N ** 4 * n}
        th = oracle.thermodynamics(m, L, T)
        assert th == {"e": -2.0, "c": 0.0, "abs_m": 1.0, "chi": 0.0, "binder": 2.0 / 3.0}


def test_empty_measurement():
    ms, _, t = oracle.scan(8, 1, True, [2.0, 3.0], therm=4, meas=2, every=3)
    assert t == 12
    assert all(m["n_samples"] == 0 and m["sum_M4"] == 0 for m in ms)
    with pytest.raises(ValueError):
        oracle.thermodynamics(ms[0], 8, 2.0)
