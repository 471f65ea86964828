"""Pins for the oracle's local update rule and thresholds.

Table 1 of the paper (tests/golden/table1_delta_e.csv) fixes, for every
configuration of a spin and its four neighbours, the 3-bit group value
(number of antiparallel neighbours) and dE; the Metropolis rule of Section 2
fixes which dE need a random number.  Thresholds are checked against a
50-digit evaluation of floor(exp(-4k/T) 2^32).
"""
import csv
import itertools
import os

import mpmath
import numpy as np

import oracle


def _table1(golden_dir):
    with open(os.path.join(golden_dir, "table1_delta_e.csv")) as f:
        rows = [r for r in csv.DictReader(line for line in f if not line.startswith("#"))]
    assert len(rows) == 10
    return rows


def test_table1_energies_are_consistent(golden_dir):
    # E = -J s * (sum of neighbours); E' = -E; dE = E' - E
    for row in _table1(golden_dir):
        s = 1 if row["selected"] == "up" else -1
        nsum = int(row["neighbours_up"]) - int(row["neighbours_down"])
        assert int(row["E"]) == -s * nsum
        assert int(row["E_prime"]) == s * nsum
        assert int(row["dE"]) == int(row["E_prime"]) - int(row["E"])


def test_table1_accept_rule(golden_dir):
    """Every one of the 32 (spin, 4 neighbours) configurations: the oracle's
    count of antiparallel neighbours equals the table's 3-bit group, and its
    decision equals the Metropolis rule with the table's dE."""
    by_key = {}
    for row in _table1(golden_dir):
        by_key[(row["selected"], int(row["neighbours_up"]))] = row
    T = 2.3
    t4, t8 = oracle.thresholds(T)
    us = [0, 1, t8 - 1, t8, t8 + 1, t4 - 1, t4, t4 + 1, 2**31, 2**32 - 1]
    for spin in (0, 1):
        for nb in itertools.product((0, 1), repeat=4):
            n_anti = sum(1 for x in nb if x != spin)
            row = by_key[("up" if spin else "down", sum(nb))]
            assert int(row["group"], 2) == n_anti
            dE = int(row["dE"])
            # a lattice whose centre has this neighbourhood: count through the oracle
            s = np.ones((4, 4), dtype=np.uint8)
            s[1, 1] = spin
            s[0, 1], s[2, 1], s[1, 0], s[1, 2] = nb
            E0, _ = oracle.observables(s)
            s2 = s.copy()
            s2[1, 1] ^= 1
            E1, _ = oracle.observables(s2)
            assert E1 - E0 == dE  # energy change of the flip, units of J
            for u in us:
                if dE <= 0:
                    want = True
                elif dE == 4:
                    want = u < t4
                else:
                    want = u < t8
                assert oracle.accept(n_anti, u, t4, t8) == want, (spin, nb, u)


def _exact_threshold(x_num, T):
    with mpmath.workdps(50):
        v = mpmath.exp(mpmath.mpf(x_num) / mpmath.mpf(T)) * mpmath.mpf(2) ** 32
        return v


def test_thresholds_match_high_precision():
    Ts = list(np.linspace(0.05, 10.0, 397)) + [1.5, 2.0, 2.269, 2.6, 3.5, 1.5 + 2 * 3 / 7]
    for T in Ts:
        t4, t8 = oracle.thresholds(T)
        for got, k in ((t4, 4), (t8, 8)):
            exact = _exact_threshold(-k, float(T))
            fl = int(mpmath.floor(exact))
            frac = float(exact - fl)
            if 1e-5 < frac < 1 - 1e-5:  # libm's last-ulp error cannot move floor here
                assert got == min(fl, 2**32 - 1), (T, k)
            else:
                assert abs(got - fl) <= 1


def test_thresholds_limits():
    assert oracle.thresholds(0.1) == (0, 0)  # exp(-40) 2^32 < 1
    t4, t8 = oracle.thresholds(1e300)
    assert t4 == 2**32 - 1 and t8 == 2**32 - 1
    prev = (-1, -1)
    for T in np.linspace(0.2, 50, 200):
        cur = oracle.thresholds(T)
        assert cur[0] >= prev[0] and cur[1] >= prev[1]
        assert cur[1] <= cur[0]
        prev = cur


def test_acceptance_frequencies_per_class():
    """Binomial check of the three classes on a state built so that the
    colour-0 sites of rows 0,2 (mod 4) have one antiparallel neighbour,
    rows 1 (mod 4) two, rows 3 (mod 4) none.  Colour-0 sites are final after
    the first half of the sweep, so their flips count acceptances."""
    L, T = 64, 2.0
    t4, t8 = oracle.thresholds(T)
    base = np.ones((L, L), dtype=np.uint8)
    rr, cc = np.meshgrid(np.arange(L), np.arange(L), indexing="ij")
    base[(rr % 4 == 1) & ((rr + cc) % 2 == 1)] = 0
    colour0 = (rr + cc) % 2 == 0
    cls = {1: colour0 & ((rr % 4 == 0) | (rr % 4 == 2)), 2: colour0 & (rr % 4 == 1), 0: colour0 & (rr % 4 == 3)}
    flips = {0: 0, 1: 0, 2: 0}
    trials = {0: 0, 1: 0, 2: 0}
    for seed in range(60):
        s = base.copy()
        oracle.sweep(s, seed, 0, 1, T, threads=1)
        for k, m in cls.items():
            flips[k] += int((s[m] != base[m]).sum())
            trials[k] += int(m.sum())
    assert flips[2] == trials[2]
    for k, t in ((1, t4), (0, t8)):
        p = t / 2**32
        mean = trials[k] * p
        sd = (trials[k] * p * (1 - p)) ** 0.5
        assert abs(flips[k] - mean) < 5 * sd, (k, flips[k], mean, sd)
