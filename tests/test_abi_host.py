"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every entry point include/ising.h declares, and its argument checks, geometry
and thresholds (host code only) behave as documented."""
import os
import re

import pytest

import oracle
import paper_1811_04384_amd as ising
from paper_1811_04384_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "ising.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ising_[a-z_0-9]+)\s*\(", text)))


def test_header_and_binding_agree():
    declared = _declared()
    assert len(declared) >= 30
    assert declared == sorted(_lib.SIGNATURES)


def test_library_exports_every_declared_symbol():
    lib = ising.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert ising.ising_version().startswith("ising-msc")


def test_library_was_built_from_these_sources():
    # load() refuses a library whose embedded source hash differs; the tests
    # (and the benchmark) therefore never run a stale build
    from paper_1811_04384_amd.build import source_hash

    assert ising.ising_version().endswith(" src " + source_hash())


def test_instruction_rate_microbenchmark_is_built():
    # a program of the benchmark, built beside bench.py (not by the library's
    # build); bench.py --valu-rates runs it
    from bench import VALU_RATES, VALU_RATES_SRC

    assert os.path.isfile(VALU_RATES) and os.access(VALU_RATES, os.X_OK)
    assert os.path.getmtime(VALU_RATES) >= os.path.getmtime(VALU_RATES_SRC)
    assert not os.path.exists(os.path.join(ROOT, "paper_1811_04384_amd", "valu_rates"))


def test_geometry_matches_oracle():
    for L in list(range(4, 400, 2)) + [1008, 2016, 4096, 32768, 1 << 18]:
        assert ising.ising_word_rows(L) == oracle.word_rows(L)
        assert ising.ising_required_bytes(L) == 8 * oracle.word_rows(L) * L
    for L in (0, 2, 3, 5, 1001, (1 << 18) + 2, -4):
        assert ising.ising_word_rows(L) == 0 and ising.ising_required_bytes(L) == 0


def test_thresholds_equal_oracle_exactly():
    import numpy as np

    for T in list(np.linspace(0.05, 12, 600)) + [1.5, 2.269, 2.6, 3.5, 1e-3, 1e6]:
        assert ising.ising_thresholds(T) == oracle.thresholds(T), T
    for bad in (0.0, -2.0, float("inf"), float("nan")):
        with pytest.raises(ising.IsingError) as e:
            ising.ising_thresholds(bad)
        assert e.value.code == ising.ISING_EINVAL


def test_invalid_sizes_fail_before_touching_a_gpu():
    for L in (0, 2, 5, 1 << 19):
        with pytest.raises(ising.IsingError) as e:
            ising.ising_create(L, 1, ising.ISING_HOT, stream=0)
        assert e.value.code == ising.ISING_EINVAL
        assert "L must be even" in ising.ising_last_error()
    with pytest.raises(ising.IsingError):
        ising.ising_create(64, 1, 7, stream=0)
    with pytest.raises(ising.IsingError):
        ising.ising_batch_create([64, 63], [1, 2], [1, 1], stream=0)
    with pytest.raises(ising.IsingError):
        ising.ising_server_create(1 << 20, 0, 10, stream=0)


def test_thermodynamics_host_equals_oracle():
    """The library's host-side derivation of e, c, |m|, chi and the Binder
    cumulant from exact moment sums agrees with the oracle's exact rational
    evaluation, including sums that need every 64-bit limb."""
    import random

    rng = random.Random(7)
    cases = []
    for L in (4, 64, 4096, 32768, 1 << 18):
        N = L * L
        for _ in range(6):
            n = rng.randint(1, 5000)
            Es = [-rng.randint(N // 2, 2 * N) for _ in range(min(n, 50))]
            Ms = [rng.randint(-N, N) for _ in range(min(n, 50))]
            reps = n // len(Es) or 1
            m = oracle.moments(Es * reps, Ms * reps)
            cases.append((m, L, rng.uniform(0.5, 6.0)))
    for m, L, T in cases:
        got = ising.ising_thermodynamics(m, L, T)
        want = oracle.thermodynamics(m, L, T)
        for k in ("e", "abs_m", "binder"):
            assert got[k] == pytest.approx(want[k], rel=1e-12, abs=1e-15), (k, L)
        for k in ("c", "chi"):  # differences of near-equal means: relative to the larger term
            scale = max(abs(want[k]), 1e-6 * (4.0 if k == "c" else 1.0) * L * L / T)
            assert abs(got[k] - want[k]) <= 1e-9 * scale, (k, L, got[k], want[k])
    assert m["sum_M4"] >= 1 << 128  # the third limb was exercised


def test_moment_calls_reject_bad_arguments_without_a_gpu():
    zero = {"n_samples": 0, "sum_E": 0, "sum_E2": 0, "sum_absM": 0, "sum_M2": 0, "sum_M4": 0}
    one = dict(zero, n_samples=1, sum_E=-32, sum_E2=1024, sum_absM=16, sum_M2=256, sum_M4=65536)
    with pytest.raises(ising.IsingError) as e:
        ising.ising_thermodynamics(zero, 4, 2.0)
    assert e.value.code == ising.ISING_EINVAL
    for L, T in ((5, 2.0), (4, 0.0), (4, float("nan")), (0, 2.0)):
        with pytest.raises(ising.IsingError):
            ising.ising_thermodynamics(one, L, T)
    assert ising.ising_thermodynamics(one, 4, 2.0) == {"e": -2.0, "c": 0.0, "abs_m": 1.0, "chi": 0.0,
                                                        "binder": 2.0 / 3.0}
    lib = ising.load()
    assert lib.ising_scan(None, 1, None, 0, 1, 1, None) == ising.ISING_EINVAL
    assert lib.ising_batch_scan(None, 1, None, 0, 1, 1, None) == ising.ISING_EINVAL
    assert lib.ising_sweep_moments(None, 2.0, 1, 1, None) == ising.ISING_EINVAL
    assert lib.ising_batch_moments(None, None) == ising.ISING_EINVAL


def test_batch_plan_check_bounds_resident_lattices():
    # one workgroup per lattice is refused for sizes far beyond one
    # workgroup's LDS (a 2^18 lattice is 26 GB and its word offsets need 64
    # bits), before any batch or GPU exists
    ok = dict(resident_max_L=4096, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=50)
    ising.ising_batch_check_plan(ok)
    ising.ising_batch_check_plan(dict(ok, draw_sweeps=4096))
    for bad in (dict(ok, resident_max_L=1 << 18), dict(ok, resident_max_L=4098), dict(ok, resident_max_L=-2),
                dict(ok, words_per_thread=3), dict(ok, tiled_block=96), dict(ok, resident_block=2048),
                dict(ok, sweeps_per_graph=0), dict(ok, draw_sweeps=-1), dict(ok, draw_sweeps=4097)):
        with pytest.raises(ising.IsingError) as e:
            ising.ising_batch_check_plan(bad)
        assert e.value.code == ising.ISING_EINVAL
    with pytest.raises(ising.IsingError):
        ising.ising_batch_check_plan(dict(ok, resident_max_L=1 << 18))
    assert "resident_max_L" in ising.ising_last_error()
