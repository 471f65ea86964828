"""Pins for the oracle's random numbers.

Philox4x32-10 is checked against (a) the published known-answer vectors
(tests/golden/philox4x32_10_kat.txt) and (b) an independent open-source
implementation compiled and run here: ATen's PhiloxRNGEngine.h from the
installed PyTorch headers.  The site -> counter map is checked for the
property that makes it a valid map: no two sites of a sweep share a draw.
"""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle


def _kat_rows(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(golden_dir):
    rows = _kat_rows(golden_dir)
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert oracle.philox4x32_10(ctr, key) == want


ATEN_PROG = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
    // args: key0 key1 c0 c1 c2 c3 (decimal); prints 4 outputs
    uint64_t seed = (uint64_t)strtoull(argv[1], 0, 10) | ((uint64_t)strtoull(argv[2], 0, 10) << 32);
    uint64_t offset = (uint64_t)strtoull(argv[3], 0, 10) | ((uint64_t)strtoull(argv[4], 0, 10) << 32);
    uint64_t subseq = (uint64_t)strtoull(argv[5], 0, 10) | ((uint64_t)strtoull(argv[6], 0, 10) << 32);
    at::Philox4_32 eng(seed, subseq, offset);
    for (int i = 0; i < 4; ++i) printf("%u ", (unsigned)eng());
    printf("\n");
    return 0;
}
"""


@pytest.fixture(scope="module")
def aten_philox():
    import torch

    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")) or shutil.which("g++") is None:
        pytest.skip("ATen Philox header or g++ not available")
    d = tempfile.mkdtemp()
    src = os.path.join(d, "p.cpp")
    exe = os.path.join(d, "p")
    with open(src, "w") as f:
        f.write(ATEN_PROG)
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", inc, src, "-o", exe], check=True)

    def run(ctr, key):
        # ATen keeps the counter as (offset lo, offset hi, subsequence lo, subsequence hi)
        out = subprocess.run([exe, str(key[0]), str(key[1]), str(ctr[0]), str(ctr[1]), str(ctr[2]), str(ctr[3])],
                             check=True, capture_output=True, text=True).stdout.split()
        return [int(x) for x in out]

    yield run
    shutil.rmtree(d, ignore_errors=True)


def test_philox_matches_aten(aten_philox):
    rng = np.random.default_rng(5)
    cases = [([0, 0, 0, 0], [0, 0]), ([1, 2, 3, 4], [5, 6])]
    for _ in range(14):
        cases.append((list(rng.integers(0, 2**32, 4)), list(rng.integers(0, 2**32, 2))))
    for ctr, key in cases:
        assert oracle.philox4x32_10(ctr, key) == aten_philox(ctr, key), (ctr, key)


@pytest.mark.parametrize("L", [4, 42, 64, 84, 126])
def test_site_draws_are_distinct(L):
    """Each site of a sweep owns its own output word.  A map that let two
    sites share a counter/output slot would produce exact duplicates; chance
    collisions among <= 16k 32-bit values have probability < 3%."""
    for t in (0, 1, 2**32 + 5):
        for stream in (0, 1):
            u = [oracle.site_uniform(99, stream, t, L, r, c) for r in range(L) for c in range(L)]
            assert len(set(u)) == len(u), (L, t, stream)


def test_site_draws_distinct_across_sweeps_and_streams():
    L = 42
    seen = set()
    for t in (0, 1, 2):
        for stream in (0, 1):
            for r in range(L):
                for c in range(L):
                    seen.add(oracle.site_uniform(3, stream, t, L, r, c))
    assert len(seen) == 6 * L * L


def test_site_draws_uniform():
    """Kolmogorov-Smirnov check of one sweep's draws on a lattice with all
    21 positions per word live (L = 1008 = 21 * 48)."""
    from scipy import stats

    L = 1008
    rng = np.random.default_rng(0)
    rs = rng.integers(0, L, 20000)
    cs = rng.integers(0, L, 20000)
    u = np.array([oracle.site_uniform(11, 1, 17, L, int(r), int(c)) for r, c in zip(rs, cs)], dtype=np.float64)
    assert stats.kstest(u / 2.0**32, "uniform").pvalue > 1e-4


def test_word_rows():
    # smallest even N with 21 N >= L; equals L/21 for the paper's sizes with N even
    assert oracle.word_rows(2016) == 96
    assert oracle.word_rows(1008) == 48
    assert oracle.word_rows(4) == 2
    assert oracle.word_rows(64) == 4
    assert oracle.word_rows(4096) == 196
    assert oracle.word_rows(32768) == 1562
    for L in range(4, 3000, 2):
        n = oracle.word_rows(L)
        assert n % 2 == 0 and 21 * n >= L and (n == 2 or 21 * (n - 2) < L)
