"""Host-side logic of bench.py, checked without a GPU: the refusal of more
than one GPU, the roofline arithmetic, the word count of the headline
lattice, the rule that drops stale HBM-traffic counters, and the batched mix
the plain-form sample stands for, and the lane-op fraction every secondary
rate carries."""
import collections
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_headline_word_count():
    # N(L) = smallest even integer >= L / 21 word rows of L words
    # (Section 3): 1562 rows at L = 32768
    assert bench.ising_words_main() == 1562 * 32768 == 51_183_616


def test_roofline_arithmetic():
    avg_ms = 0.2272
    r = bench.roofline(avg_ms, 826_340_317)
    attempts = 32768 ** 2 // 2  # one colour of the lattice per launch
    achieved = 18 * attempts / (avg_ms * 1e-3) / 1e12
    peak = 256 * 4 * 32 * 2.4e9 / 1e12  # 78.64 T lane-ops/s
    assert r["bound"] == "alu" and r["unit"] == "Tops/s"
    assert r["peak"] == pytest.approx(78.64, abs=0.01)
    assert r["achieved"] == pytest.approx(achieved, abs=0.01)
    assert r["frac"] == pytest.approx(achieved / peak, abs=1e-4)
    assert r["traffic"] == 826_340_317
    # one read of the lattice and one write of one colour: 1.5 x 8 bytes per word
    assert r["hbm_gbs_algorithmic"] == pytest.approx(1.5 * 8 * 51_183_616 / (avg_ms * 1e-3) / 1e9, abs=0.1)


def test_traffic_is_dropped_when_stale_or_for_another_plan(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "halfsweep_L32768_traffic.json")) as f:
        d = json.load(f)
    w2 = {"words_per_thread": 2, "block": 256}
    fresh = d["kernel_source_sha256_16"] == bench.kernel_source_hash()
    assert bench.load_traffic(w2) == (d["bytes_per_launch"] if fresh else None)
    assert d["bytes_per_launch"] == d["fetch_bytes_per_launch"] + d["write_bytes_per_launch"]
    # counters taken on a two-words-per-thread launch say nothing of another plan
    assert bench.load_traffic({"words_per_thread": 1, "block": 64}) is None
    # nor of kernels built from other sources
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.load_traffic(w2) is None


def test_batched_mix_holds_every_size_equally():
    Ls, Ts, seeds = bench.batched_config()
    assert len(Ls) == len(Ts) == len(seeds) == 2048
    assert collections.Counter(Ls) == {256: 512, 512: 512, 1024: 512, 2048: 512}
    assert Ls[:4] == [256, 512, 1024, 2048]  # the plain-form sample: one lattice of each size
    assert min(Ts) == pytest.approx(1.5) and max(Ts) == pytest.approx(3.5)
    assert len(set(Ts)) == 32
    assert seeds == list(range(2048))


def test_every_secondary_rate_carries_its_lane_op_fraction():
    # 18 lane-op slots per attempt against 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz
    res = bench.lane_op_fractions({"value": 2251.29, "unit": "attempts/ns",
                                   "plain_same_mix": {"value": 184.46},
                                   "runs": [{"value": 910.0, "p99_s": 0.67}],
                                   "batched_value": 63.0, "plain_value": 0.457, "wall_s": 3.0})
    frac = lambda v: 18 * v / (256 * 4 * 32 * 2.4)
    assert res["lane_op_frac"] == pytest.approx(frac(2251.29), abs=1e-5)
    assert res["plain_same_mix"]["lane_op_frac"] == pytest.approx(frac(184.46), abs=1e-5)
    assert res["runs"][0]["lane_op_frac"] == pytest.approx(frac(910.0), abs=1e-5)
    assert res["batched_lane_op_frac"] == pytest.approx(frac(63.0), abs=1e-5)
    assert res["plain_lane_op_frac"] == pytest.approx(frac(0.457), abs=1e-5)
    assert "wall_s" in res and "lane_op_frac_s" not in res  # only rates get a fraction
