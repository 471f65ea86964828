#!/usr/bin/env python3
"""Benchmark of the multi-spin-coded checkerboard Metropolis sweep on one MI355X.

Headline workload (one "step"): a single L = 32768 lattice (1.07e9 spins,
409.5 MB packed at 21 spins per uint64), hot start with seed 11, run at each
of T = 2.0, 2.269, 2.6 for 2000 sweeps from a fresh start, final E and M read
back -- 3 x 2000 x 32768^2 = 6.44e12 spin-flip attempts per step.  Inputs are
synthetic (generated on the device from the seed); the lattice buffer is
allocated before the timed region.

Printed: ONE JSON line with the contract fields, a `roofline` object for the
dominant kernel (the half-sweep kernel, integer-ALU bound), a `cpu_baseline`
object (the CPU oracle on a bounded sample of the same workload) and a
`secondary` object with the other workloads: the plain one-lattice-per-launch
L = 4096 run, the batched mixed-L run, the L = 64 temperature scan, heating
scans of L = 1008 replicas with the lattice carried over (energy and specific
heat per temperature), the paper's own 101-temperature scan of its L = 84
lattice, the paper's three Table 2 cases run with its own random-pick strip
dynamics, 21 replicas of L = 8192 packed field by field into one word
lattice, and a served request stream with p50/p99 latency (as specified,
at lower rates, and with a device-memory budget small enough that admission
by footprint binds).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "spin-flip attempts/ns (L=32768 single; batched mixed-L) + p50/p99 latency"
UNIT = "attempts/ns"

# Integer-ALU roofline: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz single-slot
# 32-bit lane operations per second, the rate that gives the published
# 157.3 TFLOP/s FP32 vector peak when a lane op is an FMA, and the rate at
# which simple 32-bit vector operations issue (bench.py --valu-rates).
ALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
# Algorithmic integer lane-op slots per spin-flip attempt: a quarter of one
# Philox4x32-10 block (10 rounds x (2 wide 32x32->64 products at 2 slots
# each + 2 three-input XORs) = 60 slots per block -> 15), two threshold
# comparisons, and one slot for the bit-sliced neighbour count and flip.
OPS_PER_ATTEMPT = 18.0
HBM_PEAK_GBS = 8000.0

L_MAIN, SEED_MAIN, TEMPS_MAIN, SWEEPS_MAIN = 32768, 11, (2.0, 2.269, 2.6), 2000


# The instruction-rate microbenchmark (bench_valu_rates.hip beside this file),
# a program of its own built by build_valu_rates() and run by --valu-rates.
VALU_RATES_SRC = os.path.join(ROOT, "bench_valu_rates.hip")
VALU_RATES = os.path.join(ROOT, "bench_valu_rates")


def build_valu_rates(verbose=False):
    """Compile the microbenchmark for gfx950 (hipcc cross-compiles on a host
    without a GPU); returns the program's path."""
    import subprocess

    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = VALU_RATES + ".tmp"
    cmd = [hipcc, "-O3", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", VALU_RATES_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {VALU_RATES_SRC}:\n{r.stdout}{r.stderr}")
    os.replace(tmp, VALU_RATES)
    return VALU_RATES


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _events():
    import torch

    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def run_main(ising, steps, warmup, sweeps):
    import torch

    lat = ising.Lattice(L_MAIN, SEED_MAIN, hot=True)
    wpt, block = lat.plan()
    results = []
    loop_ms = []

    def one_step(record):
        out = []
        for T in TEMPS_MAIN:
            lat.reset(SEED_MAIN, hot=True)
            e0, e1 = _events()
            e0.record()
            lat.sweep(T, sweeps)
            e1.record()
            E, M = lat.observables()  # synchronises the stream
            if record:
                loop_ms.append(e0.elapsed_time(e1))
            out.append({"T": T, "E": E, "M": M, "e_per_spin": E / L_MAIN ** 2, "m_per_spin": M / L_MAIN ** 2})
        return out

    for _ in range(warmup):
        one_step(False)
    torch.cuda.synchronize()
    step_ms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        results = one_step(True)  # ends synchronised (observables)
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lat.close()
    ms_per_step = (t1 - t0) * 1e3 / steps
    attempts = len(TEMPS_MAIN) * sweeps * L_MAIN ** 2
    launches = 2 * sweeps * len(TEMPS_MAIN) * steps
    avg_launch_ms = sum(loop_ms) / launches
    return {
        "ms_per_step": ms_per_step,
        "value": attempts / (ms_per_step * 1e6),
        "avg_halfsweep_ms": avg_launch_ms,
        "step_ms": step_ms,
        "plan": {"words_per_thread": wpt, "block": block},
        "final": results,
    }


def roofline(avg_halfsweep_ms, traffic):
    """The dominant kernel against the integer-ALU peak (`frac`) and against
    the HBM peak: `hbm_frac_algorithmic` from the bytes a half-sweep launch
    must move (every word read once, the updated colour written once: 1.5 x
    the packed lattice), `hbm_frac_counters` from the copy-calibrated
    rocprofv3 FETCH_SIZE + WRITE_SIZE per launch (`traffic`, None when the
    committed counters do not match these kernel sources)."""
    attempts_per_launch = L_MAIN ** 2 / 2
    launch_s = avg_halfsweep_ms * 1e-3
    achieved = OPS_PER_ATTEMPT * attempts_per_launch / launch_s / 1e12
    gbs_alg = 1.5 * 8 * ising_words_main() / launch_s / 1e9
    return {
        "bound": "alu",
        "achieved": round(achieved, 2),
        "peak": round(ALU_PEAK_TOPS, 2),
        "unit": "Tops/s",
        "frac": round(achieved / ALU_PEAK_TOPS, 4),
        "traffic": traffic,
        "kernel": "k_halfsweep_single",
        "ops_per_attempt": OPS_PER_ATTEMPT,
        "attempts_per_launch": attempts_per_launch,
        "avg_launch_ms": round(avg_halfsweep_ms, 5),
        "hbm_gbs_algorithmic": round(gbs_alg, 1),
        "hbm_frac_algorithmic": round(gbs_alg / HBM_PEAK_GBS, 4),
        "hbm_gbs_counters": None if traffic is None else round(traffic / launch_s / 1e9, 1),
        "hbm_frac_counters": None if traffic is None else round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4),
    }


def ising_words_main():
    n = (L_MAIN + 20) // 21
    n += n & 1
    return n * L_MAIN


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in ("ising_device.hpp", "ising_kernels.hip", "ising_common.hpp", "ising_moments.hpp"):
        with open(os.path.join(ROOT, "paper_1811_04384_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(plan):
    """HBM bytes per half-sweep launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE per dispatch, scaled by what the same
    counters read for a copy of known size).  None if the summary is
    missing, was taken on different kernel sources or another plan."""
    path = os.path.join(ROOT, "profiles", "halfsweep_L32768_traffic.json")
    try:
        with open(path) as f:
            d = json.load(f)
        if d.get("kernel_source_sha256_16") != kernel_source_hash():
            return None
        if f"<{plan['words_per_thread']}," not in d["kernel"]:
            return None
        return d["bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(target_s=12.0, single_s=4.0):
    """The CPU oracle on a bounded sample of the headline workload: a
    4096 x 4096 window of the L = 32768 hot-start lattice (seed 11) evolved
    at T = 2.269 for as many sweeps as fit in about target_s seconds on all
    host threads (the per-site work is the same as on the full lattice), and
    a 1024 x 1024 window on one thread for about single_s seconds."""
    import oracle

    L, seed, T = L_MAIN, SEED_MAIN, 2.269

    def rate(w, threads, budget):
        win = oracle.init_window(L, seed, True, 0, 0, w, w)
        done = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget:
            oracle.sweep_window(win, L, seed, done, 2, T, 0, 0, threads=threads)
            done += 2
        dt = time.perf_counter() - t0
        return done * (w - 2) * (w - 2) / (dt * 1e9), done, dt  # the window minus its border

    threads = oracle.max_threads()
    value, done, dt = rate(4096, 0, target_s)
    single, done1, dt1 = rate(1024, 1, single_s)
    return {"value": round(value, 5), "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"4096x4096 window of the L=32768 hot-start lattice (seed 11), T=2.269, {done} sweeps, "
                      f"{dt:.1f} s on {threads} threads",
            "single_thread_value": round(single, 5),
            "single_thread_sample": f"1024x1024 window of the same lattice, {done1} sweeps, {dt1:.1f} s on 1 thread",
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


# ---------------------------------------------------------------------------
# secondary workloads
# ---------------------------------------------------------------------------

def run_plain4096(ising, sweeps=10000, every=10, plain=True):
    """Single lattice L=4096, hot start seed 7, T=2.269, E/M every 10 sweeps,
    one lattice per launch (the plain form), in the library's default plan
    for this size (resident tiles: 256 bands of 16 word columns kept in LDS
    for 1000 sweeps per launch, trading boundary words every half-sweep) and
    with one launch per half-sweep."""
    import torch

    def timed(resident):
        lat = ising.Lattice(4096, 7, hot=True)
        if not resident:
            lat.set_resident_tiles(0)
        plan = {"resident_tiles": lat.resident_tiles(), "half_sweep_plan": lat.plan()}
        lat.sweep_measure(2.269, 100, every)
        lat.reset(7, hot=True)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        E, M = lat.sweep_measure(2.269, sweeps, every)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        e = E.double().mean().item() / 4096 ** 2
        lat.close()
        return ms, e, plan

    ms, e, plan = timed(True)
    out = {"workload": "L=4096 single, hot seed 7, T=2.269, 10000 sweeps, E/M every 10",
           "value": round(4096 ** 2 * sweeps / (ms * 1e6), 2), "unit": UNIT, "ms": round(ms, 2),
           "plan": plan, "mean_e_per_spin": round(e, 6)}
    if plain:
        ms_h, e_h, _ = timed(False)
        assert e == e_h, "the two plans must give the same series"
        out["half_sweep_launches"] = {"value": round(4096 ** 2 * sweeps / (ms_h * 1e6), 2), "ms": round(ms_h, 2)}
    return out


def run_graph4096(ising, sweeps=10000, every=10):
    """The same L=4096 workload through the batch engine with one lattice:
    still one lattice per launch, but the launches replayed from hipGraph
    chunks instead of issued one by one from the host."""
    import torch

    # the launch shape of the plain run's default plan for this size
    b = ising.Batch([4096], [7], hot=True)
    b.set_plan(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=100)
    b.sweep([2.269], 100, every=every)
    b.close()
    b = ising.Batch([4096], [7], hot=True)
    b.set_plan(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=100)
    b.sweep([2.269], 100, every=every)  # capture the chunk graph before timing
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    b.sweep([2.269], sweeps, every=every)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    b.close()
    return {"workload": "L=4096 single, hot seed 7, T=2.269, 10000 sweeps, E/M every 10, graph-replayed launches",
            "value": round(4096 ** 2 * sweeps / (ms * 1e6), 2), "unit": UNIT, "ms": round(ms, 2)}


def batched_config():
    Ls = [(256, 512, 1024, 2048)[i % 4] for i in range(2048)]
    Ts = [1.5 + 2.0 * ((i // 4) % 32) / 31 for i in range(2048)]
    seeds = list(range(2048))
    return Ls, Ts, seeds


def run_batched(ising, sweeps=5000, every=10, autotune=True, plain=True):
    """2048 lattices, L in {256, 512, 1024, 2048} (512 each), 32 temperatures
    over [1.5, 3.5], hot start seed = index, 5000 sweeps, E/M every 10; the
    plan from the autotuner (or the default plan), chunks replayed as
    hipGraphs."""
    import torch

    Ls, Ts, seeds = batched_config()
    b = ising.Batch(Ls, seeds, hot=True)
    cache = os.path.join(os.path.expanduser("~"), ".cache", "ising_msc", "tune.json")
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    t_tune = time.perf_counter()
    plan = b.autotune(Ts, cache) if autotune else b.plan()
    t_tune = time.perf_counter() - t_tune
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    b.sweep(Ts, sweeps, every=every)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    res = b.results()
    spins = sum(L * L for L in Ls)
    b.close()
    value = spins * sweeps / (ms * 1e6)
    out = {"workload": f"2048 lattices L in {{256,512,1024,2048}}, 32 T in [1.5,3.5], hot, {sweeps} sweeps, "
                       f"E/M every 10",
           "value": round(value, 2), "unit": UNIT, "ms": round(ms, 1), "plan": plan,
           "autotune_s": round(t_tune, 2), "samples_per_lattice": int(res["n_samples"][0])}
    if plain:
        out["plain_same_mix"] = run_batched_as_plain(ising, Ls, Ts, seeds, every=every)
        out["batched_over_plain"] = round(value / out["plain_same_mix"]["value"], 2)
    return out


def run_batched_as_plain(ising, Ls, Ts, seeds, sweeps=2000, every=10):
    """The batched mix run the plain way, one lattice per launch and one
    lattice after another, each in the single-lattice default plan for its
    size (resident tiles for all four sizes), on a sample: lattices 0..3 of
    the mix (one of each size, with their seeds and temperatures), 2000
    sweeps each with E/M every 10 (about 60 ms).  The mix holds the four
    sizes in equal numbers, so the sample's rate is the mix's rate."""
    import torch

    lats = [ising.Lattice(Ls[i], seeds[i], hot=True) for i in range(4)]
    for lat, T in zip(lats, Ts[:4]):
        lat.sweep_measure(T, 20, every)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for lat, T in zip(lats, Ts[:4]):
        lat.sweep_measure(T, sweeps, every)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    for lat in lats:
        lat.close()
    return {"sample": f"lattices 0..3 of the mix (L = {', '.join(str(L) for L in Ls[:4])}), {sweeps} sweeps each, "
                      f"E/M every {every}, one lattice per launch, one lattice after another",
            "value": round(sum(L * L for L in Ls[:4]) * sweeps / (ms * 1e6), 2), "unit": UNIT, "ms": round(ms, 2)}


def run_scan64(ising, therm=2000, meas=2000, plain=True):
    """L=64, cold start, 8 temperatures over [1.5, 3.5], seed 1234, 2000 + 2000
    sweeps (sample every measured sweep): batched (codes drawn chip-wide, one
    workgroup per lattice applying them in LDS) and as 8 plain lattices one
    after another, each in the single-lattice default plan (the whole lattice
    in one workgroup, resident in LDS for up to 1000 sweeps per launch)."""
    import torch

    Ts = [1.5 + 2.0 * i / 7 for i in range(8)]
    b = ising.Batch([64] * 8, [1234] * 8, hot=False)
    # the acceptance codes of 2000 sweeps drawn over the whole chip, then
    # applied by one two-wavefront workgroup per lattice (62 attempts/ns
    # measured; drawing them inside each lattice's own workgroup: 16)
    b.set_plan(resident_max_L=64, resident_block=128, words_per_thread=1, tiled_block=256, sweeps_per_graph=2000,
               draw_sweeps=2000)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    b.sweep(Ts, therm)
    b.sweep(Ts, meas, every=1)
    e1.record()
    torch.cuda.synchronize()
    ms_b = e0.elapsed_time(e1)
    res = b.results()
    b.close()
    mean_e = [round(float(s) / n / 64 ** 2, 5) for s, n in zip(res["sum_E"], res["n_samples"])]
    mean_m = [round(float(s) / n / 64 ** 2, 5) for s, n in zip(res["sum_absM"], res["n_samples"])]
    att = 8 * 64 * 64 * (therm + meas)
    if not plain:
        return {"workload": "8 x L=64 cold, seed 1234, T=1.5..3.5, 2000+2000 sweeps",
                "batched_value": round(att / (ms_b * 1e6), 3), "unit": UNIT}
    lats = [ising.Lattice(64, 1234, hot=False) for _ in Ts]
    torch.cuda.synchronize()
    e0.record()
    for lat, T in zip(lats, Ts):
        lat.sweep(T, therm)
        lat.sweep_measure(T, meas, 1)
    e1.record()
    torch.cuda.synchronize()
    ms_p = e0.elapsed_time(e1)
    for lat in lats:
        lat.close()
    att = 8 * 64 * 64 * (therm + meas)
    return {"workload": "8 x L=64 cold, seed 1234, T=1.5..3.5, 2000+2000 sweeps",
            "batched_value": round(att / (ms_b * 1e6), 3), "plain_value": round(att / (ms_p * 1e6), 3),
            "unit": UNIT, "mean_e_per_spin": mean_e, "mean_absm_per_spin": mean_m}


def run_heating_scan(ising, L=1008, replicas=16, therm=500, meas=1000):
    """Heating scans with the lattice carried over from one temperature to
    the next: 16 replicas of the L = 1008 (N = 48) lattice, ordered (cold)
    start, seeds 0..15, T = 1.5, 1.6, ..., 3.5, at each T 500 sweeps to
    re-equilibrate and
    1000 sweeps sampled after each one, exact moment sums on the device.
    Reports the whole-scan throughput and the replica-averaged e(T), c(T)."""
    import torch

    Ts = [round(1.5 + 0.1 * j, 10) for j in range(21)]
    b = ising.Batch([L] * replicas, list(range(replicas)), hot=False)
    # resident tiles of 64 word columns (16 per lattice, one per compute unit)
    # that trade boundary words every half-sweep, 200 sweeps per chunk: the
    # fastest plan measured for this shape (half-sweep launches: 1024 sampled,
    # 1101 unsampled attempts/ns; these tiles 1349 and 1494)
    b.set_plan(resident_max_L=0, resident_block=256, words_per_thread=1, tiled_block=64, sweeps_per_graph=200,
               tile_max_L=L, tile_sweeps=1, tile_cols=64, tile_block=1024, tile_exchange=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = b.scan(Ts, therm, meas, 1)
    wall = time.perf_counter() - t0
    plan = b.plan()
    b.close()
    e_T, c_T = [], []
    for j, T in enumerate(Ts):
        th = [ising.ising_thermodynamics(out[j][r], L, T) for r in range(replicas)]
        e_T.append(round(sum(x["e"] for x in th) / replicas, 5))
        c_T.append(round(sum(x["c"] for x in th) / replicas, 4))
    att = replicas * L * L * len(Ts) * (therm + meas)
    return {"workload": f"{replicas} x L={L} (N=48) cold, heating T=1.5..3.5 step 0.1, {therm}+{meas} sweeps per T",
            "value": round(att / (wall * 1e9), 3), "unit": UNIT, "wall_s": round(wall, 3), "plan": plan,
            "T": Ts, "mean_e_per_spin": e_T, "c_per_spin": c_T, "c_peak_T": Ts[max(range(len(Ts)), key=c_T.__getitem__)]}


def run_paper_scan(ising, L=84, replicas=8, iterations=400, per_iteration=10):
    """The paper's own temperature loop on its demonstration lattice (N = 4,
    L = 84): random start, T = 0.001, 0.101, ..., 10.001 with the lattice
    carried over, at each T 400 iterations of 10 updates per spin (10 sweeps),
    the energy recorded after every iteration and all iterations averaged.
    Eight replicas (seeds 0..7) in one batch."""
    import torch

    Ts = [0.001 + 0.1 * k for k in range(101)]
    b = ising.Batch([L] * replicas, list(range(replicas)), hot=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = b.scan(Ts, 0, iterations * per_iteration, per_iteration)
    wall = time.perf_counter() - t0
    b.close()
    e_T = [sum(out[j][r]["sum_E"] for r in range(replicas)) / (replicas * iterations * L * L) for j in range(len(Ts))]
    att = replicas * L * L * len(Ts) * iterations * per_iteration
    return {"workload": f"{replicas} x L={L} (N=4) hot, T=0.001..10.001 step 0.1 carried over, "
                        f"{iterations} iterations x {per_iteration} sweeps, E after each iteration",
            "value": round(att / (wall * 1e9), 3), "unit": UNIT, "wall_s": round(wall, 3),
            "T_every_5th": [round(T, 3) for T in Ts[::5]], "mean_e_per_spin_every_5th": [round(e, 4) for e in e_T[::5]]}


def run_paper_cases(ising, strip_cols=2, T=2.269, iterations=None):
    """The paper's three test cases (Table 2) with its own dynamics: random
    word picks inside strips of `strip_cols` word columns (L / strip_cols
    processes, each a GPU thread), left half then right half per iteration,
    ten updates per word per iteration, the energy recorded after every
    iteration.  Case 1: N = 96 (L = 2016), 5000 iterations; case 2: N = 96,
    4500 iterations; case 3: N = 48 (L = 1008), 4500 iterations.  Hot start,
    seed = case number, T = 2.269 (the paper gives no temperature for its
    timing runs; the work per iteration does not depend on it)."""
    import torch

    out = {}
    for case, (L, iters) in enumerate(((2016, 5000), (2016, 4500), (1008, 4500)), start=1):
        iters = iterations or iters
        lat = ising.Lattice(L, case, hot=True)
        acc = torch.zeros(10, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        lat.random_iterations(T, strip_cols, iters, 1, acc)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        m = ising.moments_of(acc)
        lat.close()
        att = 10 * L * L * iters
        out[f"case{case}"] = {"L": L, "N": L // 21, "iterations": iters, "processes": L // strip_cols,
                              "value": round(att / (ms * 1e6), 3), "ms_per_iteration": round(ms / iters, 4),
                              "mean_e_per_spin": round(m["sum_E"] / m["n_samples"] / L ** 2, 5)}
    return {"workload": f"Table 2 cases, strip dynamics with {strip_cols}-column strips, T={T}", "unit": UNIT,
            **out}


def run_replicas(ising, L=8192, sweeps=200, seed=21):
    """Replica multi-spin coding: 21 independent L = 8192 lattices (1.41e9
    spins) packed field by field into one 537 MB word lattice, replica k at
    T = 1.5 + 0.1 k, hot start; 200 sweeps, then the 21 replicas' E and M.
    Every words-per-thread plan is timed; the best is reported."""
    import torch

    Ts = [round(1.5 + 0.1 * k, 10) for k in range(21)]
    rep = ising.Replicas(L, seed, hot=True)
    rates = {}
    for wpt in (1, 2, 4):
        rep.set_plan(wpt)
        rep.sweep(Ts, 5)
        torch.cuda.synchronize()
        e0, e1 = _events()
        e0.record()
        rep.sweep(Ts, sweeps)
        e1.record()
        torch.cuda.synchronize()
        rates[wpt] = 21 * L * L * sweeps / (e0.elapsed_time(e1) * 1e6)
    E, M = rep.observables()
    rep.close()
    best = max(rates, key=rates.get)
    return {"workload": f"21 replicas of L={L} in one word lattice, T=1.5..3.5 step 0.1, hot start, {sweeps} sweeps",
            "value": round(rates[best], 2), "unit": UNIT, "words_per_thread": best,
            "by_words_per_thread": {str(k): round(v, 2) for k, v in rates.items()},
            "e_per_spin": [round(int(e) / L ** 2, 4) for e in E]}


SERVING_RATE, SERVING_DURATION, SERVING_QUANTUM, SERVING_SLOTS = 200.0, 60.0, 200, 128
SERVING_BUDGET = 16 << 30


def run_serving(ising, rate=SERVING_RATE, duration=SERVING_DURATION, quantum=SERVING_QUANTUM, seed=2026,
                slots=SERVING_SLOTS, hbm_budget=SERVING_BUDGET):
    """Poisson request stream: L = 2^U{7..12}, T ~ U[1.5, 3.5], sweeps ~
    U{1000..20000}, hot start with seed = request id; continuous batching.
    Latency runs from a request's submission to the read-back of its result;
    the stream is served until every request is done (at 200 req/s the
    offered work is several times what one GPU sustains, so p50/p99 include
    the drain of the queue)."""
    import numpy as np

    rng = np.random.default_rng(seed)
    arrivals = []
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        arrivals.append((t, rid, int(2 ** rng.integers(7, 13)), float(rng.uniform(1.5, 3.5)),
                         int(rng.integers(1000, 20001))))
        rid += 1
    srv = ising.Server(hbm_budget=hbm_budget, max_slots=slots, quantum_sweeps=quantum)
    peak_bytes = peak_resident = 0
    lat_s = []
    attempts = 0
    i = 0
    t0 = time.perf_counter()
    done = 0
    next_report = 10.0
    while done < len(arrivals):
        if time.perf_counter() - t0 > next_report:
            st = srv.stats()
            log(f"  serving t={time.perf_counter() - t0:.0f}s submitted={i} done={done} queued={st['queued']} "
                f"resident={st['resident']}")
            next_report += 10.0
        now = time.perf_counter() - t0
        while i < len(arrivals) and arrivals[i][0] <= now:
            _, r, L, T, sw = arrivals[i]
            srv.submit(r, L, T, sw)
            i += 1
        active = srv.step()
        st = srv.stats()
        peak_bytes = max(peak_bytes, st["bytes_in_use"])
        peak_resident = max(peak_resident, st["resident"])
        for r in srv.poll():
            lat_s.append(r["t_done_s"] - r["t_submit_s"])
            attempts += r["L"] * r["L"] * r["sweeps"]
            done += 1
        if active == 0 and i < len(arrivals):
            time.sleep(max(0.0, min(0.01, arrivals[i][0] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    srv.close()
    lat = np.sort(np.array(lat_s))
    offered = sum(a[2] * a[2] * a[4] for a in arrivals) / (duration * 1e9)
    return {"workload": f"Poisson {rate:g} req/s for {duration:g} s, L=2^U{{7..12}}, T~U[1.5,3.5], "
                        f"sweeps~U{{1000..20000}}, hot start seed = request id",
            "quantum_sweeps": quantum, "resident_slots": slots, "hbm_budget_bytes": hbm_budget,
            "peak_bytes_in_use": peak_bytes, "peak_resident": peak_resident,
            "requests": len(arrivals), "p50_s": round(float(np.percentile(lat, 50)), 3),
            "p99_s": round(float(np.percentile(lat, 99)), 3), "throughput_req_s": round(len(arrivals) / wall, 2),
            "value": round(attempts / (wall * 1e9), 2), "unit": UNIT, "wall_s": round(wall, 2),
            "drain_s": round(wall - duration, 2), "offered_attempts_per_ns": round(offered, 1)}


def run_serving_bounded(ising, rates=(25.0, 50.0, 75.0), duration=10.0, quantum=100):
    """The same stream at lower rates for `duration` seconds each: the
    highest rate the server keeps up with, i.e. whose last request is done
    within 2 s of the end of the arrivals, so that latency stays bounded
    instead of growing with the queue."""
    runs = []
    best = None
    for rate in rates:
        log(f"  serving at {rate:g} req/s for {duration:g} s")
        r = run_serving(ising, rate, duration, quantum)
        runs.append({"rate_req_s": rate, "p50_s": r["p50_s"], "p99_s": r["p99_s"], "drain_s": r["drain_s"],
                     "value": r["value"]})
        if r["drain_s"] <= 2.0:
            best = rate
    return {"workload": f"the served stream at {', '.join(f'{x:g}' for x in rates)} req/s for {duration:g} s each, "
                        f"quantum {quantum}", "highest_bounded_rate_req_s": best, "runs": runs, "unit": UNIT}


def run_serving_small_budget(ising, rate=50.0, duration=10.0, quantum=100, budget=64 << 20):
    """The 50 req/s stream once with the default device-memory budget and
    once with a budget of 64 MiB, which holds about 45 requests of the mean
    footprint (1.4 MB) and 9 of the largest (L = 4096, 6.4 MB): admission by
    footprint then binds before the 128 slots do, and the requests wait in
    the queue for memory instead."""
    out = {"workload": f"Poisson {rate:g} req/s for {duration:g} s (the served stream), device-memory budget "
                       f"{SERVING_BUDGET >> 30} GiB against {budget >> 20} MiB, quantum {quantum}", "unit": UNIT}
    for name, b in (("default_budget", SERVING_BUDGET), ("small_budget", budget)):
        log(f"  serving at {rate:g} req/s with a budget of {b >> 20} MiB")
        r = run_serving(ising, rate, duration, quantum, hbm_budget=b)
        out[name] = {k: r[k] for k in ("hbm_budget_bytes", "peak_bytes_in_use", "peak_resident", "p50_s", "p99_s",
                                       "drain_s", "throughput_req_s", "value")}
    return out


def lane_op_fractions(res):
    """Add, beside every rate (attempts/ns) of a secondary result, its
    fraction of the lane-op roof (OPS_PER_ATTEMPT slots per attempt against
    ALU_PEAK_TOPS), recursing into nested results: the plain and batched forms
    of each workload then both carry a stated fraction of the roofline."""
    if isinstance(res, dict):
        out = {}
        for k, v in res.items():
            out[k] = lane_op_fractions(v)
            if k in ("value", "batched_value", "plain_value") and isinstance(v, (int, float)):
                out[k.replace("value", "lane_op_frac")] = round(OPS_PER_ATTEMPT * v / 1e3 / ALU_PEAK_TOPS, 5)
        return out
    if isinstance(res, list):
        return [lane_op_fractions(x) for x in res]
    return res


def run_secondary(ising, name, args):
    if name == "plain4096":
        return run_plain4096(ising, plain=not args.no_plain)
    if name == "graph4096":
        return run_graph4096(ising)
    if name == "batched":
        return run_batched(ising, sweeps=args.batched_sweeps, autotune=not args.no_autotune, plain=not args.no_plain)
    if name == "scan64":
        return run_scan64(ising, plain=not args.no_plain)
    if name == "heating_scan":
        return run_heating_scan(ising)
    if name == "paper_scan":
        return run_paper_scan(ising)
    if name == "paper_cases":
        return run_paper_cases(ising, iterations=args.paper_iterations)
    if name == "replicas":
        return run_replicas(ising)
    if name == "serving_bounded":
        return run_serving_bounded(ising)
    if name == "serving_small_budget":
        return run_serving_small_budget(ising)
    if name == "serving":
        return run_serving(ising, args.serving_rate, args.serving_duration, args.serving_quantum,
                           slots=args.serving_slots)
    raise SystemExit(f"unknown workload {name}")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=SWEEPS_MAIN, help="sweeps per temperature (headline: 2000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--secondary",
                    default="plain4096,graph4096,batched,scan64,heating_scan,paper_scan,paper_cases,replicas,"
                            "serving_bounded,serving_small_budget,serving",
                    help="comma list of secondary workloads, or 'none'")
    ap.add_argument("--serving-rate", type=float, default=SERVING_RATE)
    ap.add_argument("--serving-duration", type=float, default=SERVING_DURATION)
    ap.add_argument("--serving-sweep", default="", metavar="RATES",
                    help="only run the served stream at each comma-separated rate (req/s) for --serving-duration "
                         "seconds and print one JSON line per rate")
    ap.add_argument("--serving-quantum", type=int, default=SERVING_QUANTUM)
    ap.add_argument("--serving-slots", type=int, default=SERVING_SLOTS,
                    help="requests resident at once (the rest wait in FIFO order)")
    ap.add_argument("--valu-rates", action="store_true",
                    help="only run the instruction-rate microbenchmark (cycles per wave64 instruction of the "
                         "vector instructions the half-sweep uses) and print its JSON line")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run 10 device-to-device copies of BYTES bytes (HBM counter calibration)")
    ap.add_argument("--only", default="", metavar="WORKLOADS",
                    help="run only these comma-separated secondary workloads (no headline, no CPU baseline) and "
                         "print one JSON line with their results (for profiling one kernel at a time)")
    ap.add_argument("--batched-sweeps", type=int, default=5000,
                    help="sweeps of the batched mix (5000 as specified; fewer for a profiling run)")
    ap.add_argument("--paper-iterations", type=int, default=None, metavar="N",
                    help="run each of the paper's Table 2 cases for N iterations instead of its own count "
                         "(for counter runs)")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the one-launch-per-half-sweep comparisons of the L = 4096 lattice, the batched "
                         "mix and the L = 64 scan (tens of thousands of short launches; for counter runs)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="run the batched mix in its default plan instead of the autotuned one")
    ap.add_argument("--build-valu-rates", action="store_true",
                    help="only compile the instruction-rate microbenchmark (no GPU needed) and exit")
    args = ap.parse_args()

    if args.build_valu_rates:
        print(build_valu_rates(verbose=True))
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the lattice kernels run on a single MI355X and there is no "
              "multi-GPU path (a single lattice would shard by word-column strips with one boundary-column "
              "exchange per half-sweep; batches and served requests by whole lattices).", file=sys.stderr)
        sys.exit(2)

    if args.valu_rates:  # a child process of its own, started before this one touches the GPU
        import subprocess

        prog = VALU_RATES
        if not os.path.exists(prog):
            print(f"{prog} is not built (python bench.py --build-valu-rates)", file=sys.stderr)
            sys.exit(1)
        r = subprocess.run([prog], capture_output=True, text=True, timeout=300)
        log(r.stdout + r.stderr)
        lines = [x for x in r.stdout.splitlines() if x.startswith("{")]
        if r.returncode != 0 or not lines:
            sys.exit(r.returncode or 1)
        print(lines[-1], flush=True)
        return

    import torch

    import paper_1811_04384_amd as ising

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ising.load()
    torch.cuda.set_device(0)
    if args.serving_sweep:
        for rate in [float(x) for x in args.serving_sweep.split(",")]:
            log(f"serving at {rate:g} req/s for {args.serving_duration:g} s")
            print(json.dumps({"rate_req_s": rate, "quantum": args.serving_quantum, "slots": args.serving_slots,
                              **run_serving(ising, rate, args.serving_duration, args.serving_quantum,
                                            slots=args.serving_slots)}), flush=True)
        return
    if args.copy_probe:
        src = torch.empty(args.copy_probe // 4, dtype=torch.int32, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe, "copies": 10}), flush=True)
        return

    if args.only:
        out = {}
        for name in args.only.split(","):
            log(f"only: {name}")
            out[name] = lane_op_fractions(run_secondary(ising, name, args))
            log(f"  {out[name]}")
        print(json.dumps({"only": out}), flush=True)
        return

    log(f"headline: L={L_MAIN} x T={TEMPS_MAIN} x {args.sweeps} sweeps, warmup {args.warmup}, steps {args.steps}")
    main_res = run_main(ising, args.steps, args.warmup, args.sweeps)
    log(f"headline: {main_res['value']:.1f} attempts/ns, {main_res['ms_per_step']:.1f} ms/step")
    traffic = load_traffic(main_res["plan"])

    secondary = {}
    wanted = [] if args.secondary == "none" else args.secondary.split(",")
    for name in wanted:
        log(f"secondary: {name}")
        secondary[name] = lane_op_fractions(run_secondary(ising, name, args))
        log(f"  {secondary.get(name)}")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline()

    line = {
        "metric": METRIC,
        "value": round(main_res["value"], 2),
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 2),
        "step_ms": [round(x, 2) for x in main_res["step_ms"]],
        "value_median_step": round(len(TEMPS_MAIN) * args.sweeps * L_MAIN ** 2
                                   / (sorted(main_res["step_ms"])[len(main_res["step_ms"]) // 2] * 1e6), 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic (Philox hot start on the device)",
        "config": {
            "workload": f"single lattice L=32768, hot start seed 11, T in {{2.0, 2.269, 2.6}}, "
                        f"{args.sweeps} sweeps each, final E/M",
            "L": L_MAIN, "temperatures": list(TEMPS_MAIN), "sweeps_per_T": args.sweeps, "seed": SEED_MAIN,
            "plan": main_res["plan"], "parallelism": "single GPU",
        },
        "roofline": roofline(main_res["avg_halfsweep_ms"], traffic),
        "cpu_baseline": cpu,
        "final_observables": main_res["final"],
        "secondary": secondary,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
