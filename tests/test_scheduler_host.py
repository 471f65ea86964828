"""The server's scheduling core (ising_sched.hpp) on the host, without a GPU:
admission by memory footprint in arrival order, slot reuse, arena
fragmentation and merging, per-quantum sweep accounting."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_driver")
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    os.path.join(ROOT, "tests", "sched_driver.cpp"), "-o", exe], check=True)

    def run(cmds, budget=1 << 20, slots=4, quantum=10):
        out = subprocess.run([exe, str(budget), str(slots), str(quantum)], input="\n".join(cmds) + "\n",
                             capture_output=True, text=True, check=True)
        return out.stdout.split("\n")[:-1]

    return run


def test_fifo_admission_respects_budget_and_slots(driver):
    out = driver(["submit 1 300 5", "submit 2 300 5", "submit 3 300 5", "submit 4 100 5", "admit", "stats"],
                 budget=1024, slots=4)
    assert out[:4] == ["ok"] * 4
    # 300 rounds to 512: two fit in 1024; request 3 blocks (no overtaking by request 4)
    assert out[4] == "admitted 0:1@0 1:2@512"
    assert out[5] == "stats 2 2 1024"


def test_oversized_request_is_rejected(driver):
    assert driver(["submit 1 5000 1"], budget=4096) == ["reject"]


def test_slots_limit_and_reuse(driver):
    cmds = [f"submit {i} 10 {5 * (i + 1)}" for i in range(4)] + ["admit", "quantum", "retire 0", "admit", "stats"]
    out = driver(cmds, budget=1 << 16, slots=2, quantum=5)
    assert out[4] == "admitted 0:0@0 1:1@256"
    assert out[5] == "finished 0:0"  # request 0 needs 5 sweeps = one quantum
    assert out[7] == "admitted 0:2@0"  # slot 0 and its memory reused
    assert out[8] == "stats 1 2 512"


def test_quantum_accounting(driver):
    out = driver(["submit 7 10 23", "admit", "quantum", "quantum", "quantum"], quantum=10)
    assert out[2:] == ["finished", "finished", "finished 0:7"]


def test_arena_merges_freed_ranges(driver):
    cmds = ["submit 1 256 1", "submit 2 256 1", "submit 3 256 1", "submit 4 256 1", "admit",
            "quantum", "retire 1", "retire 2", "submit 5 512 1", "admit", "stats"]
    out = driver(cmds, budget=1024, slots=8)
    assert out[4] == "admitted 0:1@0 1:2@256 2:3@512 3:4@768"
    assert out[9] == "admitted 1:5@256"  # the two freed neighbours merged into one 512-byte range
    assert out[10] == "stats 0 3 1024"
