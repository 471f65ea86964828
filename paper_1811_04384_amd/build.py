"""Compile the gfx950 library ``libising.so`` in-tree with hipcc.

    python -m paper_1811_04384_amd.build        # or python paper_1811_04384_amd/build.py
"""
import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libising.so")
ARCH = "gfx950"

SOURCES = [s for s in ["ising_kernels.hip", "ising_tiles.hip", "ising_persist.hip", "ising_small.hip", "ising_drawahead.hip",
                       "ising_static.hip",
                       "ising_strips.hip", "ising_replicas.hip",
                       "ising_lattice.cpp",
                       "ising_batch.cpp", "ising_server.cpp", "ising_replicas.cpp"]
           if os.path.exists(os.path.join(CSRC, s))]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"--offload-arch={ARCH}",
          "-I", os.path.join(HERE, "..", "include")]
# packed-FP32 instructions are never generated (no float math on the hot path,
# and the forms of them are avoided altogether)
DEVICE_ONLY = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def source_hash() -> str:
    """Hash of every source the library is built from (csrc/ and the C
    header); the build embeds it in ising_version() so that a library built
    from other sources is refused when loaded."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".hpp", ".cpp", ".h")))
    for f in files + ["../../include/ising.h"]:
        h.update(f.encode())
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _compile(src, verbose, defines):
    obj = os.path.join(BUILD, src.replace(".", "_") + ".o")  # x.hip and x.cpp get distinct objects
    cmd = ([HIPCC] + COMMON + defines + (DEVICE_ONLY if src.endswith(".hip") else []) +
           ["-c", os.path.join(CSRC, src), "-o", obj])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in line and "is not a recognized feature" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msgs}")
    if verbose and msgs.strip():
        print(msgs)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    defines = [f'-DISING_SOURCE_HASH="{source_hash()}"']
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, defines), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
