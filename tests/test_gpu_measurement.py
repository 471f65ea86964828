"""The measurement tools run on the GPU: the instruction-rate microbenchmark
prints one line per instruction and a JSON summary whose figures are
plausible issue costs (cycles per wave64 instruction per SIMD)."""
import json
import subprocess

import pytest

from bench import VALU_RATES

pytestmark = pytest.mark.gpu


def test_valu_rates_reports_every_instruction():
    print("valu_rates microbenchmark", flush=True)
    r = subprocess.run([VALU_RATES], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    summary = json.loads([x for x in r.stdout.splitlines() if x.startswith("{")][-1])
    cycles = summary["cycles"]
    assert summary["cus"] > 0 and summary["clock_mhz"] > 0
    for name in ("v_add_u32 (v)", "v_bitop3_b32 (s)", "v_mad_u64_u32 (s)", "v_cndmask_b32_e64 (s mask)"):
        assert name in cycles, name
    # a wave64 instruction needs at least one cycle of a SIMD and, with the
    # SIMD kept busy by 8 wavefronts, far fewer than 50
    assert all(0.5 < c < 50 for c in cycles.values()), cycles
