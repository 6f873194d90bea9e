"""The diagnostic library libwcc_timeline.so (include/wcc_timeline.h): it
exports the product ABI plus the timeline calls, the product library does not
export the timeline calls, the summary arithmetic on synthetic records, and
on the GPU a recorded run of the 1D and 2D benchmark workloads."""
import ctypes
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from paper_2104_04347_amd import binding, build, timeline

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def timeline_decls():
    txt = open(os.path.join(ROOT, "include", "wcc_timeline.h")).read()
    return sorted(set(re.findall(r"^int\s+(wcc_timeline_\w+)\s*\(", txt, re.M)))


def test_header_declares_clear_and_read_per_family():
    assert timeline_decls() == sorted(f"wcc_timeline_{op}_{fam}" for op in ("clear", "read")
                                      for fam in ("1d", "1d_wide", "2d"))
    txt = open(os.path.join(ROOT, "include", "wcc_timeline.h")).read()
    assert re.search(r"#define WCC_TIMELINE_WAVES (\d+)", txt).group(1) == str(timeline.WAVES)


def test_timeline_library_exports_product_abi_and_timeline_calls():
    lib = ctypes.CDLL(build.TIMELINE_LIB)
    for name in list(binding.SIGNATURES) + timeline_decls():
        assert hasattr(lib, name), name


def test_product_library_has_no_timeline_calls():
    lib = binding.load()
    for name in timeline_decls():
        assert not hasattr(lib, name), name


def test_summary_of_synthetic_records():
    # 8 waves on 2 SIMDs: each SIMD holds 4 waves over [0, 10) us, the second
    # SIMD's waves living half as long; clocks 1.5 and 2.0 GHz
    rec = np.zeros(timeline.WAVES, dtype=timeline.REC)
    base = 10_000_000
    for w in range(8):
        simd = w // 4
        life_ticks = 1000 if simd == 0 else 500      # 10 us / 5 us at 100 MHz
        mhz = 1500.0 if simd == 0 else 2000.0
        rec[w]["t0"] = base
        rec[w]["t1"] = base + life_ticks
        rec[w]["c0"] = 123
        rec[w]["c1"] = 123 + int(life_ticks / 100e6 * mhz * 1e6)
        rec[w]["hw_id"] = simd << 4
        rec[w]["xcc_id"] = 3
    s = timeline.summarize(rec, launch_us=11.0)
    assert s["waves"] == 8 and s["simds"] == 2 and s["span_us"] == 10.0
    # 4 x 10 + 4 x 5 wave-us over 2 SIMDs x 10 us
    assert s["mean_waves_per_simd"] == 3.0
    # cycle-weighted: (4 x 10 x 1500 + 4 x 5 x 2000) / 60
    assert s["clock_mhz"] == pytest.approx((40 * 1500 + 20 * 2000) / 60, abs=0.1)
    assert s["clock_mhz_p0_10_50_90_100"][0] == 1500.0 and s["clock_mhz_p0_10_50_90_100"][-1] == 2000.0
    assert s["clock_mhz_by_xcd"] == {3: s["clock_mhz"]}


def test_summary_of_short_lived_waves():
    rec = np.zeros(timeline.WAVES, dtype=timeline.REC)
    rec[:2]["t0"] = 1000
    rec[:2]["t1"] = 1050                      # 0.5 us
    rec[:2]["c0"] = 0
    rec[:2]["c1"] = 1000                      # 2 GHz
    s = timeline.summarize(rec, launch_us=1.0)
    assert s["waves"] == 2 and s["clock_mhz"] == 2000.0


def test_summary_refuses_empty_records():
    with pytest.raises(RuntimeError):
        timeline.summarize(np.zeros(timeline.WAVES, dtype=timeline.REC), 1.0)


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["1d", "2d-vortex-lim"])
def test_recorded_run(case):
    # its own process: the diagnostic library replaces the product one there
    cmd = [sys.executable, "-m", "paper_2104_04347_amd.timeline", "--case", case, "--warmup", "4", "--steps", "4",
           "--variant", "0" if case == "1d" else "3"]
    print("timeline run:", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    s = json.loads(r.stdout.strip().splitlines()[-1])
    assert s["waves"] > 256 and s["simds"] > 256
    assert 0 < s["wave_life_us_p0_10_50_90_100"][-1] <= s["span_us"]
    assert 300.0 < s["clock_mhz"] < 3000.0


_SAME_BITS = r"""
import hashlib, sys
import numpy as np
import torch
from paper_2104_04347_amd import binding, inputs
binding.load(sys.argv[1])
h = hashlib.sha256()
q0, _ = inputs.euler_riemann(0, 3, 300)
s = binding.Solver("euler", 3, 300, "transmissive", limiter=True, precision="fp64")
s.write(q0)
s.run(50, 0.25)
q, info = s.read()
h.update(q.tobytes()); h.update(np.float64(info.t).tobytes())
s.close()
q0 = inputs.riemann2d(1, 2, 24)
s = binding.Solver2D("euler", 2, 24, 24, limiter=True, bc="transmissive", x_left=-1.0, x_right=1.0, y_left=-1.0,
                     y_right=1.0)
s.write(q0)
s.run(6, 0.3)
q, info = s.read()
h.update(q.tobytes()); h.update(np.float64(info.t).tobytes())
s.close()
print(h.hexdigest())
"""


@pytest.mark.gpu
def test_diagnostic_build_computes_the_same_bits():
    """The timestamped kernels are the product kernels: 1D and 2D runs give
    the same bits with either library (each in a process of its own)."""
    out = []
    for lib in (build.LIB, build.TIMELINE_LIB):
        print("same-bits run with", lib, flush=True)
        r = subprocess.run([sys.executable, "-c", _SAME_BITS, lib], cwd=ROOT, capture_output=True, text=True,
                           timeout=300)
        assert r.returncode == 0, r.stderr[-3000:]
        out.append(r.stdout.strip().splitlines()[-1])
    assert out[0] == out[1]
