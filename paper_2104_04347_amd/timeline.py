"""Per-wave timeline of the half-step kernels from the diagnostic library
libwcc_timeline.so (include/wcc_timeline.h): wave lifetimes, how many waves
share a SIMD over a launch, and the shader clock the waves ran at.

The kernel trace gives a launch's duration; an instruction-issue roof also
needs the clock the SIMDs ran at, which under a sustained binary64 load sits
well below the 2.4 GHz peak engine clock.  Each wave's record holds the
constant 100 MHz clock and the shader clock counter at its entry and exit;
their ratio over the wave's life is its clock.

Run as a program, in a process of its own (it loads the diagnostic library in
place of the product one):

    python -m paper_2104_04347_amd.timeline --case 1d [--precision fp32_mixed]
    python -m paper_2104_04347_amd.timeline --case 2d-vortex-lim

The workload of each case is the benchmark leg of the same name (sizes,
initial data, CFL number); the launch shape is the autotuner's cached one when
the cache holds it, else the library default, unless --variant/--threads/
--blocks are given.  The records are cleared before the state is written;
then `--warmup` and `--steps` half-steps run back to back with no host
synchronisation between them, so the clock has settled under the sustained
load; the records hold the last launch and the launch time is the mean over
the last `--steps`.  (The state write stamps only the exit of its wave-speed
kernel's waves; records without an entry stamp are ignored.)
`--record` stores the clock in profiles/clock.json under the kernel's record
key (the key of its counter records), stamped with the SHA-256 of the kernel
sources (the diagnostic build compiles the same sources), for the
benchmark's issue roof.
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os
import sys

import numpy as np

from paper_2104_04347_amd import binding, build, inputs, records

REC = np.dtype([("t0", "<u8"), ("t1", "<u8"), ("c0", "<u8"), ("c1", "<u8"), ("hw_id", "<u4"), ("xcc_id", "<u4"),
                ("pad", "<u4", 2)])
assert REC.itemsize == 48
WAVES = 16384
RT_HZ = 100e6  # s_memrealtime
CFL_1D = 0.25
SEED = 0   # the benchmark's default seed of the 2D Burgers data

CASES_2D = {
    # name: equation, P, N, limiter, domain, boundaries, cfl, initial data
    "2d-burgers": ("burgers", 3, 2048, True, (0.0, 2.0, 0.0, 2.0), "periodic", 0.25,
                   lambda: inputs.taylor2d(inputs.modes2d(SEED), 3, 2048, 2048)),
    "2d-vortex": ("euler", 3, 1024, False, (-5.0, 5.0, -5.0, 5.0), "periodic", 0.25,
                  lambda: inputs.isentropic_vortex(3, 1024)),
    "2d-vortex-lim": ("euler", 3, 1024, True, (-5.0, 5.0, -5.0, 5.0), "periodic", 0.25,
                      lambda: inputs.isentropic_vortex(3, 1024)),
    "2d-riemann": ("euler", 3, 1200, True, (-1.0, 1.0, -1.0, 1.0), "transmissive", 0.25,
                   lambda: inputs.riemann2d(1, 3, 1200)),
}


def load() -> ctypes.CDLL:
    lib = binding.load(build.TIMELINE_LIB)
    if not hasattr(lib, "wcc_timeline_read_1d"):
        raise RuntimeError("the product library is loaded in this process; run the timeline in a process of its own")
    for fam in ("1d", "1d_wide", "2d"):
        getattr(lib, f"wcc_timeline_clear_{fam}").argtypes = []
        getattr(lib, f"wcc_timeline_read_{fam}").argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    return lib


def clear(lib, fam: str) -> None:
    rc = getattr(lib, f"wcc_timeline_clear_{fam}")()
    if rc:
        raise RuntimeError(f"wcc_timeline_clear_{fam}: {rc}")


def read(lib, fam: str) -> np.ndarray:
    buf = np.zeros(WAVES, dtype=REC)
    rc = getattr(lib, f"wcc_timeline_read_{fam}")(ctypes.c_void_p(buf.ctypes.data), buf.nbytes)
    if rc:
        raise RuntimeError(f"wcc_timeline_read_{fam}: {rc}")
    return buf


def summarize(rec: np.ndarray, launch_us: float) -> dict:
    """Waves that stamped both ends in the last launch: their lives, the
    residency of waves per SIMD over the launch, and the shader clock."""
    r = rec[(rec["t0"] > 0) & (rec["t1"] > rec["t0"])]
    if len(r) == 0:
        raise RuntimeError("no wave records: was a half-step run with this library?")
    t0 = r["t0"].astype(np.int64)
    t1 = r["t1"].astype(np.int64)
    c = (r["c1"] - r["c0"]).astype(np.float64)
    life_us = (t1 - t0) / RT_HZ * 1e6
    base = t0.min()
    span_us = (t1.max() - base) / RT_HZ * 1e6
    hw = r["hw_id"].astype(np.int64)
    simd = (r["xcc_id"].astype(np.int64) & 15) << 16 | (hw >> 4 & 3) | (hw >> 8 & 15) << 2 | (hw >> 12 & 0xF) << 6
    nsimd = len(np.unique(simd))
    # clocks from waves that lived at least 1 us (100 ticks of the constant
    # clock), unless none did
    long_ = life_us >= 1.0
    if not long_.any():
        long_ = np.ones_like(long_)
    mhz = c / ((t1 - t0) / RT_HZ) / 1e6
    xcc = r["xcc_id"].astype(np.int64) & 15
    pct = lambda a, q: [round(float(x), 2) for x in np.percentile(a, q)]   # noqa: E731
    out = {
        "waves": int(len(r)), "simds": int(nsimd), "launch_us": round(launch_us, 2), "span_us": round(span_us, 2),
        "wave_life_us_p0_10_50_90_100": pct(life_us, [0, 10, 50, 90, 100]),
        "wave_end_us_p0_10_50_90_100": pct((t1 - base) / RT_HZ * 1e6, [0, 10, 50, 90, 100]),
        "mean_waves_per_simd": round(float(life_us.sum() / (nsimd * span_us)), 3),
        # life-weighted mean: total shader cycles over total wave time
        "clock_mhz": round(float(c[long_].sum() / ((t1 - t0)[long_].sum() / RT_HZ) / 1e6), 1),
        "clock_mhz_p0_10_50_90_100": pct(mhz[long_], [0, 10, 50, 90, 100]),
        "clock_mhz_by_xcd": {int(x): round(float(c[long_ & (xcc == x)].sum() /
                                                ((t1 - t0)[long_ & (xcc == x)].sum() / RT_HZ) / 1e6), 1)
                             for x in np.unique(xcc[long_])},
    }
    return out


def run_1d(lib, args) -> tuple:
    P, N = 3, 1 << 20
    q0, _ = inputs.euler_riemann(0, P, N)
    s = binding.Solver("euler", P, N, "transmissive", limiter=True, precision=args.precision)
    shape = _shape_1d(s, args)
    fam = "1d_wide" if shape["variant"] == 4 else "1d"
    clear(lib, fam)
    s.write(q0)
    s.run(args.warmup, CFL_1D)
    s.run(args.steps, CFL_1D)
    _sync()
    launch_us = s.last_run_ms() * 1e3 / args.steps
    rec = read(lib, fam)
    s.close()
    return {"case": "1d", "workload": f"Euler P=3 N=2^20 transmissive limiter {args.precision}", **shape}, rec, \
        launch_us


def _shape_1d(s, args) -> dict:
    from paper_2104_04347_amd import autotune
    if args.variant is None:
        c = autotune.cached_single(s)
        if c:
            s.set_launch(c["threads"], c["blocks"], c.get("variant", -1))
    else:
        s.set_launch(args.threads, args.blocks, args.variant)
    return s.get_launch()


def run_2d(lib, args) -> tuple:
    from paper_2104_04347_amd import autotune
    eq, P, N, lim, dom, bc, cfl, make = CASES_2D[args.case]
    q0 = make()
    s = binding.Solver2D(eq, P, N, N, limiter=lim, x_left=dom[0], x_right=dom[1], y_left=dom[2], y_right=dom[3],
                         bc=bc)
    if args.variant is None:
        c = autotune.cached_2d(s)
        if c:
            s.set_launch(c["threads"], c["blocks"], c["variant"])
    else:
        s.set_launch(args.threads, args.blocks, args.variant)
    shape = s.get_launch()
    clear(lib, "2d")
    s.write(q0)
    s.run(args.warmup, cfl)
    s.run(args.steps, cfl)
    _sync()
    launch_us = s.last_run_ms() * 1e3 / args.steps
    rec = read(lib, "2d")
    s.close()
    return {"case": args.case, "workload": f"{eq} P={P} {N}x{N} {bc} {'limiter' if lim else 'no limiter'}",
            **shape}, rec, launch_us


def _sync() -> None:
    import torch
    torch.cuda.synchronize()


def record(key: str, sources: str, N: int, summary: dict, path: str | None = None) -> None:
    """Store the measured clock under `key` in profiles/clock.json, stamped
    with the kernel sources' hash."""
    from paper_2104_04347_amd.profsum import kernel_source_hash
    path = path or os.path.join(os.path.dirname(build.HERE), "profiles", "clock.json")
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        d = {}
    d[key] = {"source_sha256": kernel_source_hash(sources), "N": N, "clock_mhz": summary["clock_mhz"],
              "clock_mhz_p0_10_50_90_100": summary["clock_mhz_p0_10_50_90_100"],
              "launch_us": summary["launch_us"], "mean_waves_per_simd": summary["mean_waves_per_simd"]}
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--case", required=True, choices=["1d", *CASES_2D])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_mixed"])
    ap.add_argument("--variant", type=int, default=None)
    ap.add_argument("--threads", type=int, default=256)
    ap.add_argument("--blocks", type=int, default=0)
    ap.add_argument("--warmup", type=int, default=0, help="half-steps before the recorded run (default per case)")
    ap.add_argument("--steps", type=int, default=0, help="half-steps of the recorded run (default per case)")
    ap.add_argument("--record", action="store_true", help="store the clock in profiles/clock.json")
    args = ap.parse_args(argv)
    one_d = args.case == "1d"
    # about 0.2 s of back-to-back half-steps before the recorded ones
    args.warmup = args.warmup or (5000 if one_d else 1000)
    args.steps = args.steps or (200 if one_d else 20)
    lib = load()
    head, rec, launch_us = (run_1d if one_d else run_2d)(lib, args)
    summary = {**head, **summarize(rec, launch_us)}
    print(json.dumps(summary), flush=True)
    if args.record:
        if one_d:
            key, src = records.key_1d(args.precision, 3, head["variant"])
            N = 1 << 20
        else:
            eq, P, N, lim, _, bc, _, _ = CASES_2D[args.case]
            key, src = records.key_2d(eq, P, lim, head["variant"], bc == "periodic", head["threads"],
                                      head["blocks"]), "2d"
        record(key, src, N, summary)


if __name__ == "__main__":
    main(sys.argv[1:])
