#!/usr/bin/env python3
"""Benchmark of the WCC half-step on one MI355X.

Workload (the headline configuration): 1D Euler, gamma = 1.4, on [0, 1] with
N = 1,048,576 mesh intervals, degree P = 3 (4th order), seeded Riemann data
(rho ~ U(0.1, 1), u ~ U(-1, 1), p ~ U(0.1, 1) on each side of x = 0.5) with the
density sine rho*(1 + 0.2 sin 5x), transmissive ends, limiter on (characteristic
variables), CFL 0.25 per half-step.  A step is one half-step of the whole path
(expansion, flux integral, average and derivative update, limiter, wave speed,
time control) over all cells; inputs are resident in HBM before timing starts.

Printed: one JSON line.  `value` is cell-DOF updates per second in binary64
(the bit-exact mode); the FP32-mixed mode, the batched workload (4096 uneven
instances, solves/s for 100 half-steps each) and the oracle's CPU timing are
reported beside it, with the roofline of the dominant kernel measured live with
HIP events on the stream the kernels run on.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12          # bytes/s, MI355X HBM3E
FP64_VALU_PEAK = 78.6e12   # flop/s, fma counted as 2
# binary32 without packed instructions (this build compiles with the packed
# FP32 operations disabled): one 64-lane instruction per 4 cycles per SIMD,
# the binary64 rate
FP32_VALU_PEAK = 78.6e12
# VALU issue: 256 CUs x 4 SIMDs, one 64-lane (wave) VALU instruction per 4
# cycles per SIMD at the 2.4 GHz peak engine clock
N_SIMD = 1024
CLOCK_HZ = 2.4e9
CYCLES_PER_VALU_INST = 4
VALU_ISSUE_PEAK = N_SIMD * CLOCK_HZ / CYCLES_PER_VALU_INST   # wave-instructions/s
MALL_BYTES = 256 * 1048576  # Infinity Cache (MALL) of the MI355X
CFL_BY_P = [0.4, 0.4, 0.3, 0.25, 0.25]


def measured_traffic(kernel: str, N: int, sources: str = "1d"):
    """HBM bytes per launch from the committed counter record (FETCH_SIZE and
    WRITE_SIZE, scaled by the copy-kernel calibration), or None when the
    record is for another kernel build or size."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2104_04347_amd.profsum import kernel_source_hash
    e = rec.get(kernel)
    if not e or e.get("source_sha256") != kernel_source_hash(sources) or e.get("N") != N:
        return None
    return e["fetch_bytes"] + e["write_bytes"]


def valu_insts(kernel: str, N: int, sources: str = "1d"):
    """Mean SQ_INSTS_VALU (64-lane VALU instructions) per launch from the
    committed counter record, or None when it is for another build or size."""
    path = os.path.join(ROOT, "profiles", "valu_insts.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2104_04347_amd.profsum import kernel_source_hash
    e = rec.get(kernel)
    if not e or e.get("source_sha256") != kernel_source_hash(sources) or e.get("N") != N:
        return None
    return e["sq_insts_valu"]


def shader_clock(kernel: str, N: int, sources: str = "1d"):
    """Shader clock (MHz) that the per-wave timeline measured for this kernel
    on the benchmark's workload (the committed record: 0.2 s of back-to-back
    half-steps, possibly on another box), or None when the record is for
    another build or size."""
    path = os.path.join(ROOT, "profiles", "clock.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    from paper_2104_04347_amd.profsum import kernel_source_hash
    e = rec.get(kernel)
    if not e or e.get("source_sha256") != kernel_source_hash(sources) or e.get("N") != N:
        return None
    return e["clock_mhz"]


def issue_roof(kernel: str, N: int, launch_s: float, sources: str = "1d"):
    """VALU issue roof: the launch's VALU instructions at one per 4 cycles on
    every SIMD at the peak clock, against the measured launch time; with a
    committed clock record, also at the clock the waves ran at."""
    insts = valu_insts(kernel, N, sources)
    if insts is None:
        return None
    t_issue = insts / VALU_ISSUE_PEAK
    out = {"bound": "alu", "unit": "Ginst/s", "achieved": round(insts / launch_s / 1e9, 1),
           "peak": round(VALU_ISSUE_PEAK / 1e9, 1), "frac": round(t_issue / launch_s, 4),
           "valu_insts_per_launch": insts, "issue_floor_us": round(t_issue * 1e6, 2)}
    mhz = shader_clock(kernel, N, sources)
    if mhz:
        at = VALU_ISSUE_PEAK * (mhz * 1e6 / CLOCK_HZ)
        out |= {"shader_clock_mhz": mhz, "peak_at_clock": round(at / 1e9, 1),
                "frac_at_clock": round(insts / at / launch_s, 4)}
    return out


def flop_counts():
    with open(os.path.join(ROOT, "paper_2104_04347_amd", "flop_counts.json")) as f:
        return json.load(f)["counts"]


def cells_updated(N: int, bc: str, parity0: int, steps: int) -> int:
    """New cells written over `steps` half-steps starting on mesh parity0."""
    if bc == "periodic":
        return N * steps
    tot, par = 0, parity0
    for _ in range(steps):
        tot += N if par == 0 else N + 1   # original (N+1 cells) -> staggered (N) and back
        par ^= 1
    return tot


def bytes_per_launch(N: int, P: int, nc: int, precision: str) -> float:
    """Algorithmic HBM bytes of one half-step: every old cell read once and
    every new cell written once (point value in binary64, derivatives in the
    bulk type).  Averaged over the two parities of a transmissive run."""
    b_cell = nc * (8 + P * (8 if precision == "fp64" else 4))
    n_old_plus_new = 2 * N + 1
    return float(n_old_plus_new * b_cell)


def launch_shape_single(args, s, q0, cfl=None, **tune_kw) -> dict:
    """Launch shape of the single-instance kernel: a cached autotuner result
    when there is one (and --tune is not 'force'), else tune now (--tune off:
    the library's default).  Results do not depend on the shape."""
    from paper_2104_04347_amd import autotune
    if getattr(args, "c3_variant", -1) >= 0 and cfl is None:
        s.set_launch(256, 0, args.c3_variant)
        return {**s.get_launch(), "tile": autotune.TILE_SHAPE[args.c3_variant], "source": "--c3-variant"}
    if args.tune == "off":
        return {**s.get_launch(), "source": "library default"}
    if args.tune == "auto" and autotune.apply_single(s):
        c = autotune.cached_single(s)
        v = c.get("variant", 0)
        return {"threads": c["threads"], "blocks": c["blocks"], "variant": v, "tile": autotune.TILE_SHAPE[v],
                "source": "autotune cache"}
    best = autotune.tune_single(s, q0, args.cfl if cfl is None else cfl, **tune_kw)
    return {"threads": best["threads"], "blocks": best["blocks"], "variant": best["variant"], "tile": best["tile"],
            "source": "autotuned",
            "best_us_per_variant": {str(v): round(ms * 1e3, 2) for v, ms in best["per_variant_ms"].items()}}


def kernel_record(precision: str, P: int, variant: int):
    """Key and source set of the counter records of the 1D Euler kernel."""
    from paper_2104_04347_amd import records
    return records.key_1d(precision, P, variant)


def time_single(args, precision: str, q0, keep_state: bool = False):
    import torch
    from paper_2104_04347_amd import binding
    P, N = args.P, args.N
    s = binding.Solver("euler", P, N, "transmissive", limiter=True, precision=precision)
    shape = launch_shape_single(args, s, q0)
    s.write(q0)
    s.run(args.warmup, args.cfl)
    torch.cuda.synchronize()
    parity0 = s.info().parity
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    s.run(args.steps, args.cfl)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_ms = e0.elapsed_time(e1)
    lib_ms = s.last_run_ms()
    info = s.info()
    ok = (info.flags & 3) == 0
    cells = cells_updated(N, "transmissive", parity0, args.steps)
    dofs = cells * 3 * (P + 1)
    out = dict(value=dofs / wall, wall_s=wall, event_ms=ev_ms, lib_event_ms=lib_ms, flags=int(info.flags),
               ok=ok, t=info.t, half_steps=int(info.half_steps), launch=shape)
    if keep_state:
        out["q"] = s.read()[0]
    s.close()
    return out


def mixed_vs_fp64(q_mixed, q_fp64) -> dict:
    """Point-value L1 (mean) and Linf distance of the FP32-mixed result from
    the binary64 result (itself bit for bit the FP64 oracle's), per
    component, relative to the largest |value| of the binary64 field."""
    d = q_mixed[:, 0] - q_fp64[:, 0]
    scale = np.abs(q_fp64[:, 0]).max(axis=1)
    return {"L1_rel": [float(np.abs(d[c]).mean() / scale[c]) for c in range(d.shape[0])],
            "Linf_rel": [float(np.abs(d[c]).max() / scale[c]) for c in range(d.shape[0])]}


def time_batch(args):
    import torch
    from paper_2104_04347_amd import binding, inputs
    spec = inputs.batch_spec(args.batch_B, args.seed)
    bt = binding.Batch("euler", spec.P, spec.N, "transmissive", limiter=True, precision="fp32_mixed")
    from paper_2104_04347_amd import autotune

    def load_instances(again=False):
        if again:
            bt.rebind()
        for b in range(spec.P.size):
            bt.write(b, inputs.batch_instance(spec, b))
        bt.prepare()

    load_instances()
    sched = None
    if args.batch_schedule:
        sched = [int(v) for v in args.batch_schedule.split(",")]
        bt.set_schedule(*sched)
    elif args.tune != "off":
        c = autotune.cached_batch(bt) if args.tune == "auto" else None
        if c is None:
            c = autotune.tune_batch(bt, CFL_BY_P)
            load_instances(again=True)            # time from the initial state again
        sched = [c["threads"], c["blocks"], c["mode"]]
        bt.set_schedule(*sched)
    bt.run(args.batch_warmup, CFL_BY_P)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt.run(args.batch_steps, CFL_BY_P)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = bt.last_run_ms()
    flags = 0
    for b in range(0, spec.P.size, max(1, spec.P.size // 64)):
        flags |= bt.read(b)[1].flags & 3
    cells = int(np.sum(spec.N)) * args.batch_steps          # ~N per half-step per instance
    dofs = int(np.sum(spec.N * 3 * (spec.P + 1))) * args.batch_steps
    # algorithmic bytes of one half-step of every instance (old + new cells)
    bph = sum(bytes_per_launch(int(n), int(p), 3, "fp32_mixed") for n, p in zip(spec.N, spec.P))
    gbs = bph * args.batch_steps / (ms / 1e3) / 1e9
    out = dict(value=spec.P.size / wall, unit="solves/s", instances=int(spec.P.size),
               half_steps_each=args.batch_steps, wall_s=wall, event_ms=ms, cell_dof_per_s=dofs / wall,
               total_cells=int(np.sum(spec.N)), cells_per_s=cells / wall, bytes_per_half_step=bph,
               gbs=round(gbs, 1), hbm_frac=round(gbs * 1e9 / HBM_PEAK, 4), flags=int(flags),
               schedule=sched or "default")
    # the single-launch form: every instance's half-step in ONE persistent
    # launch (fused schedules 1 and 3: direct / staged stores), timed the same way
    fused = {}
    for mode in args.batch_fused_modes:
        load_instances(again=True)
        bt.set_schedule(sched[0] if sched else 256, 0, mode)
        bt.run(args.batch_warmup, CFL_BY_P)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt.run(args.batch_steps, CFL_BY_P)
        torch.cuda.synchronize()
        w = time.perf_counter() - t0
        m = bt.last_run_ms()
        g = bph * args.batch_steps / (m / 1e3) / 1e9
        fl = 0
        for b in range(0, spec.P.size, max(1, spec.P.size // 64)):
            fl |= bt.read(b)[1].flags & 3
        fused[str(mode)] = {"value": spec.P.size / w, "unit": "solves/s", "event_ms": m,
                            "launches_per_half_step": 1, "gbs": round(g, 1),
                            "hbm_frac": round(g * 1e9 / HBM_PEAK, 4), "flags": int(fl)}
        print(f"[bench] batched, one launch per half-step (mode {mode}): {spec.P.size / w:.1f} solves/s",
              file=sys.stderr, flush=True)
    if fused:
        out["one_launch_form"] = fused
    bt.close()
    return out


def time_2d(args):
    """The 2D half-step (Section 3): Burgers with the limiter, P = 3, on a
    2048 x 2048 periodic mesh of [0, 2]^2 with seeded sine modes; and the
    Euler isentropic vortex of Table 3, P = 3, 1024 x 1024 on [-5, 5]^2,
    unlimited (LCCS) and with the rotated characteristic limiter (WCCS); the
    first 2D Riemann problem of Section 5.3 with 1200 x 1200 intervals on
    [-1, 1]^2, transmissive edges, limited, P = 3.
    Binary64; launch shape from the autotuner (row-marching variant, threads,
    grid; --tune off: the library's default).
    Algorithmic bytes per launch: every old cell read once and every new cell
    written once, nc * ndof doubles each; `traffic` is the measured HBM bytes
    per launch from the committed counter record (null if it is stale)."""
    import torch
    from paper_2104_04347_amd import binding, inputs
    out = {}
    cases = [("burgers_lim_P3", "burgers", 3, args.n2d, True, (0.0, 2.0, 0.0, 2.0), 0.25,
              lambda: inputs.taylor2d(inputs.modes2d(args.seed), 3, args.n2d, args.n2d)),
             ("euler_vortex_P3", "euler", 3, args.n2d_euler, False, (-5.0, 5.0, -5.0, 5.0), 0.25,
              lambda: inputs.isentropic_vortex(3, args.n2d_euler)),
             ("euler_vortex_lim_P3", "euler", 3, args.n2d_euler, True, (-5.0, 5.0, -5.0, 5.0), 0.25,
              lambda: inputs.isentropic_vortex(3, args.n2d_euler)),
             ("riemann2d_1_lim_P3", "euler", 3, args.n2d_riemann, True, (-1.0, 1.0, -1.0, 1.0), 0.25,
              lambda: inputs.riemann2d(1, 3, args.n2d_riemann))]
    from paper_2104_04347_amd import autotune
    for name, eq, P, N, lim, dom, cfl, make in cases:
        q0 = make()
        bc = "transmissive" if name.startswith("riemann") else "periodic"
        s = binding.Solver2D(eq, P, N, N, limiter=lim, x_left=dom[0], x_right=dom[1], y_left=dom[2], y_right=dom[3],
                             bc=bc)
        # launch shape: the library's default (row marching with prefetch and
        # band-major work items, 256 threads, device-filling grid), a cached
        # autotuner result, or tune now
        launch = {"variant": 3, "threads": 256, "blocks": 0, "source": "library default"}
        if args.tune != "off":
            c = autotune.cached_2d(s) if args.tune == "auto" else None
            if c is None:
                c = autotune.tune_2d(s, q0, cfl)
                launch = {k: c[k] for k in ("variant", "threads", "blocks")} | {
                    "source": "autotuned",
                    "best_us_per_variant": {str(v): round(ms * 1e3, 2) for v, ms in c["per_variant_ms"].items()}}
            else:
                launch = {k: c[k] for k in ("variant", "threads", "blocks")} | {"source": "autotune cache"}
            s.set_launch(launch["threads"], launch["blocks"], launch["variant"])
        s.write(q0)
        s.run(args.warmup2d, cfl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(args.steps2d, cfl)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launch_s = s.last_run_ms() / 1e3 / args.steps2d
        info = s.info()
        nc, nd = s.nc, s.nd
        # cells per half-step: N^2 on both meshes (periodic); (N+1)^2 and N^2
        # alternately (transmissive), averaged
        cells = N * N if bc == "periodic" else 0.5 * ((N + 1) ** 2 + N * N)
        dofs = cells * nc * nd * args.steps2d
        bpl = 2.0 * cells * nc * nd * 8
        from paper_2104_04347_amd import records
        kernel = records.kernel_2d(eq, P, lim, launch["variant"])
        # the counter record belongs to the kernel, the mesh and the launch
        # grid (the grid sets how many priming rows are re-read)
        eff = s.get_launch()                   # the grid actually launched (0 resolved)
        rec_key = records.key_2d(eq, P, lim, launch["variant"], bc == "periodic", eff["threads"], eff["blocks"])
        e = {"value": dofs / wall, "unit": "cell-DOF updates/s", "N": N, "P": P, "limiter": lim, "bc": bc,
             "cfl": cfl, "half_steps": args.steps2d, "kernel": kernel, "launch": launch, "launch_us": launch_s * 1e6,
             "bytes_per_launch": bpl, "hbm_frac": bpl / launch_s / HBM_PEAK,
             "traffic": measured_traffic(rec_key, N, "2d"), "traffic_key": rec_key,
             "issue_roof": issue_roof(rec_key, N, launch_s, "2d"),
             "valid": bool((info.flags & 3) == 0)}
        s.close()
        if not args.no_cpu:
            import oracle
            pb = oracle.Problem2D(eq, P, N, N, limiter=lim, x_left=dom[0], x_right=dom[1], y_left=dom[2],
                                  y_right=dom[3], bc=bc)
            t0 = time.perf_counter()
            r = oracle.run2d(pb, q0, cfl=cfl, max_half_steps=1)
            cw = time.perf_counter() - t0
            # one half-step from parity 0: N x N new cells on either boundary
            e["cpu_baseline"] = {"value": N * N * nc * nd * r.half_steps / cw, "unit": "cell-DOF updates/s",
                                 "cores": 1, "kind": "oracle",
                                 "sample": f"first half-step of the same workload, FP64 oracle, single thread, "
                                           f"{cw:.1f} s"}
        out[name] = e
        del q0
        print(f"[bench] 2D {name}: {e['value']:.3e} DOF/s", file=sys.stderr, flush=True)
    return out


def cpu_baseline_batch(args):
    """The FP64 oracle on one half-step of every instance of the batched
    workload, the instances spread over all host threads (the oracle's C
    calls release the interpreter lock, so a thread pool runs them in
    parallel; the oracle keeps no shared mutable state), and the same on one
    thread for every 8th instance.  The cost of a half-step does not depend
    on which one it is, so solves/s for `batch_steps` half-steps is
    extrapolated from it."""
    import concurrent.futures as cf
    import oracle
    from paper_2104_04347_amd import inputs
    spec = inputs.batch_spec(args.batch_B, args.seed)
    oracle.threads()                      # load the serial build before the threads start
    jobs = []
    for b in range(spec.P.size):
        P, N = int(spec.P[b]), int(spec.N[b])
        jobs.append((oracle.Problem("euler", P, N, bc="transmissive", limiter=True), inputs.batch_instance(spec, b),
                     CFL_BY_P[P], cells_updated(N, "transmissive", 0, 1) * 3 * (P + 1)))

    def one(j):
        oracle.run(j[0], j[1], cfl=j[2], max_half_steps=1)

    nt = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=nt) as ex:
        list(ex.map(one, jobs))
    wall = time.perf_counter() - t0
    dofs = sum(j[3] for j in jobs)
    sub = jobs[::8]
    t0 = time.perf_counter()
    for j in sub:
        one(j)
    w1 = time.perf_counter() - t0
    d1 = sum(j[3] for j in sub)
    return {"value": spec.P.size / (wall * args.batch_steps), "unit": "solves/s",
            "cell_dof_per_s": dofs / wall, "cores": nt, "kind": "oracle",
            "sample": f"one half-step of each of the {spec.P.size} instances, instances spread over {nt} threads "
                      f"({wall:.1f} s), scaled to {args.batch_steps} half-steps per solve",
            "single_thread": {"cell_dof_per_s": d1 / w1, "cores": 1,
                              "value": spec.P.size / (dofs / (d1 / w1) * args.batch_steps), "unit": "solves/s",
                              "sample": f"one half-step of every 8th instance ({len(sub)}), one thread, {w1:.1f} s; "
                                        f"solves/s from its cell-DOF rate"}}


def time_large(args):
    """Large 1D Euler: N = 16,777,216, P = 4, 8 seeded jumps with 9 states and
    the density sine, periodic, CFL 0.20 per half-step, `large_steps`
    half-steps in FP32-mixed and in binary64.  Reports throughput, the
    conserved-total drift of the mixed run and its L1/Linf distance from the
    binary64 run."""
    import torch
    from paper_2104_04347_amd import binding, inputs
    N, P, cfl = args.large_N, 4, 0.20
    q0, _ = inputs.euler_multi_jump(args.seed, P, N, n_jumps=8, bc="periodic")
    out = {"config": f"1D Euler N={N}, P={P}, 8 jumps, periodic, CFL {cfl}, {args.large_steps} half-steps"}
    finals = {}
    for prec in ("fp32_mixed", "fp64"):
        s = binding.Solver("euler", P, N, "periodic", limiter=True, precision=prec)
        if args.large_variant >= 0:
            s.set_launch(256, 0, args.large_variant)
            shape = {"threads": 256, "blocks": 0, "variant": args.large_variant, "source": "--large-variant"}
        else:
            # kernel variant only (a short tune: each candidate costs ~1 ms per half-step)
            shape = launch_shape_single(args, s, q0, cfl, steps=96, threads=(256,), block_factors=(0,))
        s.write(q0)
        tot0 = s.totals()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(args.large_steps, cfl)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        tot = s.totals()
        q, info = s.read()
        finals[prec] = q[:, 0].copy()
        abs0 = np.abs(q0[:, 0]).sum(axis=1) * (1.0 / N)   # scale of the totals
        launch_s = s.last_run_ms() / 1e3 / args.large_steps
        # periodic: N old + N new cells per launch
        bpl = 2.0 * N * 3 * (8 + P * (8 if prec == "fp64" else 4))
        out[prec] = {"value": N * 3 * (P + 1) * args.large_steps / wall, "unit": "cell-DOF updates/s",
                     "wall_s": wall, "ms_per_step": s.last_run_ms() / args.large_steps, "t": info.t,
                     "launch": shape, "launch_us": round(launch_s * 1e6, 2), "bytes_per_launch": bpl,
                     "gbs": round(bpl / launch_s / 1e9, 1), "frac": round(bpl / launch_s / HBM_PEAK, 4),
                     "mall_resident": bool(bpl <= MALL_BYTES),
                     "flags": int(info.flags),
                     "drift_rel": [float(abs(a - b) / c) for a, b, c in zip(tot, tot0, abs0)]}
        del q
        s.close()
    if not args.no_cpu and args.large_cpu_steps > 0:
        import oracle
        from oracle import build as obuild
        pb = oracle.Problem("euler", P, N, bc="periodic", limiter=True)
        with oracle.use_library(obuild.LIB_OMP):
            nt = oracle.threads()
            t0 = time.perf_counter()
            r = oracle.run(pb, q0, cfl=cfl, max_half_steps=args.large_cpu_steps)
            wall = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": N * 3 * (P + 1) * r.half_steps / wall, "unit": "cell-DOF updates/s",
                               "cores": nt, "kind": "oracle",
                               "sample": f"first {r.half_steps} half-steps of the large workload, FP64 oracle "
                                         f"(OpenMP build, {nt} threads), {wall:.1f} s"}
    d = finals["fp32_mixed"] - finals["fp64"]
    scale = np.abs(finals["fp64"]).max(axis=1)
    out["mixed_vs_fp64_point_values"] = {"L1_rel": [float(np.abs(d[c]).mean() / scale[c]) for c in range(3)],
                                         "Linf_rel": [float(np.abs(d[c]).max() / scale[c]) for c in range(3)],
                                         "t_fp64": out["fp64"]["t"], "t_fp32_mixed": out["fp32_mixed"]["t"]}
    return out


def cpu_baseline(args, q0):
    """The FP64 oracle as it stands on a bounded sample of the same workload
    (the first half-steps of the full mesh): the OpenMP build of the same
    source on all host threads (`value`), and the serial build on one thread."""
    import oracle
    from oracle import build as obuild
    pb = oracle.Problem("euler", args.P, args.N, bc="transmissive", limiter=True)

    def timed(lib, steps):
        with oracle.use_library(lib):
            nt = oracle.threads()
            t0 = time.perf_counter()
            r = oracle.run(pb, q0, cfl=args.cfl, max_half_steps=steps)
            wall = time.perf_counter() - t0
        dofs = cells_updated(args.N, "transmissive", 0, r.half_steps) * 3 * (args.P + 1)
        return dofs / wall, nt, r.half_steps, wall

    v1, _, n1, w1 = timed(obuild.LIB, args.cpu_steps)
    vm, nt, nm, wm = timed(obuild.LIB_OMP, args.cpu_omp_steps)
    cpu_model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu_model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": vm, "unit": "cell-DOF updates/s", "cores": nt, "kind": "oracle",
            "sample": f"first {nm} half-steps of the full workload (N={args.N}, P={args.P}), FP64 oracle, "
                      f"OpenMP build over cells, {nt} threads, {wm:.1f} s",
            "single_thread": {"value": v1, "unit": "cell-DOF updates/s", "cores": 1, "kind": "oracle",
                              "sample": f"first {n1} half-steps, serial build, {w1:.1f} s"},
            "cpu_model": cpu_model, "host_threads": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed half-steps")
    ap.add_argument("--warmup", type=int, default=480, help="untimed half-steps first (clocks settle, graphs built)")
    ap.add_argument("--P", type=int, default=3)
    ap.add_argument("--N", type=int, default=1 << 20)
    ap.add_argument("--cfl", type=float, default=0.25)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-p2", action="store_true", help="skip the P = 2 legs of the benchmark workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--batch-B", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--batch-warmup", type=int, default=24)
    ap.add_argument("--batch-schedule", default="", help="threads,blocks,mode for the batched kernels")
    ap.add_argument("--batch-fused-modes", default="1,3",
                    help="also time these fused (one launch per half-step) batch schedules ('' for none)")
    ap.add_argument("--cpu-steps", type=int, default=12, help="serial oracle half-steps timed")
    ap.add_argument("--cpu-omp-steps", type=int, default=48, help="OpenMP oracle half-steps timed")
    ap.add_argument("--large-cpu-steps", type=int, default=2,
                    help="OpenMP oracle half-steps timed on the large workload")
    ap.add_argument("--no-2d", action="store_true", help="skip the 2D legs")
    ap.add_argument("--n2d", type=int, default=2048, help="2D Burgers mesh (n2d x n2d)")
    ap.add_argument("--n2d-euler", type=int, default=1024, help="2D Euler vortex mesh")
    ap.add_argument("--n2d-riemann", type=int, default=1200, help="2D Riemann problem mesh (intervals per side)")
    ap.add_argument("--steps2d", type=int, default=240)
    ap.add_argument("--warmup2d", type=int, default=96)
    ap.add_argument("--seeds", default="0,1,2,3,4",
                    help="also time the FP64 and mixed legs on these seeds of the same workload ('' for none)")
    ap.add_argument("--no-large", action="store_true", help="skip the large 16.7M-cell P=4 workload")
    ap.add_argument("--large-N", type=int, default=1 << 24)
    ap.add_argument("--large-steps", type=int, default=10000)
    ap.add_argument("--large-variant", type=int, default=-1, choices=(-1, 0, 1, 2, 3),
                    help="launch variant of the large workload (256 threads, default grid); -1: per --tune")
    ap.add_argument("--c3-variant", type=int, default=-1, choices=(-1, 0, 1, 2, 3, 4),
                    help="pin the launch variant of the N=2^20 legs (256 threads, default grid; counter passes)")
    ap.add_argument("--tune", choices=("auto", "force", "off"), default="auto",
                    help="launch shapes: cached autotuner result else tune (auto), always tune, or library default")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="also run 5 device-to-device copies of this many MiB (counter calibration)")
    args = ap.parse_args()
    args.batch_fused_modes = [int(v) for v in args.batch_fused_modes.split(",") if v.strip()]

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library has no multi-GPU path; run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_04347_amd import binding, inputs
    if not torch.cuda.is_available():
        print("bench.py needs the GPU", file=sys.stderr)
        sys.exit(1)
    binding.load()
    torch.cuda.set_device(0)

    q0, _ = inputs.euler_riemann(args.seed, args.P, args.N)
    print(f"[bench] workload ready: Euler P={args.P} N={args.N}", file=sys.stderr, flush=True)
    r64 = time_single(args, "fp64", q0, keep_state=not args.no_mixed)
    print(f"[bench] fp64: {r64['value']:.3e} DOF/s", file=sys.stderr, flush=True)
    rmx = None
    if not args.no_mixed:
        rmx = time_single(args, "fp32_mixed", q0, keep_state=True)
        print(f"[bench] fp32_mixed: {rmx['value']:.3e} DOF/s", file=sys.stderr, flush=True)
        rmx["vs_fp64"] = mixed_vs_fp64(rmx.pop("q"), r64.pop("q"))
        rmx["vs_fp64"].update(t_fp64=r64["t"], t_fp32_mixed=rmx["t"],
                              half_steps=r64["half_steps"])
    seeds_out = {}
    for sd in [int(v) for v in args.seeds.split(",") if v.strip()]:
        if sd == args.seed:
            continue
        qs, _ = inputs.euler_riemann(sd, args.P, args.N)
        e = {"fp64": time_single(args, "fp64", qs)["value"]}
        if not args.no_mixed:
            e["fp32_mixed"] = time_single(args, "fp32_mixed", qs)["value"]
        seeds_out[str(sd)] = e
        print(f"[bench] seed {sd}: fp64 {e['fp64']:.3e} DOF/s", file=sys.stderr, flush=True)
    if seeds_out:
        seeds_out[str(args.seed)] = {"fp64": r64["value"], **({"fp32_mixed": rmx["value"]} if rmx else {})}
    # the same workload at P = 2 (CFL 0.3 per half-step), both precisions
    rp2 = None
    if not args.no_p2:
        import copy
        a2 = copy.copy(args)
        a2.P, a2.cfl, a2.c3_variant = 2, 0.3, -1
        q2, _ = inputs.euler_riemann(args.seed, 2, args.N)
        rp2 = {}
        for prec in ("fp64",) + (() if args.no_mixed else ("fp32_mixed",)):
            r = time_single(a2, prec, q2)
            bpl = bytes_per_launch(args.N, 2, 3, prec)
            ls = r["lib_event_ms"] / 1e3 / args.steps
            rp2[prec] = {"value": r["value"], "unit": "cell-DOF updates/s", "ms_per_step": r["wall_s"] * 1e3 / args.steps,
                         "launch_us": round(ls * 1e6, 2), "bytes_per_launch": bpl,
                         "hbm_frac": round(bpl / ls / HBM_PEAK, 4), "mall_resident": bool(bpl <= MALL_BYTES),
                         "valid": bool(r["ok"]), "launch": r["launch"]}
            print(f"[bench] P=2 {prec}: {r['value']:.3e} DOF/s", file=sys.stderr, flush=True)
        del q2

    rb = None
    if not args.no_batch:
        rb = time_batch(args)
        print(f"[bench] batched: {rb['value']:.1f} solves/s", file=sys.stderr, flush=True)

    r2 = None
    if not args.no_2d:
        try:
            r2 = time_2d(args)
        except Exception as exc:          # reported, never hides the 1D line
            r2 = {"error": f"{type(exc).__name__}: {exc}"}
            print(f"[bench] 2D legs failed: {exc}", file=sys.stderr, flush=True)

    rl = None
    if not args.no_large:
        rl = time_large(args)
        print(f"[bench] large: mixed {rl['fp32_mixed']['value']:.3e} DOF/s, fp64 {rl['fp64']['value']:.3e} DOF/s",
              file=sys.stderr, flush=True)

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 5 x {nbytes} bytes", file=sys.stderr, flush=True)

    counts = flop_counts()
    fl = counts[f"euler/P{args.P}/lim"]["flops"]

    def roof(r, precision):
        launch_s = (r["lib_event_ms"] / 1e3) / args.steps
        bpl = bytes_per_launch(args.N, args.P, 3, precision)
        cells_per_launch = args.N + 0.5
        bw = bpl / launch_s
        flops = fl * cells_per_launch / launch_s
        peak_alu = FP64_VALU_PEAK if precision == "fp64" else FP32_VALU_PEAK
        return dict(launch_us=launch_s * 1e6, bytes_per_launch=bpl, gbs=bw / 1e9, hbm_frac=bw / HBM_PEAK,
                    tflops=flops / 1e12, alu_frac=flops / peak_alu, alu_peak=peak_alu)

    ro = roof(r64, "fp64")
    # the counter records are per kernel variant (prefetch / staged stores / tile shape)
    kernel_key, ksrc = kernel_record("fp64", args.P, r64["launch"]["variant"])
    launch_s = ro["launch_us"] / 1e6
    issue = issue_roof(kernel_key, args.N, launch_s, ksrc)
    # the binding roof is the one with the longer floor: algorithmic bytes at
    # the HBM peak, or the measured VALU instructions at the issue peak
    t_hbm = ro["bytes_per_launch"] / HBM_PEAK
    bound_hbm = issue is None or t_hbm >= issue["issue_floor_us"] / 1e6
    hbm = {"bound": "hbm", "achieved": round(ro["gbs"], 1), "peak": HBM_PEAK / 1e9, "unit": "GB/s",
           "frac": round(ro["hbm_frac"], 4), "traffic": measured_traffic(kernel_key, args.N, ksrc),
           # old + new state fit the Infinity Cache: the bytes are served from
           # it, so this is not a fraction of HBM bandwidth actually used
           "mall_resident": bool(ro["bytes_per_launch"] <= MALL_BYTES)}
    roofline = {**(hbm if bound_hbm else issue),
                "kernel": kernel_key,
                "launch_us": round(ro["launch_us"], 2),
                "bytes_per_launch": ro["bytes_per_launch"],
                "issue_roof": issue,
                "hbm_roof": hbm,
                "flop_roof": {"bound": "alu", "achieved": round(ro["tflops"], 3), "unit": "TFLOP/s",
                              "peak": FP64_VALU_PEAK / 1e12, "frac": round(ro["alu_frac"], 4),
                              "note": "algorithmic flops (fma = 2, a division or square root = 1)"}}
    if not bound_hbm:
        roofline["traffic"] = hbm["traffic"]

    line = {
        "metric": "cell-DOF updates/s, 1D Euler P=3 (FP64 vs FP32-mixed); batched solves/s",
        "value": r64["value"],
        "unit": "cell-DOF updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"1D Euler gamma=1.4, N={args.N}, P={args.P}, seeded Riemann (seed {args.seed}) "
                               f"+ density sine, transmissive, limiter on, CFL {args.cfl} per half-step",
                   "N": args.N, "P": args.P, "precision": "fp64", "parallelism": "single GPU"},
        "valid": bool(r64["ok"]),
        "launch": r64["launch"],
        "roofline": roofline,
    }
    if rmx is not None:
        rm = roof(rmx, "fp32_mixed")
        mkey, msrc = kernel_record("fp32_mixed", args.P, rmx["launch"]["variant"])
        line["fp32_mixed"] = {"value": rmx["value"], "unit": "cell-DOF updates/s", "dtype": "f32 bulk + f64 average",
                              "ms_per_step": rmx["wall_s"] * 1e3 / args.steps, "valid": bool(rmx["ok"]),
                              "launch_us": round(rm["launch_us"], 2), "hbm_frac": round(rm["hbm_frac"], 4),
                              "mall_resident": bool(rm["bytes_per_launch"] <= MALL_BYTES),
                              "gbs": round(rm["gbs"], 1), "tflops": round(rm["tflops"], 3),
                              "issue_roof": issue_roof(mkey, args.N, rm["launch_us"] / 1e6, msrc),
                              "vs_fp64": rmx["vs_fp64"], "launch": rmx["launch"]}
    if rp2 is not None:
        line["P2"] = {"config": f"the same workload at P = 2, CFL 0.3 per half-step", **rp2}
    if rb is not None:
        line["batched"] = rb
    if r2 is not None:
        line["two_d"] = r2
    if rl is not None:
        line["large"] = rl
    if seeds_out:
        line["seeds"] = seeds_out
    if not args.no_cpu:
        print("[bench] CPU baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(args, q0)
        if rb is not None:
            print("[bench] CPU baseline, batched workload (oracle) ...", file=sys.stderr, flush=True)
            line["batched"]["cpu_baseline"] = cpu_baseline_batch(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
