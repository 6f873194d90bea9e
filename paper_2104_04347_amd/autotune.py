"""Launch-shape autotuner for the WCC half-step kernels.

Results never depend on the launch shape (every tile runs the same per-cell
arithmetic; the batched kernels are checked bit for bit against
single-instance runs in both schedules), so the tuner only measures time:

* single instance: kernel variant (prefetch, staged line-aligned stores,
  both, neither) x threads per block (64..256) x blocks per launch
  (multiples of the device's resident-block capacity);
* 2D: row-marching variant x threads x blocks per launch;
* batched: schedule mode (fused: one launch per half-step switching on the
  degree per tile; grouped: one launch per degree, in sequence or as
  parallel graph branches; each with or without staged stores) x threads x
  blocks.

Each candidate is timed with HIP events around graph-replayed half-steps on
the caller's stream, after a warm-up; the fastest few are then re-timed
round-robin (`refine`) and the one with the smallest median wins.  The best
shape is cached in a JSON file
(``$WCC_AUTOTUNE_CACHE``, default ``~/.cache/wcc_autotune.json``) keyed by
equation, degree, precision, limiter and a power-of-two size bucket.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import binding


def cache_path() -> str:
    return os.environ.get("WCC_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache",
                                                             "wcc_autotune.json"))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_cache(c: dict) -> None:
    """Best effort: a cache that cannot be written only costs a re-tune."""
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
        tmp = p + ".tmp"
        with open(tmp, "w") as f:
            json.dump(c, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def key_single(equation: str, P: int, N: int, precision: str, limiter: bool) -> str:
    return f"single/{equation}/P{P}/{precision}/{'lim' if limiter else 'nolim'}/N2^{int(np.log2(max(N, 2)))}"


# wave-tile shape of each single-instance launch variant: old cells per tile
# and per lane (variants 0-3 differ in prefetch and staged stores only)
TILE_SHAPE = {0: "64x1", 1: "64x1", 2: "64x1", 3: "64x1", 4: "128x2"}


def refine(candidates: list, time_one, top: int = 4, rounds: int = 3) -> dict:
    """Second stage of every tuner: re-time the `top` fastest candidates of
    the sweep `rounds` times each, round-robin with the order rotated every
    round, and return the one with the smallest median.  A single timing of
    a candidate carries the GPU's clock transitions after the idle gaps
    between candidates (up to ~10% either way), enough to pick a shape that
    is slower in steady state; interleaving and the median spread those
    transitions over the finalists.  time_one(c) -> ms per half-step.  Each
    finalist gets `refined_ms` (the median) and `refined_all`."""
    pool = sorted(candidates, key=lambda c: c["ms_per_step"])[:max(1, top)]
    times = [[] for _ in pool]
    for r in range(rounds):
        for j in range(len(pool)):
            i = (j + r) % len(pool)
            times[i].append(time_one(pool[i]))
    for c, t in zip(pool, times):
        c["refined_all"] = t
        c["refined_ms"] = float(np.median(t))
    return min(pool, key=lambda c: c["refined_ms"])


def tune_single(solver: "binding.Solver", q0: np.ndarray, cfl: float, steps: int = 480,
                threads=(128, 256), block_factors=(0, 2, 3, 4, 5, 6, 8), variants=(0, 1, 2, 3, 4),
                verbose: bool = False) -> dict:
    """Time the candidate shapes on `solver` (state q0, CFL cfl); keep the best.
    Blocks per launch = block factor x compute units; factor 0 = the
    library's default (resident-block capacity)."""
    import torch
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    default = solver.get_launch()          # the library's choice for this size
    results = []
    for var in variants:
        for th in threads:
            for bf in block_factors:
                blocks = 0 if bf == 0 else max(1, int(round(bf * cu)))
                solver.set_launch(th, blocks, var)
                solver.write(q0)
                solver.run(48, cfl)            # warm-up, builds the graphs of this shape
                torch.cuda.synchronize()
                solver.run(steps, cfl)
                ms = solver.last_run_ms()
                results.append({"variant": var, "threads": th, "blocks": blocks, "ms_per_step": ms / steps})
                if verbose:
                    print(f"  variant={var} threads={th:4d} blocks={blocks:6d}: {ms / steps * 1e3:8.2f} us/half-step",
                          flush=True)
    def time_one(c):
        solver.set_launch(c["threads"], c["blocks"], c["variant"])
        solver.write(q0)
        solver.run(48, cfl)
        torch.cuda.synchronize()
        solver.run(steps, cfl)
        return solver.last_run_ms() / steps

    default_ms = time_one(default)
    per_variant = {v: min(r["ms_per_step"] for r in results if r["variant"] == v) for v in variants}
    finalists = [r for r in results if (r["variant"], r["threads"], r["blocks"]) !=
                 (default["variant"], default["threads"], default["blocks"])]
    best = refine(finalists + [{**default, "ms_per_step": default_ms, "is_default": True}], time_one)
    best = {k: v for k, v in best.items() if k not in ("refined_all",)}
    best["ms_per_step"] = best.pop("refined_ms")
    best["default_ms_per_step"] = default_ms
    best["per_variant_ms"] = per_variant
    best["tile"] = TILE_SHAPE[best["variant"]]
    best["tried"] = results
    c = _load_cache()
    c[key_single(solver.equation, solver.P, solver.N, binding.PRECISIONS_NAME[solver.params.precision],
                 bool(solver.params.limiter))] = {k: best[k] for k in ("variant", "tile", "threads", "blocks",
                                                                      "ms_per_step")}
    _save_cache(c)
    solver.set_launch(best["threads"], best["blocks"], best["variant"])
    return best


def cached_single(solver: "binding.Solver"):
    """The cached shape for `solver`'s configuration, or None."""
    return _load_cache().get(key_single(solver.equation, solver.P, solver.N,
                                        binding.PRECISIONS_NAME[solver.params.precision],
                                        bool(solver.params.limiter)))


def key_batch(batch: "binding.Batch") -> str:
    return f"batch/B{batch.B}/{binding.PRECISIONS_NAME[batch.params.precision]}"


def cached_batch(batch: "binding.Batch"):
    """The cached schedule for `batch`'s size and precision, or None."""
    return _load_cache().get(key_batch(batch))


def apply_single(solver: "binding.Solver") -> bool:
    """Apply a cached shape to `solver` if one exists; returns whether it did."""
    k = key_single(solver.equation, solver.P, solver.N, binding.PRECISIONS_NAME[solver.params.precision],
                   bool(solver.params.limiter))
    c = _load_cache().get(k)
    if not c:
        return False
    solver.set_launch(c["threads"], c["blocks"], c.get("variant", -1))
    return True


def tune_batch(batch: "binding.Batch", cfl_by_P, steps: int = 24, modes=(1, 2, 3, 4, 5, 6),
               threads=(128, 256), block_factors=(0, 1, 2, 4), verbose: bool = False) -> dict:
    """Time batched schedules on a batch whose instances are written and
    prepared.  Candidates run consecutively from the evolving state (the cost
    of a half-step does not depend on which half-step it is)."""
    import torch
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    results = []
    for mode in modes:
        for th in threads:
            for bf in block_factors:
                blocks = 0 if bf == 0 else max(1, int(round(bf * cu)))
                batch.set_schedule(th, blocks, mode)
                batch.run(steps, cfl_by_P)          # warm-up, builds the graphs of this schedule
                torch.cuda.synchronize()
                batch.run(steps, cfl_by_P)
                ms = batch.last_run_ms()
                results.append({"mode": mode, "threads": th, "blocks": blocks, "ms_per_step": ms / steps})
                if verbose:
                    print(f"  mode={mode} threads={th} blocks={blocks}: {ms / steps:.3f} ms/half-step", flush=True)
    def time_one(c):
        batch.set_schedule(c["threads"], c["blocks"], c["mode"])
        batch.run(steps, cfl_by_P)
        torch.cuda.synchronize()
        batch.run(steps, cfl_by_P)
        return batch.last_run_ms() / steps

    best = dict(refine(results, time_one))
    best["ms_per_step"] = best.pop("refined_ms")
    best.pop("refined_all", None)
    batch.set_schedule(best["threads"], best["blocks"], best["mode"])
    c = _load_cache()
    c[key_batch(batch)] = {
        k: best[k] for k in ("mode", "threads", "blocks", "ms_per_step")}
    _save_cache(c)
    best["tried"] = results
    return best


def key_2d(solver: "binding.Solver2D") -> str:
    bx, by = solver.bcs
    return (f"2d/{solver.equation}/P{solver.P}/{'lim' if solver.params.limiter else 'nolim'}/"
            f"{solver.Nx}x{solver.Ny}/{bx},{by}")


def cached_2d(solver: "binding.Solver2D"):
    """The cached launch shape for `solver`'s configuration, or None."""
    return _load_cache().get(key_2d(solver))


def tune_2d(solver: "binding.Solver2D", q0: np.ndarray, cfl: float, steps: int = 96, threads=(128, 256),
            block_factors=(0, 0.5, 1, 2, 3, 4), variants=(1, 2, 3), verbose: bool = False) -> dict:
    """Time 2D launch shapes on `solver` (state q0): row-marching variant
    (1 without, 2 with the next row prefetched, 3 as 2 with band-major work
    items) x threads per block x blocks
    per launch (block factor x compute units; 0 = the library's default,
    which fills the device at the kernel's occupancy).  Longer runs per wave
    re-expand fewer priming rows, more waves hide more latency; the best
    balance depends on the degree and the mesh, hence the measurement."""
    import torch
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    results = []
    for var in variants:
        for th in threads:
            for bf in block_factors:
                blocks = 0 if bf == 0 else max(1, int(round(bf * cu)))
                solver.set_launch(th, blocks, var)
                solver.write(q0)
                solver.run(48, cfl)            # warm-up, builds the graphs of this shape
                torch.cuda.synchronize()
                solver.run(steps, cfl)
                ms = solver.last_run_ms() / steps
                results.append({"variant": var, "threads": th, "blocks": blocks, "ms_per_step": ms})
                if verbose:
                    print(f"  variant={var} threads={th:4d} blocks={blocks:6d}: {ms * 1e3:8.2f} us/half-step", flush=True)
    def time_one(c):
        solver.set_launch(c["threads"], c["blocks"], c["variant"])
        solver.write(q0)
        solver.run(48, cfl)
        torch.cuda.synchronize()
        solver.run(steps, cfl)
        return solver.last_run_ms() / steps

    per_variant = {v: min(r["ms_per_step"] for r in results if r["variant"] == v) for v in variants}
    best = dict(refine(results, time_one))
    best["ms_per_step"] = best.pop("refined_ms")
    best.pop("refined_all", None)
    c = _load_cache()
    c[key_2d(solver)] = {k: best[k] for k in ("variant", "threads", "blocks", "ms_per_step")}
    _save_cache(c)
    solver.set_launch(best["threads"], best["blocks"], best["variant"])
    best["per_variant_ms"] = per_variant
    best["tried"] = results
    return best
