"""Host logic around the kernels (no GPU): the benchmark's bookkeeping, the
rocprofv3 summaries and counter record, the autotuner's cache keys."""
import json
import os
import sqlite3

import numpy as np
import pytest

import bench
from paper_2104_04347_amd import autotune, profsum, records, timeline


def test_cells_updated():
    assert bench.cells_updated(100, "periodic", 0, 7) == 700
    # transmissive: N new cells from the original mesh, N + 1 back
    assert bench.cells_updated(100, "transmissive", 0, 4) == 100 + 101 + 100 + 101
    assert bench.cells_updated(100, "transmissive", 1, 3) == 101 + 100 + 101


def test_bytes_per_launch():
    # Euler P = 3: binary64 96 B per cell, FP32-mixed 3 x (8 + 12) = 60 B
    assert bench.bytes_per_launch(1 << 20, 3, 3, "fp64") == (2 * (1 << 20) + 1) * 96
    assert bench.bytes_per_launch(1 << 20, 3, 3, "fp32_mixed") == (2 * (1 << 20) + 1) * 60


def test_code_only_ignores_comments():
    a = "int f(int x) {  // doubles x\n  /* a\n block */ return 2 * x;\n}\n"
    b = "int f(int x) {\n\n  return 2 * x;   \n}"
    assert profsum.code_only(a) == profsum.code_only(b)
    assert profsum.code_only(a) != profsum.code_only(a.replace("2 * x", "3 * x"))


def test_source_hash_follows_code_not_comments():
    real = profsum.kernel_source_hash("2d")
    texts = {n: open(os.path.join(profsum.CSRC, n)).read() for n in profsum.KERNEL_SOURCES_2D}
    commented = dict(texts)
    commented["wcc2d_kernels.hip"] = "// a new comment\n" + texts["wcc2d_kernels.hip"]
    assert profsum.kernel_source_hash("2d", commented.__getitem__) == real
    changed = dict(texts)
    changed["wcc2d_kernels.hip"] = texts["wcc2d_kernels.hip"].replace("0.25 *", "0.5 *", 1)
    assert profsum.kernel_source_hash("2d", changed.__getitem__) != real
    assert profsum.kernel_source_hash("1d") != real


def _fake_db(path, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, counter_name text, "
                "value real)")
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()


def test_traffic_scaling_and_dispatch_selection(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by what the
    counter reads for a copy of known size in the same run; a kernel shared
    by two legs is split by dispatch order."""
    k, copy = "void k2d<2, 3>(args)", profsum.COPY_KERNEL
    fetch = [(1, copy, "FETCH_SIZE", 262144.0)]                      # a 512 MiB copy reads as half
    fetch += [(10 + i, k, "FETCH_SIZE", 1000.0) for i in range(3)]
    fetch += [(20 + i, k, "FETCH_SIZE", 3000.0) for i in range(3)]
    write = [(1, copy, "WRITE_SIZE", 524288.0)]
    write += [(10 + i, k, "WRITE_SIZE", 800.0) for i in range(3)] + [(20 + i, k, "WRITE_SIZE", 900.0) for i in range(3)]
    _fake_db(tmp_path / "f.db", fetch)
    _fake_db(tmp_path / "w.db", write)
    out = tmp_path / "traffic.json"
    rec = profsum.traffic(str(tmp_path / "f.db"), str(tmp_path / "w.db"), "k2d<2, 3>", "leg2", 64, 512, str(out),
                          "2d", slice(3, 6))
    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
    assert rec["fetch_bytes"] == 3000.0 * 1024 * 2 and rec["write_bytes"] == 900.0 * 1024
    assert rec["dispatches"] == [3, 3] and rec["source_sha256"] == profsum.kernel_source_hash("2d")
    assert json.load(open(out))["leg2"]["N"] == 64
    # the benchmark reads such a record only for the same code and size
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(out.read_text())
    assert bench.measured_traffic("leg2", 64, "2d") == rec["fetch_bytes"] + rec["write_bytes"]
    assert bench.measured_traffic("leg2", 65, "2d") is None
    assert bench.measured_traffic("leg2", 64, "1d") is None


def test_committed_records_match_the_sources():
    """The committed counter records belong to the kernels as they are."""
    rec = json.load(open(os.path.join(bench.ROOT, "profiles", "traffic.json")))
    assert rec, "no records"
    for key, e in rec.items():
        assert e["source_sha256"] == profsum.kernel_source_hash(e.get("sources", "1d")), key
        assert bench.measured_traffic(key, e["N"], e.get("sources", "1d")) > 0
    path = os.path.join(bench.ROOT, "profiles", "valu_insts.json")
    if os.path.exists(path):
        for key, e in json.load(open(path)).items():
            assert e["source_sha256"] == profsum.kernel_source_hash(e.get("sources", "1d")), key
            assert bench.valu_insts(key, e["N"], e.get("sources", "1d")) > 0


def test_valu_instruction_record_and_issue_roof(tmp_path, monkeypatch):
    """SQ_INSTS_VALU per dispatch -> record -> issue roof: instructions at one
    per 4 cycles on 1024 SIMDs at 2.4 GHz, against the launch time."""
    k = "void wcc::k_half_step<2, 3, true, double, 0>(args)"
    rows = [(i, k, "SQ_INSTS_VALU", 1.0e6 + (i % 2) * 2.0) for i in range(6)]
    rows += [(i, k, "SQ_WAVES", 3072.0) for i in range(6)]
    _fake_db(tmp_path / "i.db", rows)
    out = tmp_path / "valu_insts.json"
    rec = profsum.insts(str(tmp_path / "i.db"), "k_half_step<2, 3, true, double, 0>", "key1", 128, str(out))
    assert rec["sq_insts_valu"] == 1.0e6 + 1.0 and rec["sq_waves"] == 3072.0 and rec["dispatches"] == 6
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "valu_insts.json").write_text(out.read_text())
    assert bench.valu_insts("key1", 128) == rec["sq_insts_valu"]
    assert bench.valu_insts("key1", 129) is None
    launch_s = 10e-6
    r = bench.issue_roof("key1", 128, launch_s)
    floor = rec["sq_insts_valu"] * 4 / (1024 * 2.4e9)
    assert abs(r["frac"] - round(floor / launch_s, 4)) < 1e-12
    assert abs(r["issue_floor_us"] - round(floor * 1e6, 2)) < 1e-12
    assert bench.issue_roof("key1", 129, launch_s) is None
    assert "frac_at_clock" not in r
    # with a clock record for the same build and size: the roof at that clock
    timeline.record("key1", "1d", 128, {"clock_mhz": 1800.0, "clock_mhz_p0_10_50_90_100": [1700.0] * 5,
                                        "launch_us": 10.0, "mean_waves_per_simd": 3.0},
                    path=str(tmp_path / "profiles" / "clock.json"))
    r = bench.issue_roof("key1", 128, launch_s)
    assert r["shader_clock_mhz"] == 1800.0
    assert abs(r["frac_at_clock"] - round(floor * 2400.0 / 1800.0 / launch_s, 4)) < 1e-12
    assert bench.shader_clock("key1", 128, "2d") is None and bench.shader_clock("key1", 64) is None


def test_committed_clock_records_match_the_sources():
    path = os.path.join(bench.ROOT, "profiles", "clock.json")
    if not os.path.exists(path):
        pytest.skip("no clock records committed")
    for key, e in json.load(open(path)).items():
        src = "2d" if key.startswith("k2d") else ("1d_wide" if key.startswith("k_half_step_wide") else "1d")
        assert e["source_sha256"] == profsum.kernel_source_hash(src), key
        assert 300.0 < bench.shader_clock(key, e["N"], src) < 3000.0


def test_record_keys_are_those_of_the_committed_counter_records():
    keys = set(json.load(open(os.path.join(bench.ROOT, "profiles", "valu_insts.json"))))
    assert records.key_1d("fp64", 3, 0) == ("k_half_step<euler,P=3,limiter,f64,variant=0>", "1d")
    assert records.key_1d("fp32_mixed", 3, 4) == ("k_half_step_wide<euler,P=3,limiter,f32>", "1d_wide")
    assert records.key_2d("euler", 3, True, 3, False, 256, 256) in keys
    assert records.key_2d("euler", 3, False, 3, True, 256, 256) in keys
    assert records.key_2d("burgers", 3, True, 3, True, 256, 512) in keys


def test_autotune_keys():
    assert autotune.key_single("euler", 3, 1 << 20, "fp64", True) == "single/euler/P3/fp64/lim/N2^20"
    assert autotune.key_single("euler", 3, (1 << 20) + 5, "fp64", True) == "single/euler/P3/fp64/lim/N2^20"
    assert autotune.key_single("burgers", 2, 3000, "fp32_mixed", False) == "single/burgers/P2/fp32_mixed/nolim/N2^11"


def test_autotune_cache_roundtrip(tmp_path, monkeypatch):
    monkeypatch.setenv("WCC_AUTOTUNE_CACHE", str(tmp_path / "sub" / "cache.json"))
    assert autotune._load_cache() == {}
    autotune._save_cache({"k": {"threads": 128}})
    assert autotune._load_cache() == {"k": {"threads": 128}}
    # an unwritable location only costs a re-tune
    monkeypatch.setenv("WCC_AUTOTUNE_CACHE", "/proc/no/such/dir/cache.json")
    autotune._save_cache({"k": 1})
    assert autotune._load_cache() == {}


def test_gpu_count_guard():
    """bench.py measures one GPU and says so for any other count."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


class _FakeSolver:
    """Stands in for binding.Solver: scripted per-shape timings, no GPU."""
    equation, P, N = "euler", 3, 1 << 20

    class params:
        precision, limiter = 0, 1

    def __init__(self, times, default):
        self.times, self.shape, self.calls = times, dict(default), []

    def get_launch(self):
        return dict(self.shape)

    def set_launch(self, threads=0, blocks=0, variant=-1):
        self.shape = {"threads": threads or 256, "blocks": blocks,
                      "variant": self.shape["variant"] if variant < 0 else variant}
        self.calls.append(dict(self.shape))

    def write(self, q0):
        pass

    def run(self, steps, cfl):
        self.steps = steps

    def last_run_ms(self):
        s = self.shape
        return self.times.get((s["variant"], s["threads"], s["blocks"]), 1.0) * self.steps


def test_autotune_single_picks_fastest_and_reports_variants(tmp_path, monkeypatch):
    import types
    monkeypatch.setenv("WCC_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(
        get_device_properties=lambda i: types.SimpleNamespace(multi_processor_count=256),
        synchronize=lambda: None))
    monkeypatch.setitem(__import__("sys").modules, "torch", fake_torch)
    times = {(2, 256, 768): 0.5, (1, 128, 0): 0.7, (1, 256, 0): 0.8}
    s = _FakeSolver(times, {"threads": 256, "blocks": 0, "variant": 1})
    best = autotune.tune_single(s, None, 0.25, steps=10, threads=(128, 256), block_factors=(0, 3), variants=(0, 1, 2))
    assert (best["variant"], best["threads"], best["blocks"]) == (2, 256, 768)
    assert best["per_variant_ms"] == {0: 1.0, 1: 0.7, 2: 0.5}
    assert s.get_launch() == {"threads": 256, "blocks": 768, "variant": 2}
    # the library's own default is timed too and kept when nothing beats it
    s2 = _FakeSolver({(1, 256, 0): 0.1}, {"threads": 256, "blocks": 0, "variant": 1})
    b2 = autotune.tune_single(s2, None, 0.25, steps=10, threads=(128,), block_factors=(3,), variants=(0, 2))
    assert (b2["variant"], b2["threads"], b2["blocks"]) == (1, 256, 0) and b2["ms_per_step"] == 0.1
    cache = json.load(open(tmp_path / "c.json"))
    assert cache["single/euler/P3/fp64/lim/N2^20"]["variant"] == 1


def test_autotune_single_chooses_between_tile_shapes(tmp_path, monkeypatch):
    """The default candidates span both wave-tile shapes (64 cells, one per
    lane: variants 0-3; 128 cells, two per lane: variant 4); the faster one
    per workload wins and the cache records which shape it is."""
    import types
    monkeypatch.setenv("WCC_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(
        get_device_properties=lambda i: types.SimpleNamespace(multi_processor_count=256),
        synchronize=lambda: None))
    monkeypatch.setitem(__import__("sys").modules, "torch", fake_torch)
    s = _FakeSolver({(4, 256, 1024): 0.4, (0, 256, 768): 0.45}, {"threads": 256, "blocks": 0, "variant": 1})
    best = autotune.tune_single(s, None, 0.25, steps=10)
    assert (best["variant"], best["tile"], best["blocks"]) == (4, "128x2", 1024)
    assert set(best["per_variant_ms"]) == {0, 1, 2, 3, 4}
    assert json.load(open(tmp_path / "c.json"))["single/euler/P3/fp64/lim/N2^20"]["tile"] == "128x2"
    s = _FakeSolver({(4, 256, 1024): 0.5, (0, 256, 768): 0.45}, {"threads": 256, "blocks": 0, "variant": 1})
    best = autotune.tune_single(s, None, 0.25, steps=10)
    assert (best["variant"], best["tile"]) == (0, "64x1")


def test_autotune_batch_tries_every_schedule(tmp_path, monkeypatch):
    import types
    monkeypatch.setenv("WCC_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(
        get_device_properties=lambda i: types.SimpleNamespace(multi_processor_count=256),
        synchronize=lambda: None))
    monkeypatch.setitem(__import__("sys").modules, "torch", fake_torch)

    class FakeBatch:
        B = 4096

        class params:
            precision = 1

        def __init__(self):
            self.sched, self.seen = None, set()

        def set_schedule(self, threads, blocks, mode):
            self.sched = (threads, blocks, mode)
            self.seen.add(mode)

        def run(self, steps, cfl):
            self.steps = steps

        def last_run_ms(self):
            th, bl, mode = self.sched
            return (1.0 - 0.05 * mode - (0.01 if bl == 1024 else 0.0)) * self.steps

    bt = FakeBatch()
    best = autotune.tune_batch(bt, [0.4] * 5, steps=8)
    assert bt.seen == {1, 2, 3, 4, 5, 6}
    assert (best["mode"], best["blocks"]) == (6, 1024) and bt.sched == (best["threads"], 1024, 6)
    assert autotune.cached_batch(bt)["mode"] == 6


def test_autotune_2d_keys_and_choice(tmp_path, monkeypatch):
    import types
    monkeypatch.setenv("WCC_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    fake_torch = types.SimpleNamespace(cuda=types.SimpleNamespace(
        get_device_properties=lambda i: types.SimpleNamespace(multi_processor_count=256),
        synchronize=lambda: None))
    monkeypatch.setitem(__import__("sys").modules, "torch", fake_torch)

    class Fake2D:
        equation, P, Nx, Ny, bcs = "burgers", 3, 2048, 2048, ("periodic", "periodic")

        class params:
            limiter = 1

        def set_launch(self, threads, blocks, variant):
            self.shape = (variant, threads, blocks)

        def write(self, q0):
            pass

        def run(self, steps, cfl):
            self.steps = steps

        def last_run_ms(self):
            return (0.18 if self.shape == (2, 256, 256) else 0.2) * self.steps

    s = Fake2D()
    best = autotune.tune_2d(s, None, 0.25, steps=8)
    assert (best["variant"], best["threads"], best["blocks"]) == (2, 256, 256) and s.shape == (2, 256, 256)
    assert autotune.key_2d(s) == "2d/burgers/P3/lim/2048x2048/periodic,periodic"
    assert autotune.cached_2d(s)["blocks"] == 256


def test_autotune_refine_picks_the_steady_state_best():
    """A candidate that looked fastest in its single sweep timing (a clock
    transition) loses the round-robin re-timing to the one that is faster in
    steady state; finalists are re-timed in rotated order."""
    cands = [{"name": "A", "ms_per_step": 0.80}, {"name": "B", "ms_per_step": 0.90},
             {"name": "C", "ms_per_step": 0.95}, {"name": "D", "ms_per_step": 0.99},
             {"name": "E", "ms_per_step": 2.0}]
    steady = {"A": 1.0, "B": 0.9, "C": 0.97, "D": 1.1, "E": 0.5}
    order = []

    def time_one(c):
        order.append(c["name"])
        # the first timing of each round is disturbed (+20%)
        return steady[c["name"]] * (1.2 if len(order) % 4 == 1 else 1.0)

    best = autotune.refine(cands, time_one, top=4, rounds=3)
    assert best["name"] == "B" and best["refined_ms"] == 0.9
    assert "E" not in order                      # only the four fastest of the sweep are finalists
    assert order[:4] == ["A", "B", "C", "D"] and order[4:8] == ["B", "C", "D", "A"]
    assert all(len(c["refined_all"]) == 3 for c in cands[:4])
