"""Build the gfx950 HIP library libwcc.so in-tree (paper_2104_04347_amd/_lib/).

Every translation unit is compiled by hipcc for gfx950 only, with
-ffp-contract=off (the binary64 path follows a fixed operation order) and
without packed-FP32 instructions; the objects are compiled in parallel and
linked into one shared library that exports the C ABI of include/wcc.h.

The same build links the diagnostic library libwcc_timeline.so: the product
objects with the three kernel translation units replaced by their timestamped
builds (csrc/wcc_timeline_*.hip, which include the kernel sources unchanged).
Only paper_2104_04347_amd/timeline.py loads it.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libwcc.so")
TIMELINE_LIB = os.path.join(OUT_DIR, "libwcc_timeline.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["wcc_kernels.hip", "wcc_kernels_wide.hip", "wcc_ctrl.hip", "wcc_batch.hip", "wcc_api.hip", "wcc2d_kernels.hip", "wcc2d_api.hip"]
# diagnostic build: kernel translation unit -> its timestamped replacement
TIMELINE_SOURCES = {"wcc_kernels.hip": "wcc_timeline_1d.hip", "wcc_kernels_wide.hip": "wcc_timeline_1d_wide.hip",
                    "wcc2d_kernels.hip": "wcc_timeline_2d.hip"}
ARCH = "gfx950"

HIPFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def torch_lib_dir() -> str:
    """Directory of the HIP runtime bundled with PyTorch.  The library links
    that runtime (not /opt/rocm's) so one process holds ONE HIP runtime: the
    torch-allocated memory, torch streams and torch events are then the same
    objects the kernels run on."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        raise RuntimeError("PyTorch (ROCm) is required to build: it provides the HIP runtime")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so under {d}")
    return d


def _compile(src: str, obj: str, verbose: bool) -> None:
    cmd = [hipcc(), *HIPFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{out}")
    if verbose and out.strip():
        print(out)


def _link(out: str, objs: list, verbose: bool) -> None:
    tmp = out + ".tmp"
    tl = torch_lib_dir()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-no-hip-rt", "-o", tmp, *objs,
           f"-L{tl}", "-l:libamdhip64.so", f"-Wl,-rpath,{tl}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = SOURCES + list(TIMELINE_SOURCES.values())
    obj = {s: os.path.join(OUT_DIR, s.replace(".hip", ".o")) for s in srcs}
    # the two longest compiles (the 2D kernels and their timestamped build) first
    order = sorted(srcs, key=lambda s: s not in ("wcc2d_kernels.hip", "wcc_timeline_2d.hip"))
    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 1)) as ex:
        list(ex.map(lambda s: _compile(s, obj[s], verbose), order))
    _link(LIB, [obj[s] for s in SOURCES], verbose)
    _link(TIMELINE_LIB, [obj[TIMELINE_SOURCES.get(s, s)] for s in SOURCES], verbose)
    for o in obj.values():
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
