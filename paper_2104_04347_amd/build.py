"""Build the gfx950 HIP library libwcc.so in-tree (paper_2104_04347_amd/_lib/).

Every translation unit is compiled by hipcc for gfx950 only, with
-ffp-contract=off (the binary64 path follows a fixed operation order) and
without packed-FP32 instructions; the objects are compiled in parallel and
linked into one shared library that exports the C ABI of include/wcc.h.
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
ROOT = os.path.dirname(HERE)

SOURCES = ["wcc_kernels.hip", "wcc_kernels_wide.hip", "wcc_ctrl.hip", "wcc_batch.hip", "wcc_api.hip", "wcc2d_kernels.hip", "wcc2d_api.hip"]
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


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objs = [os.path.join(OUT_DIR, s.replace(".hip", ".o")) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    tl = torch_lib_dir()
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-no-hip-rt", "-o", tmp, *objs,
           f"-L{tl}", "-l:libamdhip64.so", f"-Wl,-rpath,{tl}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
