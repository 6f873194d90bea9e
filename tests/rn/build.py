"""Build tests/rn/rn_check, a test helper that runs the device rounding helpers
(paper_2104_04347_amd/csrc/wcc_rn.hpp) on operands from files.  Compiled with
the library's device flags; run by __graft_entry__.build()."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "rn_check.hip")
EXE = os.path.join(HERE, "rn_check")
CSRC = os.path.join(ROOT, "paper_2104_04347_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    tmp = EXE + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{CSRC}", SRC, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
    sys.exit(0)
