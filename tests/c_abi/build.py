"""Build the C consumers of the library's ABI (tests/c_abi/consumer for
include/wcc.h, tests/c_abi/consumer2d for include/wcc2d.h), test helpers:
plain C, the HIP runtime's C API and the headers, linked against
paper_2104_04347_amd/_lib/libwcc.so.  Run by __graft_entry__.build() after
the library is built."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PROGRAMS = {os.path.join(HERE, "consumer.c"): os.path.join(HERE, "consumer"),
            os.path.join(HERE, "consumer2d.c"): os.path.join(HERE, "consumer2d")}
LIB_DIR = os.path.join(ROOT, "paper_2104_04347_amd", "_lib")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> list:
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        raise RuntimeError("no C compiler")
    for src, exe in PROGRAMS.items():
        tmp = exe + ".tmp"
        cmd = [cc, "-std=c11", "-O2", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
               f"-I{os.path.join(ROOT, 'include')}", src, "-o", tmp, f"-L{LIB_DIR}", "-l:libwcc.so",
               f"-L{ROCM}/lib", "-l:libamdhip64.so",
               # the library relative to the program, so that the tree can move
               "-Wl,-rpath,$ORIGIN/../../paper_2104_04347_amd/_lib", f"-Wl,-rpath,{ROCM}/lib"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, exe)
    return list(PROGRAMS.values())


if __name__ == "__main__":
    print(build())
    sys.exit(0)
