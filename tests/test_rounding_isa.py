"""No uncorrected binary64 division in the built library.

The compiler's binary64 division on gfx950 is faithful, not correctly
rounded, so every quotient the kernels compute must pass through div_rn
(csrc/wcc_rn.hpp), which follows the hardware sequence with the exact
remainder a - q b.  This test disassembles the gfx950 code objects of
libwcc.so (this repository's own build) and checks that every
v_div_fixup_f64 (the last instruction of the hardware sequence) is followed
by the remainder's fma with the same denominator and numerator.  A division
that escaped the helper -- a plain `/` in new code, or a constexpr helper
evaluated at run time -- fails it."""
import os
import re
import shutil
import subprocess

import pytest

from paper_2104_04347_amd import build

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
BUNDLER = os.path.join(ROCM, "llvm", "bin", "clang-offload-bundler")
OBJDUMP = os.path.join(ROCM, "llvm", "bin", "llvm-objdump")
MAGIC = b"__CLANG_OFFLOAD_BUNDLE__"
FIXUP = re.compile(r"^\s*v_div_fixup_f64\s+(v\[\d+:\d+\]),\s*(\S+),\s*(\S+),\s*([^\s/]+)")
WINDOW = 30     # instructions after the fixup in which the remainder must appear


def _disassemble(lib: str, tmp) -> list:
    """Disassembly (lines) of every gfx950 code object in lib's offload bundles."""
    fat = tmp / "fatbin"
    # objcopy rewrites its input file when given no output file, so it works
    # on a private copy: the library itself is mapped into this process
    copy = tmp / "lib.so"
    shutil.copyfile(lib, copy)
    subprocess.run(["objcopy", "--dump-section", f".hip_fatbin={fat}", str(copy), str(tmp / "discard.so")],
                   check=True, capture_output=True)
    data = fat.read_bytes()
    starts = [m.start() for m in re.finditer(re.escape(MAGIC), data)]
    assert starts, "no offload bundle in the library"
    out = []
    for n, (a, b) in enumerate(zip(starts, starts[1:] + [len(data)])):
        src, co = tmp / f"b{n}.bin", tmp / f"b{n}.co"
        src.write_bytes(data[a:b])
        subprocess.run([BUNDLER, "--unbundle", "--type=o", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        f"--input={src}", f"--output={co}"], check=True, capture_output=True)
        if co.stat().st_size == 0:
            continue
        r = subprocess.run([OBJDUMP, "-d", "--mcpu=gfx950", str(co)], check=True, capture_output=True, text=True)
        out.append(r.stdout.splitlines())
    return out


@pytest.mark.skipif(not (shutil.which("objcopy") and os.path.exists(BUNDLER) and os.path.exists(OBJDUMP)),
                    reason="needs objcopy and the ROCm LLVM tools")
def test_every_binary64_division_is_corrected(tmp_path):
    assert os.path.exists(build.LIB), "build the library first (__graft_entry__.build())"
    divisions = 0
    missing = []
    for lines in _disassemble(build.LIB, tmp_path):
        for i, line in enumerate(lines):
            m = FIXUP.match(line)
            if not m:
                continue
            divisions += 1
            q, den, num = m.group(1), m.group(3), m.group(4)
            rem = re.compile(r"^\s*v_fma_f64\s+v\[\d+:\d+\],\s*-" + re.escape(q) + r",\s*" + re.escape(den) +
                             r",\s*" + re.escape(num) + r"(\s|$)")
            if not any(rem.match(x) for x in lines[i + 1:i + 1 + WINDOW]):
                missing.append(line.strip())
    # 1D, wide-tile, batched and 2D kernels all divide in binary64
    assert divisions > 1000, divisions
    assert not missing, (len(missing), missing[:5])
