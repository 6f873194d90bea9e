"""The boundary from C: tests/c_abi/consumer.c uses the library through
include/wcc.h alone (workspace from hipMalloc, its own HIP stream, no Python
or PyTorch in its process) and advances Sod's shock tube (Section 5.2) to
t = 0.4; tests/c_abi/consumer2d.c does the same through include/wcc2d.h for
the first 2D Riemann problem of Section 5.3.  Their results must be the
oracle's, bit for bit."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2104_04347_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c_abi", "consumer")
EXE2D = os.path.join(HERE, "c_abi", "consumer2d")


@pytest.mark.parametrize("exe", [EXE, EXE2D])
def test_consumer_is_built_against_the_library(exe):
    assert os.path.exists(exe), "built by __graft_entry__.build() (tests/c_abi/build.py)"
    out = subprocess.run(["ldd", exe], capture_output=True, text=True, check=True).stdout
    assert "libwcc.so" in out and "not found" not in out


@pytest.mark.parametrize("exe", [EXE, EXE2D])
def test_consumer_usage_error_without_gpu(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr


@pytest.mark.gpu
def test_consumer_matches_the_oracle(tmp_path):
    P, N, t_end, cfl = 3, 400, 0.4, 0.25
    q0, _ = inputs.sod(P, N)
    q0.astype("<f8").tofile(tmp_path / "in.bin")
    cmd = [EXE, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), str(P), str(N), "0", "2", repr(t_end), repr(cfl)]
    print("C consumer:", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    raw = np.fromfile(tmp_path / "out.bin", dtype="<f8")
    t, parity, taken = raw[-3], int(raw[-2]), int(raw[-1])
    pb = oracle.Problem("euler", P, N, bc="transmissive", limiter=True, x_left=0.0, x_right=2.0)
    ref = oracle.run(pb, q0, t_end=t_end, cfl=cfl)
    assert (taken, parity, t) == (ref.half_steps, ref.parity, ref.t)
    q = raw[:-3].reshape(3, P + 1, -1)
    assert q.shape == ref.q.shape
    diff = np.argwhere(q.view(np.uint64) != ref.q.view(np.uint64))
    assert len(diff) == 0, (len(diff), [(tuple(i), q[tuple(i)], ref.q[tuple(i)]) for i in diff[:8]],
                            float(np.abs(q - ref.q).max()))


@pytest.mark.gpu
def test_consumer2d_matches_the_oracle(tmp_path):
    P, N, t_end, cfl = 3, 48, 0.25, 0.25
    q0 = inputs.riemann2d(1, P, N)
    q0.astype("<f8").tofile(tmp_path / "in.bin")
    cmd = [EXE2D, str(tmp_path / "in.bin"), str(tmp_path / "out.bin"), str(P), str(N), "-1", "1", repr(t_end),
           repr(cfl)]
    print("C consumer (2D):", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    raw = np.fromfile(tmp_path / "out.bin", dtype="<f8")
    t, parity, taken = raw[-3], int(raw[-2]), int(raw[-1])
    pb = oracle.Problem2D("euler", P, N, N, limiter=True, bc="transmissive", x_left=-1.0, x_right=1.0,
                          y_left=-1.0, y_right=1.0)
    ref = oracle.run2d(pb, q0, t_end=t_end, cfl=cfl)
    assert ref.flags == 0 and taken > 20
    assert (taken, parity, t) == (ref.half_steps, ref.parity, ref.t)
    q = raw[:-3].reshape(ref.q.shape)
    diff = np.argwhere(q.view(np.uint64) != ref.q.view(np.uint64))
    assert len(diff) == 0, (len(diff), [(tuple(i), q[tuple(i)], ref.q[tuple(i)]) for i in diff[:8]],
                            float(np.abs(q - ref.q).max()))
