"""wcc_run_noalloc -- the entry point for callers that cannot allocate -- against
wcc_run through the C ABI: the same half-steps on the same state, bit for bit
in binary64 (and identical in the FP32-mixed mode, which runs the same kernels),
on two calls in a row, the second on a smaller mesh (the static scratch keeps
the first call's contents, so the second checks that every call starts clean)."""
import ctypes

import numpy as np
import pytest

from paper_2104_04347_amd import binding, inputs

pytestmark = pytest.mark.gpu


def _decode(s: binding.Solver, parity: int) -> np.ndarray:
    """State of mesh `parity` read from the state region of s's workspace
    (the layout wcc_run_noalloc documents)."""
    import torch
    nc, P = s.nc, s.P
    elem = 8 if s.params.precision == 0 else 4
    ld = (max(s.ncells(0), s.ncells(1)) + 63) // 64 * 64
    al = lambda x: (x + 255) // 256 * 256
    pb, db = al(nc * ld * 8), al(nc * P * ld * elem)
    torch.cuda.synchronize()
    raw = s.workspace[binding.WCC_WORKSPACE_STATE_OFFSET:].cpu().numpy()
    n = s.ncells(parity)
    p = raw[parity * pb: parity * pb + nc * ld * 8].view(np.float64).reshape(nc, ld)[:, :n]
    d0 = 2 * pb + parity * db
    dt = np.float64 if elem == 8 else np.float32
    d = raw[d0: d0 + nc * P * ld * elem].view(dt).reshape(nc, P, ld)[:, :, :n]
    out = np.empty((nc, P + 1, n))
    out[:, 0] = p
    out[:, 1:] = d
    return out


def _one_call(P, N, steps, precision, seed):
    q0, _ = inputs.euler_riemann(seed, P, N)
    kw = dict(limiter=True, precision=precision)
    ref = binding.Solver("euler", P, N, "transmissive", **kw)
    ref.write(q0)
    ref.run(steps, 0.25)
    q_ref, info = ref.read()
    ref.close()
    s = binding.Solver("euler", P, N, "transmissive", **kw)
    s.write(q0)                      # puts the initial state into the workspace's state region
    lib = binding.load()
    t = ctypes.c_double()
    base = s.workspace.data_ptr() + binding.WCC_WORKSPACE_STATE_OFFSET
    nbytes = s.workspace.numel() - binding.WCC_WORKSPACE_STATE_OFFSET
    print(f"wcc_run_noalloc: Euler P={P} N={N} {precision} {steps} half-steps", flush=True)
    rc = lib.wcc_run_noalloc(s.h, ctypes.c_void_p(base), nbytes, 0, 0.0, steps, 0.25, ctypes.c_void_p(s.stream),
                             ctypes.byref(t))
    assert rc == 0, binding.load().wcc_last_error(s.h)
    q = _decode(s, steps & 1)
    s.close()
    assert t.value == info.t, (t.value, info.t)
    assert info.parity == steps & 1
    assert np.array_equal(q, q_ref), f"{np.count_nonzero(q != q_ref)} values differ"


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_noalloc_equals_run_two_calls(precision):
    _one_call(3, 3000, 50, precision, seed=1)
    _one_call(3, 700, 37, precision, seed=2)    # smaller mesh, odd step count


def test_noalloc_rejects_bad_arguments():
    lib = binding.load()
    s = binding.Solver("euler", 2, 300, "transmissive")
    base = s.workspace.data_ptr() + binding.WCC_WORKSPACE_STATE_OFFSET
    nbytes = s.workspace.numel() - binding.WCC_WORKSPACE_STATE_OFFSET
    t = ctypes.c_double()
    assert lib.wcc_run_noalloc(s.h, None, nbytes, 0, 0.0, 1, 0.25, None, ctypes.byref(t)) == binding.WCC_EINVAL
    assert lib.wcc_run_noalloc(s.h, ctypes.c_void_p(base + 8), nbytes, 0, 0.0, 1, 0.25, None,
                               ctypes.byref(t)) == binding.WCC_EINVAL
    assert lib.wcc_run_noalloc(s.h, ctypes.c_void_p(base), nbytes - 1024, 0, 0.0, 1, 0.25, None,
                               ctypes.byref(t)) == binding.WCC_ESIZE
    assert lib.wcc_run_noalloc(s.h, ctypes.c_void_p(base), nbytes, 0, 0.0, 1, 1.5, None,
                               ctypes.byref(t)) == binding.WCC_EINVAL
    s.close()
