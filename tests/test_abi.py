"""CPU checks of the boundary: the HIP library loads, exports every symbol that
include/wcc.h and include/wcc2d.h declare, and validates arguments in the
calls that need no GPU."""
import ctypes
import os
import re

import pytest

from paper_2104_04347_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("wcc.h", "wcc2d.h")]


def declared():
    txt = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"^(?:int|void|const char\*)\s+(wcc(?:2d)?_\w+)\s*\(", txt, re.M)))


def test_header_declares_the_abi():
    names = declared()
    assert "wcc_create" in names and "wcc_batch_advance" in names and "wcc2d_advance" in names and len(names) >= 33


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    for name in declared():
        assert hasattr(lib, name), name
    assert set(declared()) == set(binding.SIGNATURES), set(declared()) ^ set(binding.SIGNATURES)


def test_error_strings():
    lib = binding.load()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.wcc_strerror(code)
    assert b"unknown" in lib.wcc_strerror(-99)


def test_create_rejects_bad_arguments():
    lib = binding.load()
    h = ctypes.c_void_p()
    p = binding.make_params()
    for eq, P, N, bc in [(3, 2, 100, 0), (0, 5, 100, 0), (0, -1, 100, 0), (0, 2, 1, 0), (0, 2, 100, 3)]:
        assert lib.wcc_create(eq, P, N, bc, ctypes.byref(p), ctypes.byref(h)) == binding.WCC_EINVAL
    bad = binding.make_params(x_left=1.0, x_right=0.0)
    assert lib.wcc_create(0, 2, 100, 0, ctypes.byref(bad), ctypes.byref(h)) == binding.WCC_EINVAL
    bad = binding.make_params(gamma=1.0)
    assert lib.wcc_create(2, 2, 100, 0, ctypes.byref(bad), ctypes.byref(h)) == binding.WCC_EINVAL


def test_workspace_size_and_state_errors_without_gpu():
    lib = binding.load()
    h = ctypes.c_void_p()
    p = binding.make_params(precision="fp64")
    assert lib.wcc_create(2, 3, 1 << 20, 1, ctypes.byref(p), ctypes.byref(h)) == 0
    nb = ctypes.c_size_t()
    assert lib.wcc_workspace_bytes(h, ctypes.byref(nb)) == 0
    ld = ((1 << 20) + 1 + 63) // 64 * 64
    assert nb.value >= 2 * 3 * 4 * ld * 8          # two buffers of 3 components x (P+1) doubles
    # calls before bind are refused without touching the device
    assert lib.wcc_step(h, ctypes.c_double(0.25), ctypes.c_double(0.0)) == binding.WCC_ESTATE
    assert lib.wcc_run(h, 10, ctypes.c_double(0.25)) == binding.WCC_ESTATE
    assert lib.wcc_bind(h, None, 0, None) == binding.WCC_EINVAL
    assert lib.wcc_bind(h, ctypes.c_void_p(256), 16, None) == binding.WCC_ESIZE
    assert lib.wcc_bind(h, ctypes.c_void_p(255), nb.value, None) == binding.WCC_EINVAL
    # default variant by state size: prefetch (1) below 512 MiB of state
    t, b, v = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert lib.wcc_get_launch(h, ctypes.byref(t), ctypes.byref(b), ctypes.byref(v)) == 0
    assert (t.value, b.value, v.value) == (256, 0, 1)
    assert lib.wcc_get_launch(h, None, ctypes.byref(b), ctypes.byref(v)) == binding.WCC_EINVAL
    # kernel variant bits: 1 = prefetch, 2 = staged stores; -1 keeps the current one
    for v_ in (-1, 0, 1, 2, 3):
        assert lib.wcc_set_launch(h, 128, 0, v_) == 0
    assert lib.wcc_get_launch(h, ctypes.byref(t), ctypes.byref(b), ctypes.byref(v)) == 0
    assert (t.value, b.value, v.value) == (128, 0, 3)
    # 2^24 cells of Euler P = 4 in binary64: 4 GB of state -> staged stores + prefetch
    big = ctypes.c_void_p()
    assert lib.wcc_create(2, 4, 1 << 24, 0, ctypes.byref(p), ctypes.byref(big)) == 0
    assert lib.wcc_get_launch(big, ctypes.byref(t), ctypes.byref(b), ctypes.byref(v)) == 0 and v.value == 3
    lib.wcc_destroy(big)
    assert lib.wcc_set_launch(h, 128, 0, 5) == binding.WCC_EINVAL
    assert lib.wcc_set_launch(h, 128, 0, -2) == binding.WCC_EINVAL
    lib.wcc_destroy(h)
    pm = binding.make_params(precision="fp32_mixed")
    assert lib.wcc_create(2, 3, 1 << 20, 1, ctypes.byref(pm), ctypes.byref(h)) == 0
    nm = ctypes.c_size_t()
    lib.wcc_workspace_bytes(h, ctypes.byref(nm))
    assert nm.value < nb.value                      # binary32 derivatives
    lib.wcc_destroy(h)


def test_batch_create_validates():
    lib = binding.load()
    h = ctypes.c_void_p()
    p = binding.make_params(precision="fp32_mixed")
    P = (ctypes.c_int32 * 3)(1, 2, 3)
    N = (ctypes.c_int64 * 3)(300, 1000, 70)
    assert lib.wcc_batch_create(2, 3, P, N, 1, ctypes.byref(p), ctypes.byref(h)) == 0
    nb = ctypes.c_size_t()
    assert lib.wcc_batch_workspace_bytes(h, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.wcc_batch_set_schedule(h, 100, 0, 0) == binding.WCC_EINVAL
    assert lib.wcc_batch_set_schedule(h, 128, 64, 1) == 0
    for mode in (2, 3, 4, 5, 6, 0):                 # grouped, fused / grouped staged, branches, keep
        assert lib.wcc_batch_set_schedule(h, 0, 0, mode) == 0
    assert lib.wcc_batch_set_schedule(h, 0, 0, 7) == binding.WCC_EINVAL
    assert lib.wcc_batch_set_schedule(h, 0, 0, -1) == binding.WCC_EINVAL
    lib.wcc_batch_destroy(h)
    Pbad = (ctypes.c_int32 * 3)(1, 4, 3)
    assert lib.wcc_batch_create(2, 3, Pbad, N, 1, ctypes.byref(p), ctypes.byref(h)) == binding.WCC_EINVAL


def test_product_path_has_no_cpu_fallback(monkeypatch):
    """Without the built library the binding fails loudly."""
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(RuntimeError):
        binding.load("/nonexistent/libwcc.so")


def test_2d_create_validates():
    lib = binding.load()
    h = ctypes.c_void_p()
    p = binding.wcc2d_params()
    assert lib.wcc2d_params_default(ctypes.byref(p)) == 0
    assert p.limiter == 1 and p.eps == 1e-40 and p.x_right == 1.0 and p.b == 1.0 and p.bc == 0 and p.bc_y == -1
    for eq, P, nx, ny in [(3, 2, 64, 64), (0, 4, 64, 64), (0, -1, 64, 64), (0, 2, 1, 64), (0, 2, 1 << 15, 1 << 14)]:
        assert lib.wcc2d_create(eq, P, nx, ny, ctypes.byref(p), ctypes.byref(h)) == binding.WCC_EINVAL
    p.bc = 2                                   # Dirichlet is a 1D boundary only
    assert lib.wcc2d_create(1, 2, 64, 64, ctypes.byref(p), ctypes.byref(h)) == binding.WCC_EINVAL
    p.bc = 1
    assert lib.wcc2d_create(1, 2, 64, 64, ctypes.byref(p), ctypes.byref(h)) == 0
    nb_t = ctypes.c_size_t()
    assert lib.wcc2d_workspace_bytes(h, ctypes.byref(nb_t)) == 0
    assert nb_t.value >= 2 * 6 * (65 * 65) * 8             # planes sized for the (Nx+1) x (Ny+1) mesh
    lib.wcc2d_destroy(h)
    p.bc, p.bc_y = 0, 2                        # per-direction edges: periodic or transmissive only
    assert lib.wcc2d_create(1, 2, 64, 64, ctypes.byref(p), ctypes.byref(h)) == binding.WCC_EINVAL
    p.bc_y = 1
    assert lib.wcc2d_create(1, 2, 64, 64, ctypes.byref(p), ctypes.byref(h)) == 0
    lib.wcc2d_destroy(h)
    p.bc, p.bc_y = 0, -1
    # Euler needs gamma > 1; with it, both the limited and the unlimited form exist
    p.gamma = 1.0
    assert lib.wcc2d_create(2, 2, 64, 64, ctypes.byref(p), ctypes.byref(h)) == binding.WCC_EINVAL
    p.gamma = 1.4
    assert lib.wcc2d_create(2, 2, 64, 64, ctypes.byref(p), ctypes.byref(h)) == 0
    lib.wcc2d_destroy(h)
    p.limiter = 0
    assert lib.wcc2d_create(2, 3, 100, 50, ctypes.byref(p), ctypes.byref(h)) == 0
    nb = ctypes.c_size_t()
    assert lib.wcc2d_workspace_bytes(h, ctypes.byref(nb)) == 0
    plane = (100 * 50 + 63) // 64 * 64
    assert nb.value >= 2 * 4 * 10 * plane * 8            # two buffers of 4 components x 10 DOFs
    assert lib.wcc2d_step(h, ctypes.c_double(0.25), ctypes.c_double(0.0)) == binding.WCC_ESTATE
    assert lib.wcc2d_bind(h, ctypes.c_void_p(256), 16, None) == binding.WCC_ESIZE
    assert lib.wcc2d_set_launch(h, 100, 0, -1) == binding.WCC_EINVAL
    assert lib.wcc2d_set_launch(h, 0, 0, 4) == binding.WCC_EINVAL
    assert lib.wcc2d_set_launch(h, 128, 0, 0) == 0
    t, b, v = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    assert lib.wcc2d_get_launch(h, ctypes.byref(t), ctypes.byref(b), ctypes.byref(v)) == 0
    assert t.value == 128 and v.value == 0 and b.value >= 1          # blocks resolved, never 0
    assert lib.wcc2d_set_launch(h, 256, 300, 2) == 0
    assert lib.wcc2d_get_launch(h, ctypes.byref(t), ctypes.byref(b), ctypes.byref(v)) == 0
    assert (t.value, b.value, v.value) == (256, 300, 2)
    assert lib.wcc2d_get_launch(h, None, ctypes.byref(b), ctypes.byref(v)) == binding.WCC_EINVAL
    lib.wcc2d_destroy(h)
