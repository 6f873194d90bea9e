"""Thin Python binding of the C ABI in include/wcc.h (argument marshalling only).

Every half-step runs in the gfx950 kernels of libwcc.so; PyTorch supplies the
device workspace and the HIP stream.  There is no CPU fallback: importing this
module without the built library, or using it without a GPU, raises.

The functions keep the C names (wcc_create, wcc_step, ...); `Solver` and
`Batch` wrap them with torch-owned device memory for convenience.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libwcc.so")

WCC_OK, WCC_EINVAL, WCC_ESTATE, WCC_ESIZE, WCC_EDEVICE, WCC_ENONFINITE = 0, -1, -2, -3, -4, -5
WCC_PMAX = 4
WCC_WORKSPACE_STATE_OFFSET = 12544   # include/wcc.h
EQUATIONS = {"advection": 0, "burgers": 1, "euler": 2}
BCS = {"periodic": 0, "transmissive": 1, "dirichlet": 2}
PRECISIONS = {"fp64": 0, "fp32_mixed": 1}
PRECISIONS_NAME = {v: k for k, v in PRECISIONS.items()}


class WccError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (code {code})")
        self.code = code


class wcc_params(ctypes.Structure):
    _fields_ = [
        ("x_left", ctypes.c_double), ("x_right", ctypes.c_double),
        ("a", ctypes.c_double), ("gamma", ctypes.c_double), ("eps", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("left_state", ctypes.c_double * 3), ("right_state", ctypes.c_double * 3),
    ]


class wcc_state_info(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("parity", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("n_cells", ctypes.c_int64), ("x_first_center", ctypes.c_double), ("dx", ctypes.c_double),
        ("half_steps", ctypes.c_int64), ("s_max", ctypes.c_double),
    ]


class wcc2d_params(ctypes.Structure):
    _fields_ = [
        ("x_left", ctypes.c_double), ("x_right", ctypes.c_double),
        ("y_left", ctypes.c_double), ("y_right", ctypes.c_double),
        ("a", ctypes.c_double), ("b", ctypes.c_double), ("gamma", ctypes.c_double), ("eps", ctypes.c_double),
        ("limiter", ctypes.c_int32), ("bc", ctypes.c_int32), ("bc_y", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class wcc2d_state_info(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double), ("parity", ctypes.c_int32), ("flags", ctypes.c_int32),
        ("Nx", ctypes.c_int64), ("Ny", ctypes.c_int64), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("half_steps", ctypes.c_int64), ("s_max", ctypes.c_double),
    ]


_c = ctypes
_vp, _i64, _dp = _c.c_void_p, _c.c_int64, _c.POINTER(_c.c_double)
SIGNATURES = {
    "wcc_params_default": ([_c.POINTER(wcc_params)], _c.c_int),
    "wcc_create": ([_c.c_int, _c.c_int, _i64, _c.c_int, _c.POINTER(wcc_params), _c.POINTER(_vp)], _c.c_int),
    "wcc_workspace_bytes": ([_vp, _c.POINTER(_c.c_size_t)], _c.c_int),
    "wcc_bind": ([_vp, _vp, _c.c_size_t, _vp], _c.c_int),
    "wcc_write_dofs": ([_vp, _dp, _i64, _c.c_int, _c.c_double], _c.c_int),
    "wcc_step": ([_vp, _c.c_double, _c.c_double], _c.c_int),
    "wcc_run": ([_vp, _i64, _c.c_double], _c.c_int),
    "wcc_advance": ([_vp, _c.c_double, _c.c_double, _i64, _c.POINTER(_i64)], _c.c_int),
    "wcc_read_dofs": ([_vp, _dp, _i64, _c.POINTER(wcc_state_info)], _c.c_int),
    "wcc_totals": ([_vp, _dp], _c.c_int),
    "wcc_set_launch": ([_vp, _c.c_int, _c.c_int, _c.c_int], _c.c_int),
    "wcc_get_launch": ([_vp, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)], _c.c_int),
    "wcc_last_run_ms": ([_vp, _dp], _c.c_int),
    "wcc_run_noalloc": ([_vp, _vp, _c.c_size_t, _c.c_int, _c.c_double, _i64, _c.c_double, _vp, _dp], _c.c_int),
    "wcc_strerror": ([_c.c_int], _c.c_char_p),
    "wcc_last_error": ([_vp], _c.c_char_p),
    "wcc_destroy": ([_vp], None),
    "wcc_batch_create": ([_c.c_int, _c.c_int, _c.POINTER(_c.c_int32), _c.POINTER(_i64), _c.c_int,
                          _c.POINTER(wcc_params), _c.POINTER(_vp)], _c.c_int),
    "wcc_batch_workspace_bytes": ([_vp, _c.POINTER(_c.c_size_t)], _c.c_int),
    "wcc_batch_bind": ([_vp, _vp, _c.c_size_t, _vp], _c.c_int),
    "wcc_batch_write_dofs": ([_vp, _c.c_int, _dp, _i64, _c.c_double], _c.c_int),
    "wcc_batch_prepare": ([_vp], _c.c_int),
    "wcc_batch_advance": ([_vp, _i64, _dp], _c.c_int),
    "wcc_batch_read_dofs": ([_vp, _c.c_int, _dp, _i64, _c.POINTER(wcc_state_info)], _c.c_int),
    "wcc_batch_set_schedule": ([_vp, _c.c_int, _c.c_int, _c.c_int], _c.c_int),
    "wcc_batch_last_run_ms": ([_vp, _dp], _c.c_int),
    "wcc_batch_last_error": ([_vp], _c.c_char_p),
    "wcc_batch_destroy": ([_vp], None),
    "wcc2d_params_default": ([_c.POINTER(wcc2d_params)], _c.c_int),
    "wcc2d_create": ([_c.c_int, _c.c_int, _i64, _i64, _c.POINTER(wcc2d_params), _c.POINTER(_vp)], _c.c_int),
    "wcc2d_workspace_bytes": ([_vp, _c.POINTER(_c.c_size_t)], _c.c_int),
    "wcc2d_bind": ([_vp, _vp, _c.c_size_t, _vp], _c.c_int),
    "wcc2d_write_dofs": ([_vp, _dp, _c.c_int, _c.c_double], _c.c_int),
    "wcc2d_step": ([_vp, _c.c_double, _c.c_double], _c.c_int),
    "wcc2d_run": ([_vp, _i64, _c.c_double], _c.c_int),
    "wcc2d_advance": ([_vp, _c.c_double, _c.c_double, _i64, _c.POINTER(_i64)], _c.c_int),
    "wcc2d_read_dofs": ([_vp, _dp, _i64, _c.POINTER(wcc2d_state_info)], _c.c_int),
    "wcc2d_set_launch": ([_vp, _c.c_int, _c.c_int, _c.c_int], _c.c_int),
    "wcc2d_get_launch": ([_vp, _c.POINTER(_c.c_int), _c.POINTER(_c.c_int), _c.POINTER(_c.c_int)], _c.c_int),
    "wcc2d_totals": ([_vp, _dp], _c.c_int),
    "wcc2d_last_run_ms": ([_vp, _dp], _c.c_int),
    "wcc2d_last_error": ([_vp], _c.c_char_p),
    "wcc2d_destroy": ([_vp], None),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libwcc.so (no GPU needed to load; every compute call needs one)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_2104_04347_amd/build.py "
                           "(the HIP library is the only implementation)")
    # PyTorch first: libwcc.so links the HIP runtime bundled with PyTorch, and
    # torch's memory, streams and events must be those of the same runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (argtypes, restype) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = restype
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _check(rc: int, what: str, ctx=None, batch=False, two_d=False):
    if rc != WCC_OK:
        lib = load()
        detail = ""
        if ctx is not None:
            err = lib.wcc2d_last_error if two_d else (lib.wcc_batch_last_error if batch else lib.wcc_last_error)
            detail = err(ctx) or b""
            detail = detail.decode(errors="replace")
        raise WccError(rc, f"{what}: {lib.wcc_strerror(rc).decode()}" + (f" -- {detail}" if detail else ""))


def make_params(limiter=True, precision="fp64", x_left=0.0, x_right=1.0, a=1.0, gamma=1.4, eps=1e-40,
                left_state=(0.0, 0.0, 0.0), right_state=(0.0, 0.0, 0.0)) -> wcc_params:
    p = wcc_params()
    load().wcc_params_default(ctypes.byref(p))
    p.x_left, p.x_right, p.a, p.gamma, p.eps = x_left, x_right, a, gamma, eps
    p.limiter = 1 if limiter else 0
    p.precision = PRECISIONS[precision]
    for i in range(3):
        p.left_state[i] = float(left_state[i]) if i < len(left_state) else 0.0
        p.right_state[i] = float(right_state[i]) if i < len(right_state) else 0.0
    return p


def _torch_device_buffer(nbytes: int):
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the WCC library runs only on the GPU")
    # 256-byte alignment: the caching allocator returns 512-byte aligned blocks
    buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device="cuda")
    assert buf.data_ptr() % 256 == 0
    return buf


def _torch_stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


class Solver:
    """One instance: u_t + f(u)_x = 0 advanced by the gfx950 half-step kernel."""

    def __init__(self, equation: str, P: int, N: int, bc: str = "periodic", *, limiter: bool = True,
                 precision: str = "fp64", x_left: float = 0.0, x_right: float = 1.0, a: float = 1.0,
                 gamma: float = 1.4, eps: float = 1e-40, left_state=(0.0, 0.0, 0.0),
                 right_state=(0.0, 0.0, 0.0), stream=None):
        lib = load()
        self.equation, self.P, self.N, self.bc = equation, P, N, bc
        self.nc = 3 if equation == "euler" else 1
        self.params = make_params(limiter, precision, x_left, x_right, a, gamma, eps, left_state, right_state)
        h = ctypes.c_void_p()
        _check(lib.wcc_create(EQUATIONS[equation], P, N, BCS[bc], ctypes.byref(self.params), ctypes.byref(h)),
               "wcc_create")
        self.h = h
        nb = ctypes.c_size_t()
        _check(lib.wcc_workspace_bytes(h, ctypes.byref(nb)), "wcc_workspace_bytes", h)
        self.workspace = _torch_device_buffer(nb.value)
        self.stream = stream if stream is not None else _torch_stream_handle()
        _check(lib.wcc_bind(h, ctypes.c_void_p(self.workspace.data_ptr()), nb.value, ctypes.c_void_p(self.stream)),
               "wcc_bind", h)

    def ncells(self, parity: int) -> int:
        if self.bc == "periodic":
            return self.N
        return self.N + 1 if parity % 2 == 0 else self.N

    def write(self, q: np.ndarray, parity: int = 0, t: float = 0.0) -> None:
        q = np.ascontiguousarray(q, dtype=np.float64)
        n = self.ncells(parity)
        assert q.shape == (self.nc, self.P + 1, n), (q.shape, (self.nc, self.P + 1, n))
        _check(load().wcc_write_dofs(self.h, _dptr(q), n, parity, float(t)), "wcc_write_dofs", self.h)

    def step(self, cfl: float = 0.0, dt_fixed: float = 0.0) -> None:
        _check(load().wcc_step(self.h, float(cfl), float(dt_fixed)), "wcc_step", self.h)

    def run(self, half_steps: int, cfl: float) -> None:
        _check(load().wcc_run(self.h, int(half_steps), float(cfl)), "wcc_run", self.h)

    def advance(self, t_end: float, cfl: float, max_half_steps: int = 0) -> int:
        taken = ctypes.c_int64()
        _check(load().wcc_advance(self.h, float(t_end), float(cfl), int(max_half_steps), ctypes.byref(taken)),
               "wcc_advance", self.h)
        return taken.value

    def info(self) -> wcc_state_info:
        inf = wcc_state_info()
        _check(load().wcc_read_dofs(self.h, None, 0, ctypes.byref(inf)), "wcc_read_dofs", self.h)
        return inf

    def read(self):
        inf = self.info()
        n = inf.n_cells
        out = np.empty((self.nc, self.P + 1, n), dtype=np.float64)
        _check(load().wcc_read_dofs(self.h, _dptr(out), out.size, ctypes.byref(inf)), "wcc_read_dofs", self.h)
        return out, inf

    def totals(self) -> np.ndarray:
        out = np.zeros(self.nc)
        _check(load().wcc_totals(self.h, _dptr(out)), "wcc_totals", self.h)
        return out

    def set_launch(self, threads: int = 0, blocks: int = 0, variant: int = -1) -> None:
        _check(load().wcc_set_launch(self.h, int(threads), int(blocks), int(variant)), "wcc_set_launch", self.h)

    def get_launch(self) -> dict:
        """The current launch shape: threads per block, blocks (0 = default) and kernel variant."""
        t, b, v = _c.c_int(), _c.c_int(), _c.c_int()
        _check(load().wcc_get_launch(self.h, _c.byref(t), _c.byref(b), _c.byref(v)), "wcc_get_launch", self.h)
        return {"threads": t.value, "blocks": b.value, "variant": v.value}

    def last_run_ms(self) -> float:
        ms = ctypes.c_double()
        _check(load().wcc_last_run_ms(self.h, ctypes.byref(ms)), "wcc_last_run_ms", self.h)
        return ms.value

    def close(self):
        """Destroy the context and release its device workspace (idempotent)."""
        if getattr(self, "h", None):
            load().wcc_destroy(self.h)
            self.h = None
        self.workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent instances advanced together by persistent kernels."""

    def __init__(self, equation: str, P, N, bc: str = "transmissive", *, limiter: bool = True,
                 precision: str = "fp32_mixed", x_left: float = 0.0, x_right: float = 1.0, a: float = 1.0,
                 gamma: float = 1.4, eps: float = 1e-40, stream=None):
        lib = load()
        self.P = np.ascontiguousarray(P, dtype=np.int32)
        self.N = np.ascontiguousarray(N, dtype=np.int64)
        self.B = int(self.P.size)
        self.bc = bc
        self.nc = 3 if equation == "euler" else 1
        self.params = make_params(limiter, precision, x_left, x_right, a, gamma, eps)
        h = ctypes.c_void_p()
        _check(lib.wcc_batch_create(EQUATIONS[equation], self.B,
                                    self.P.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    self.N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), BCS[bc],
                                    ctypes.byref(self.params), ctypes.byref(h)), "wcc_batch_create")
        self.h = h
        nb = ctypes.c_size_t()
        _check(lib.wcc_batch_workspace_bytes(h, ctypes.byref(nb)), "wcc_batch_workspace_bytes", h, True)
        self.workspace = _torch_device_buffer(nb.value)
        self.stream = stream if stream is not None else _torch_stream_handle()
        _check(lib.wcc_batch_bind(h, ctypes.c_void_p(self.workspace.data_ptr()), nb.value,
                                  ctypes.c_void_p(self.stream)), "wcc_batch_bind", h, True)

    def rebind(self) -> None:
        """Bind the same workspace again: every instance restarts at t = 0 with
        an empty time-control ring (the states must be written again)."""
        _check(load().wcc_batch_bind(self.h, ctypes.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                     ctypes.c_void_p(self.stream)), "wcc_batch_bind", self.h, True)

    def ncells(self, b: int, parity: int) -> int:
        if self.bc == "periodic":
            return int(self.N[b])
        return int(self.N[b]) + 1 if parity % 2 == 0 else int(self.N[b])

    def write(self, b: int, q: np.ndarray, t: float = 0.0) -> None:
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == (self.nc, int(self.P[b]) + 1, self.ncells(b, 0))
        _check(load().wcc_batch_write_dofs(self.h, int(b), _dptr(q), q.shape[2], float(t)),
               "wcc_batch_write_dofs", self.h, True)

    def prepare(self) -> None:
        _check(load().wcc_batch_prepare(self.h), "wcc_batch_prepare", self.h, True)

    def advance(self, half_steps: int, cfl_by_P) -> None:
        """wcc_batch_advance: enqueue half_steps half-steps of every instance."""
        c = np.zeros(WCC_PMAX + 1)
        c[: len(cfl_by_P)] = cfl_by_P
        _check(load().wcc_batch_advance(self.h, int(half_steps), _dptr(c)), "wcc_batch_advance", self.h, True)

    run = advance

    def read(self, b: int):
        inf = wcc_state_info()
        _check(load().wcc_batch_read_dofs(self.h, int(b), None, 0, ctypes.byref(inf)), "wcc_batch_read_dofs",
               self.h, True)
        out = np.empty((self.nc, int(self.P[b]) + 1, inf.n_cells))
        _check(load().wcc_batch_read_dofs(self.h, int(b), _dptr(out), out.size, ctypes.byref(inf)),
               "wcc_batch_read_dofs", self.h, True)
        return out, inf

    def set_schedule(self, threads: int = 0, blocks: int = 0, mode: int = 0) -> None:
        _check(load().wcc_batch_set_schedule(self.h, int(threads), int(blocks), int(mode)),
               "wcc_batch_set_schedule", self.h, True)

    def last_run_ms(self) -> float:
        ms = ctypes.c_double()
        _check(load().wcc_batch_last_run_ms(self.h, ctypes.byref(ms)), "wcc_batch_last_run_ms", self.h, True)
        return ms.value

    def close(self):
        """Destroy the batch and release its device workspace (idempotent)."""
        if getattr(self, "h", None):
            load().wcc_batch_destroy(self.h)
            self.h = None
        self.workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


DOF2D_NOTE = "DOF order: k + l ascending, then l ascending; index (k+l)(k+l+1)/2 + l"


class Solver2D:
    """One 2D instance on a rectangle of Nx x Ny intervals, periodic or with
    transmissive edges: u_t + f(u)_x + g(u)_y = 0 advanced by the gfx950 2D
    half-step kernel.  States are numpy arrays of shape (nc, ndof, ny, nx) in
    DOF order, nx x ny the cells of the state's mesh (`mesh_shape`)."""

    def __init__(self, equation: str, P: int, Nx: int, Ny: int, *, limiter: bool = True, x_left: float = 0.0,
                 x_right: float = 1.0, y_left: float = 0.0, y_right: float = 1.0, a: float = 1.0, b: float = 1.0,
                 gamma: float = 1.4, eps: float = 1e-40, bc="periodic", stream=None):
        lib = load()
        bcs = (bc, bc) if isinstance(bc, str) else tuple(bc)
        if len(bcs) != 2 or any(b not in ("periodic", "transmissive") for b in bcs):
            raise ValueError(f"2D boundary {bc!r}: periodic or transmissive, or a pair (x, y) of them")
        self.bcs = bcs
        self.equation, self.P, self.Nx, self.Ny, self.bc = equation, P, Nx, Ny, bc
        self.nc = 4 if equation == "euler" else 1
        self.nd = (P + 1) * (P + 2) // 2
        p = wcc2d_params()
        lib.wcc2d_params_default(ctypes.byref(p))
        p.x_left, p.x_right, p.y_left, p.y_right = x_left, x_right, y_left, y_right
        p.a, p.b, p.gamma, p.eps = a, b, gamma, eps
        p.limiter = 1 if limiter else 0
        p.bc, p.bc_y = BCS[bcs[0]], BCS[bcs[1]]
        self.params = p
        h = ctypes.c_void_p()
        _check(lib.wcc2d_create(EQUATIONS[equation], P, Nx, Ny, ctypes.byref(p), ctypes.byref(h)), "wcc2d_create")
        self.h = h
        nb = ctypes.c_size_t()
        _check(lib.wcc2d_workspace_bytes(h, ctypes.byref(nb)), "wcc2d_workspace_bytes", h, two_d=True)
        self.workspace = _torch_device_buffer(nb.value)
        self.stream = stream if stream is not None else _torch_stream_handle()
        _check(lib.wcc2d_bind(h, ctypes.c_void_p(self.workspace.data_ptr()), nb.value, ctypes.c_void_p(self.stream)),
               "wcc2d_bind", h, two_d=True)

    def mesh_shape(self, parity: int) -> tuple:
        ex = 1 if (self.bcs[0] == "transmissive" and parity % 2 == 0) else 0
        ey = 1 if (self.bcs[1] == "transmissive" and parity % 2 == 0) else 0
        return (self.nc, self.nd, self.Ny + ey, self.Nx + ex)

    @property
    def shape(self):
        """State shape on the parity-0 mesh."""
        return self.mesh_shape(0)

    def write(self, q: np.ndarray, parity: int = 0, t: float = 0.0) -> None:
        q = np.ascontiguousarray(q, dtype=np.float64)
        assert q.shape == self.mesh_shape(parity), (q.shape, self.mesh_shape(parity))
        _check(load().wcc2d_write_dofs(self.h, _dptr(q), parity, float(t)), "wcc2d_write_dofs", self.h, two_d=True)

    def step(self, cfl: float = 0.0, dt_fixed: float = 0.0) -> None:
        _check(load().wcc2d_step(self.h, float(cfl), float(dt_fixed)), "wcc2d_step", self.h, two_d=True)

    def run(self, half_steps: int, cfl: float) -> None:
        _check(load().wcc2d_run(self.h, int(half_steps), float(cfl)), "wcc2d_run", self.h, two_d=True)

    def advance(self, t_end: float, cfl: float, max_half_steps: int = 0) -> int:
        taken = ctypes.c_int64()
        _check(load().wcc2d_advance(self.h, float(t_end), float(cfl), int(max_half_steps), ctypes.byref(taken)),
               "wcc2d_advance", self.h, two_d=True)
        return taken.value

    def info(self) -> wcc2d_state_info:
        inf = wcc2d_state_info()
        _check(load().wcc2d_read_dofs(self.h, None, 0, ctypes.byref(inf)), "wcc2d_read_dofs", self.h, two_d=True)
        return inf

    def read(self):
        q = np.empty(self.mesh_shape(self.info().parity), dtype=np.float64)
        inf = wcc2d_state_info()
        _check(load().wcc2d_read_dofs(self.h, _dptr(q), q.size, ctypes.byref(inf)), "wcc2d_read_dofs", self.h,
               two_d=True)
        return q, inf

    def totals(self) -> np.ndarray:
        """Sum of the cell averages times dx dy per component (host sum)."""
        out = np.zeros(self.nc)
        _check(load().wcc2d_totals(self.h, _dptr(out)), "wcc2d_totals", self.h, two_d=True)
        return out

    def set_launch(self, threads: int = 0, blocks: int = 0, variant: int = -1) -> None:
        _check(load().wcc2d_set_launch(self.h, int(threads), int(blocks), int(variant)), "wcc2d_set_launch", self.h,
               two_d=True)

    def get_launch(self) -> dict:
        """The launch shape of the next half-step, with the effective block count."""
        t, b, v = _c.c_int(), _c.c_int(), _c.c_int()
        _check(load().wcc2d_get_launch(self.h, _c.byref(t), _c.byref(b), _c.byref(v)), "wcc2d_get_launch", self.h,
               two_d=True)
        return {"threads": t.value, "blocks": b.value, "variant": v.value}

    def last_run_ms(self) -> float:
        ms = ctypes.c_double()
        _check(load().wcc2d_last_run_ms(self.h, ctypes.byref(ms)), "wcc2d_last_run_ms", self.h, two_d=True)
        return ms.value

    def close(self) -> None:
        """Destroy the context and release its device workspace (idempotent)."""
        if getattr(self, "h", None):
            load().wcc2d_destroy(self.h)
            self.h = None
        self.workspace = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
