"""FP64 CPU oracle of the 1D WCC half-step (Shen & Parsani, arXiv:2104.04347).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the product package.  The arithmetic
lives in wcc_oracle.cpp (plain C++, binary64); this module only marshals
numpy arrays through ctypes.

State arrays have shape (nc, P+1, n): component, k, cell, with k = 0 the point
value and k >= 1 the scaled derivative u_kx = dx^k d^k u/dx^k at the cell
centre (Eq. 1D_Derivative_DEF, Eq. 1DPolynomial_Space).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

EQUATIONS = {"advection": 0, "burgers": 1, "euler": 2}
BCS = {"periodic": 0, "transmissive": 1, "dirichlet": 2}


class _Problem(ctypes.Structure):
    _fields_ = [
        ("equation", ctypes.c_int32),
        ("P", ctypes.c_int32),
        ("N", ctypes.c_int64),
        ("bc", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("x_left", ctypes.c_double),
        ("x_right", ctypes.c_double),
        ("a", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("eps", ctypes.c_double),
        ("left_state", ctypes.c_double * 3),
        ("right_state", ctypes.c_double * 3),
    ]


_lib = None
_lib2d = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    lib.wcc_oracle_threads.argtypes = []
    lib.wcc_oracle_threads.restype = ctypes.c_int
    lib.wcc_oracle_ncells.argtypes = [P(_Problem), ctypes.c_int]
    lib.wcc_oracle_ncells.restype = ctypes.c_int64
    lib.wcc_oracle_half_step.argtypes = [P(_Problem), ctypes.c_int, dp, ctypes.c_double, dp, dp]
    lib.wcc_oracle_half_step.restype = ctypes.c_int
    lib.wcc_oracle_max_speed.argtypes = [P(_Problem), ctypes.c_int, dp]
    lib.wcc_oracle_max_speed.restype = ctypes.c_double
    lib.wcc_oracle_run.argtypes = [P(_Problem), P(ctypes.c_int), dp, dp, dp, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int64, P(ctypes.c_int)]
    lib.wcc_oracle_run.restype = ctypes.c_int64
    lib.wcc_oracle_count_flops.argtypes = [P(_Problem), dp, dp, ctypes.c_double, dp]
    lib.wcc_oracle_count_flops.restype = ctypes.c_int
    lib.wcc_oracle_half_step_parts.argtypes = [P(_Problem), ctypes.c_int, dp, ctypes.c_double, dp, dp, dp, dp]
    lib.wcc_oracle_half_step_parts.restype = ctypes.c_int
    lib.wcc_oracle_ck_triangle.argtypes = [P(_Problem), dp, ctypes.c_double, dp]
    lib.wcc_oracle_ck_triangle.restype = ctypes.c_int
    lib.wcc_oracle_js_indicator.argtypes = [ctypes.c_int, dp]
    lib.wcc_oracle_js_indicator.restype = ctypes.c_double
    lib.wcc_oracle_limit_field.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, dp,
                                           ctypes.c_double, ctypes.c_double]
    lib.wcc_oracle_limit_field.restype = ctypes.c_int
    lib.wcc_oracle_euler_eigen.argtypes = [ctypes.c_double, dp, dp, dp]
    lib.wcc_oracle_euler_eigen.restype = ctypes.c_int
    _lib = lib
    return lib


class use_library:
    """Context manager that points this module at another build of the oracle
    source (the mutation tests compile deliberately broken copies)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib, _lib2d, _LIB_PATH
        self._saved = (_lib, _lib2d, _LIB_PATH)
        _lib, _lib2d, _LIB_PATH = None, None, self.path
        return _load()

    def __exit__(self, *exc):
        global _lib, _lib2d, _LIB_PATH
        _lib, _lib2d, _LIB_PATH = self._saved
        return False


LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")


def threads() -> int:
    """Threads one half-step of the loaded build uses (1 unless it is the
    OpenMP build, liboracle_omp.so, selected with use_library)."""
    return int(_load().wcc_oracle_threads())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Problem:
    """u_t + f(u)_x = 0 on [x_left, x_right] (Eq. 1DHCL / Eq. 1DHCLSystem)."""
    equation: str
    P: int
    N: int
    bc: object = "periodic"     # "periodic", "transmissive" or a pair (x, y) of them
    limiter: bool = False
    x_left: float = 0.0
    x_right: float = 1.0
    a: float = 1.0
    gamma: float = 1.4
    eps: float = 1e-40
    left_state: tuple = (0.0, 0.0, 0.0)
    right_state: tuple = (0.0, 0.0, 0.0)

    @property
    def nc(self) -> int:
        return 3 if self.equation == "euler" else 1

    @property
    def dx(self) -> float:
        return (self.x_right - self.x_left) / self.N

    def c_struct(self) -> _Problem:
        s = _Problem()
        s.equation = EQUATIONS[self.equation]
        s.P = self.P
        s.N = self.N
        s.bc = BCS[self.bc]
        s.limiter = 1 if self.limiter else 0
        s.x_left = self.x_left
        s.x_right = self.x_right
        s.a = self.a
        s.gamma = self.gamma
        s.eps = self.eps
        for i in range(3):
            s.left_state[i] = float(self.left_state[i]) if i < len(self.left_state) else 0.0
            s.right_state[i] = float(self.right_state[i]) if i < len(self.right_state) else 0.0
        return s

    def ncells(self, parity: int) -> int:
        if self.bc == "periodic":
            return self.N
        return self.N + 1 if parity % 2 == 0 else self.N

    def centers(self, parity: int) -> np.ndarray:
        """Cell centres x_L + (j + parity/2) dx (Section 2.1, mesh definition)."""
        n = self.ncells(parity)
        return self.x_left + (np.arange(n, dtype=np.float64) + 0.5 * (parity % 2)) * self.dx


def half_step(pb: Problem, parity: int, q: np.ndarray, dt: float):
    """One half-step with time step dt.  Returns (q_new, smax_new, flags)."""
    lib = _load()
    n_old = pb.ncells(parity)
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == (pb.nc, pb.P + 1, n_old), (q.shape, (pb.nc, pb.P + 1, n_old))
    out = np.empty((pb.nc, pb.P + 1, pb.ncells(1 - parity)), dtype=np.float64)
    sm = ctypes.c_double(0.0)
    cs = pb.c_struct()
    f = lib.wcc_oracle_half_step(ctypes.byref(cs), parity, _dp(q), float(dt), _dp(out), ctypes.byref(sm))
    if f < 0:
        raise ValueError("oracle rejected the problem")
    return out, sm.value, f


def max_speed(pb: Problem, parity: int, q: np.ndarray) -> float:
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == (pb.nc, pb.P + 1, pb.ncells(parity))
    cs = pb.c_struct()
    return lib.wcc_oracle_max_speed(ctypes.byref(cs), parity, _dp(q))


@dataclass
class RunResult:
    q: np.ndarray
    parity: int
    t: float
    smax: float
    half_steps: int
    flags: int


def run(pb: Problem, q: np.ndarray, parity: int = 0, t: float = 0.0, t_end: float = float("inf"),
        cfl: float = 0.0, dt_fixed: float = 0.0, max_half_steps: int = 1 << 62,
        smax: float | None = None) -> RunResult:
    """March half-steps: dt = (cfl*dx)/smax clipped to t_end, or dt_fixed."""
    lib = _load()
    n0 = pb.ncells(parity)
    nmax = max(pb.ncells(0), pb.ncells(1))
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == (pb.nc, pb.P + 1, n0)
    buf = np.zeros(pb.nc * (pb.P + 1) * nmax, dtype=np.float64)
    buf[: q.size] = q.reshape(-1)
    if smax is None:
        smax = max_speed(pb, parity, q)
    cp = ctypes.c_int(parity)
    ct = ctypes.c_double(t)
    cs_ = ctypes.c_double(smax)
    fl = ctypes.c_int(0)
    cs = pb.c_struct()
    taken = lib.wcc_oracle_run(ctypes.byref(cs), ctypes.byref(cp), ctypes.byref(ct), ctypes.byref(cs_),
                               _dp(buf), float(t_end), float(cfl), float(dt_fixed), int(max_half_steps),
                               ctypes.byref(fl))
    if taken < 0:
        raise ValueError("oracle rejected the problem")
    n1 = pb.ncells(cp.value)
    qn = buf[: pb.nc * (pb.P + 1) * n1].reshape(pb.nc, pb.P + 1, n1).copy()
    return RunResult(qn, cp.value, ct.value, cs_.value, int(taken), fl.value)


def count_flops(pb: Problem, q_left: np.ndarray, q_right: np.ndarray, lam: float) -> dict:
    """Floating-point operations per new cell (one old cell + one new cell)."""
    lib = _load()
    ql = np.ascontiguousarray(q_left, dtype=np.float64).reshape(-1)
    qr = np.ascontiguousarray(q_right, dtype=np.float64).reshape(-1)
    assert ql.size == pb.nc * (pb.P + 1) and qr.size == ql.size
    out = np.zeros(6, dtype=np.float64)
    cs = pb.c_struct()
    if lib.wcc_oracle_count_flops(ctypes.byref(cs), _dp(ql), _dp(qr), float(lam), _dp(out)) != 0:
        raise ValueError("oracle rejected the problem")
    keys = ["add", "mul", "fma", "div", "sqrt", "flops"]
    return {k: float(v) for k, v in zip(keys, out)}


def half_step_parts(pb: Problem, parity: int, q: np.ndarray, dt: float):
    """Unlimited half-step pieces per new cell: (abar, d, vl, vr) with shapes
    (nc, n), (nc, P+1, n), (nc, n), (nc, n).  Periodic problems only."""
    lib = _load()
    q = np.ascontiguousarray(q, dtype=np.float64)
    n = pb.ncells(1 - parity)
    abar = np.empty((pb.nc, n))
    d = np.empty((pb.nc, pb.P + 1, n))
    vl = np.empty((pb.nc, n))
    vr = np.empty((pb.nc, n))
    cs = pb.c_struct()
    if lib.wcc_oracle_half_step_parts(ctypes.byref(cs), parity, _dp(q), float(dt), _dp(abar), _dp(d),
                                      _dp(vl), _dp(vr)) != 0:
        raise ValueError("oracle rejected the problem")
    return abar, d, vl, vr


def ck_triangle(pb: Problem, q_cell: np.ndarray, lam: float) -> np.ndarray:
    """T[c, k, m] = u_{kx,mt}/(k! m!) of one cell state q_cell (nc, P+1)."""
    lib = _load()
    q = np.ascontiguousarray(q_cell, dtype=np.float64).reshape(-1)
    T = np.zeros((pb.nc, pb.P + 1, pb.P + 1))
    cs = pb.c_struct()
    if lib.wcc_oracle_ck_triangle(ctypes.byref(cs), _dp(q), float(lam), _dp(T)) != 0:
        raise ValueError("oracle rejected the problem")
    return T


def js_indicator(P: int, d: np.ndarray) -> float:
    lib = _load()
    dd = np.ascontiguousarray(d, dtype=np.float64)
    assert dd.size == P + 1
    return lib.wcc_oracle_js_indicator(P, _dp(dd))


def limit_field(P: int, abar: float, d: np.ndarray, vl: float, vr: float, eps: float = 1e-40) -> np.ndarray:
    lib = _load()
    dd = np.array(d, dtype=np.float64)
    assert dd.size == P + 1
    if lib.wcc_oracle_limit_field(P, float(eps), float(abar), _dp(dd), float(vl), float(vr)) != 0:
        raise ValueError("bad limiter arguments")
    return dd


def euler_eigen(gamma: float, U) -> tuple[np.ndarray, np.ndarray]:
    lib = _load()
    u = np.ascontiguousarray(U, dtype=np.float64)
    L = np.empty((3, 3))
    R = np.empty((3, 3))
    lib.wcc_oracle_euler_eigen(float(gamma), _dp(u), _dp(L), _dp(R))
    return L, R


# ---------------------------------------------------------------------------
# 2D half-step (wcc2d_oracle.cpp): Section 3 and Appendix B of the paper on a
# periodic Cartesian mesh.  State arrays have shape (nc, ndof, Ny, Nx): the
# DOFs u_{kx,ly} in "DOF order" (total degree k + l ascending, then l
# ascending), index 0 the point value.
# ---------------------------------------------------------------------------
class _Problem2D(ctypes.Structure):
    _fields_ = [
        ("equation", ctypes.c_int32),
        ("P", ctypes.c_int32),
        ("Nx", ctypes.c_int64),
        ("Ny", ctypes.c_int64),
        ("limiter", ctypes.c_int32),
        ("bc", ctypes.c_int32),
        ("bc_y", ctypes.c_int32),
        ("pad2", ctypes.c_int32),
        ("x_left", ctypes.c_double),
        ("x_right", ctypes.c_double),
        ("y_left", ctypes.c_double),
        ("y_right", ctypes.c_double),
        ("a", ctypes.c_double),
        ("b", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("eps", ctypes.c_double),
    ]


def _load2d():
    global _lib2d
    if _lib2d is not None:
        return _lib2d
    lib = _load()
    P = ctypes.POINTER
    dp = P(ctypes.c_double)
    lib.wcc2d_oracle_old_cell.argtypes = [P(_Problem2D), dp, ctypes.c_double, dp]
    lib.wcc2d_oracle_old_cell.restype = ctypes.c_int32
    lib.wcc2d_oracle_js_indicator.argtypes = [ctypes.c_int32, dp]
    lib.wcc2d_oracle_js_indicator.restype = ctypes.c_double
    lib.wcc2d_oracle_ndof.argtypes = [ctypes.c_int32]
    lib.wcc2d_oracle_ndof.restype = ctypes.c_int64
    lib.wcc2d_oracle_max_speed.argtypes = [P(_Problem2D), ctypes.c_int32, dp, P(ctypes.c_int32)]
    lib.wcc2d_oracle_max_speed.restype = ctypes.c_double
    lib.wcc2d_oracle_half_step.argtypes = [P(_Problem2D), ctypes.c_int32, dp, ctypes.c_double, dp, dp,
                                           P(ctypes.c_int32)]
    lib.wcc2d_oracle_half_step.restype = ctypes.c_int32
    lib.wcc2d_oracle_run.argtypes = [P(_Problem2D), P(ctypes.c_int32), dp, dp, dp, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_double, ctypes.c_int64, P(ctypes.c_int32)]
    lib.wcc2d_oracle_run.restype = ctypes.c_int64
    _lib2d = lib
    return lib


def ndof2d(P: int) -> int:
    return (P + 1) * (P + 2) // 2


def dof2d(k: int, l: int) -> int:
    n = k + l
    return n * (n + 1) // 2 + l


BCS2D = {"periodic": 0, "transmissive": 1}


@dataclass
class Problem2D:
    """u_t + f(u)_x + g(u)_y = 0 on a rectangle (Eq. 2DHCL); advection
    f = a u, g = b u; Burgers f = g = u^2/2; Euler (rho, rho u, rho v, rho e),
    limited in the characteristic fields of the rotated decomposition
    (Section 4).  `bc` names the edges of both directions, or is a pair
    (x, y).  Periodic: N cells on both meshes in that direction.
    Transmissive: the mesh of parity 0 has the N+1 cells centred at the mesh
    points (edges included), parity 1 the N cells between them (Section
    3.1); ghosts copy the adjacent cell."""
    equation: str
    P: int
    Nx: int
    Ny: int
    limiter: bool = False
    x_left: float = 0.0
    x_right: float = 1.0
    y_left: float = 0.0
    y_right: float = 1.0
    a: float = 1.0
    b: float = 1.0
    gamma: float = 1.4
    eps: float = 1e-40
    bc: object = "periodic"     # "periodic", "transmissive" or a pair (x, y) of them

    @property
    def nc(self) -> int:
        return 4 if self.equation == "euler" else 1

    @property
    def nd(self) -> int:
        return ndof2d(self.P)

    @property
    def bcs(self) -> tuple:
        return (self.bc, self.bc) if isinstance(self.bc, str) else tuple(self.bc)

    def mesh(self, parity: int) -> tuple:
        """(cells in x, cells in y) of the mesh of this parity."""
        bx, by = self.bcs
        ex = 1 if (bx == "transmissive" and parity % 2 == 0) else 0
        ey = 1 if (by == "transmissive" and parity % 2 == 0) else 0
        return self.Nx + ex, self.Ny + ey

    def mesh_shape(self, parity: int) -> tuple:
        nx, ny = self.mesh(parity)
        return (self.nc, self.nd, ny, nx)

    @property
    def dx(self) -> float:
        return (self.x_right - self.x_left) / self.Nx

    @property
    def dy(self) -> float:
        return (self.y_right - self.y_left) / self.Ny

    @property
    def shape(self):
        """State shape on the parity-0 mesh."""
        return self.mesh_shape(0)

    def c_struct(self) -> _Problem2D:
        s = _Problem2D()
        s.equation = EQUATIONS[self.equation]
        s.P, s.Nx, s.Ny = self.P, self.Nx, self.Ny
        s.limiter = 1 if self.limiter else 0
        s.bc = BCS2D[self.bcs[0]]
        s.bc_y = BCS2D[self.bcs[1]]
        s.x_left, s.x_right, s.y_left, s.y_right = self.x_left, self.x_right, self.y_left, self.y_right
        s.a, s.b, s.gamma, s.eps = self.a, self.b, self.gamma, self.eps
        return s


def old_cell2d(pb: Problem2D, q: np.ndarray, dt: float) -> dict:
    """Per-old-cell quantities of one cell (state q of shape (nc, ndof)):
    quarter-cell averages RU, RD, LU, LD, half-edge flux averages fU, fD, gR,
    gL (arrays over components) and vertex values V[c][(k, l)], k + l < P."""
    lib = _load2d()
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == (pb.nc, pb.nd)
    nv = pb.P * (pb.P + 1) // 2
    out = np.zeros(pb.nc * (8 + nv))
    cs = pb.c_struct()
    if lib.wcc2d_oracle_old_cell(ctypes.byref(cs), _dp(q), float(dt), _dp(out)) != 0:
        raise ValueError("oracle rejected the 2D problem")
    head = out[: 8 * pb.nc].reshape(pb.nc, 8)
    res = {name: head[:, i].copy() for i, name in enumerate(("RU", "RD", "LU", "LD", "fU", "fD", "gR", "gL"))}
    pairs = [(n - l, l) for n in range(pb.P) for l in range(n + 1)]
    tail = out[8 * pb.nc:].reshape(pb.nc, nv)
    res["V"] = [{kl: tail[c, i] for i, kl in enumerate(pairs)} for c in range(pb.nc)]
    return res


def js_indicator2d(P: int, d: np.ndarray) -> float:
    """Eq. 2DSmoothIndicator of the polynomial with scaled derivatives d (DOF order)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    assert d.shape == (ndof2d(P),)
    return _load2d().wcc2d_oracle_js_indicator(int(P), _dp(d))


def max_speed2d(pb: Problem2D, q: np.ndarray, parity: int = 0) -> tuple:
    """(largest s_x/dx + s_y/dy over the stored averages, status bits)."""
    lib = _load2d()
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == pb.mesh_shape(parity)
    fl = ctypes.c_int32(0)
    cs = pb.c_struct()
    v = lib.wcc2d_oracle_max_speed(ctypes.byref(cs), int(parity), _dp(q), ctypes.byref(fl))
    return v, fl.value


def half_step2d(pb: Problem2D, parity: int, q: np.ndarray, dt: float):
    """One half-step from mesh `parity`: (new state, smax of the new averages, flags)."""
    lib = _load2d()
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == pb.mesh_shape(parity)
    out = np.empty(pb.mesh_shape(1 - parity))
    sm = ctypes.c_double(0.0)
    fl = ctypes.c_int32(0)
    cs = pb.c_struct()
    rc = lib.wcc2d_oracle_half_step(ctypes.byref(cs), int(parity), _dp(q), float(dt), _dp(out), ctypes.byref(sm),
                                    ctypes.byref(fl))
    if rc != 0:
        raise ValueError("oracle rejected the 2D problem")
    return out, sm.value, fl.value


def run2d(pb: Problem2D, q: np.ndarray, parity: int = 0, t: float = 0.0, t_end: float = float("inf"),
          cfl: float = 0.0, dt_fixed: float = 0.0, max_half_steps: int = 1 << 62) -> "RunResult":
    """March 2D half-steps: dt = cfl / smax (smax the largest s_x/dx + s_y/dy),
    clipped to t_end, or dt_fixed."""
    lib = _load2d()
    q = np.ascontiguousarray(q, dtype=np.float64)
    assert q.shape == pb.mesh_shape(parity)
    # room for the larger mesh: the state changes mesh every half-step
    buf = np.zeros(pb.nc * pb.nd * (pb.Nx + 1) * (pb.Ny + 1))
    buf[: q.size] = q.ravel()
    smax, _ = max_speed2d(pb, q, parity)
    cp = ctypes.c_int32(parity)
    ct = ctypes.c_double(t)
    cs_ = ctypes.c_double(smax)
    fl = ctypes.c_int32(0)
    cs = pb.c_struct()
    taken = lib.wcc2d_oracle_run(ctypes.byref(cs), ctypes.byref(cp), ctypes.byref(ct), ctypes.byref(cs_), _dp(buf),
                                 float(t_end), float(cfl), float(dt_fixed), int(max_half_steps), ctypes.byref(fl))
    if taken < 0:
        raise ValueError("oracle rejected the 2D problem")
    shp = pb.mesh_shape(cp.value)
    out = buf[: int(np.prod(shp))].reshape(shp).copy()
    return RunResult(out, cp.value, ct.value, cs_.value, int(taken), fl.value)
