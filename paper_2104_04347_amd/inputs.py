"""Seeded synthetic initial data shared by the GPU path's tests, the benchmark
and the CPU oracle's tests.

This module holds problem data only -- initial conditions, their exact
derivatives and exact cell integrals -- and none of the scheme's arithmetic.
Every generator returns a state array of shape (nc, P+1, n) in float64 with

* k = 0: the point value u0(x_j) at the cell centre, and
* k >= 1: the scaled derivative dx^k u0^(k)(x_j) (Eq. 1D_Derivative_DEF),

so that the cell polynomial of Eq. 1DPolynomial_Space is the degree-P Taylor
polynomial of u0 at the centre.  A cell whose interior contains a jump of u0
gets the exact mean of u0 over the cell (Gauss-Legendre on each smooth piece)
as its value and zero derivatives.  The same bytes are fed to both
implementations.

Euler states are conserved variables (rho, rho u, rho e) with
rho e = p/(gamma-1) + rho u^2/2 (Section 5.2 of the paper, perfect gas).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

_GL_X, _GL_W = np.polynomial.legendre.leggauss(12)


def centers(x_left: float, x_right: float, N: int, n_cells: int, parity: int) -> np.ndarray:
    dx = (x_right - x_left) / N
    return x_left + (np.arange(n_cells, dtype=np.float64) + 0.5 * (parity % 2)) * dx


def n_cells(N: int, bc: str, parity: int) -> int:
    if bc == "periodic":
        return N
    return N + 1 if parity % 2 == 0 else N


# ---------------------------------------------------------------------------
# Smooth scalar data: constant + sum of sines  c0 + sum_m A_m sin(w_m x + phi_m)
# ---------------------------------------------------------------------------
@dataclass
class SineSum:
    c0: float
    amps: np.ndarray
    freqs: np.ndarray   # angular wavenumbers w_m
    phases: np.ndarray

    def deriv(self, x: np.ndarray, k: int) -> np.ndarray:
        """k-th derivative of u0 at x."""
        out = np.full_like(x, self.c0 if k == 0 else 0.0, dtype=np.float64)
        for a, w, ph in zip(self.amps, self.freqs, self.phases):
            out = out + a * w ** k * np.sin(w * x + ph + k * np.pi / 2)
        return out

    def __call__(self, x):
        return self.deriv(np.asarray(x, dtype=np.float64), 0)


def taylor_scalar(fn: SineSum, x: np.ndarray, dx: float, P: int) -> np.ndarray:
    q = np.empty((1, P + 1, x.size), dtype=np.float64)
    for k in range(P + 1):
        q[0, k] = dx ** k * fn.deriv(x, k)
    return q


def sine_wave(P: int, N: int, x_left: float, x_right: float, c0: float = 0.0, amp: float = 1.0,
              w: float = np.pi, phase: float = 0.0, bc: str = "periodic", parity: int = 0):
    """u0 = c0 + amp*sin(w x + phase) on the mesh of the given parity."""
    fn = SineSum(c0, np.array([amp]), np.array([w]), np.array([phase]))
    x = centers(x_left, x_right, N, n_cells(N, bc, parity), parity)
    return taylor_scalar(fn, x, (x_right - x_left) / N, P), fn


def burgers_modes(seed: int, P: int, N: int, x_left: float = 0.0, x_right: float = 2.0,
                  n_modes: int = 3, c0: float = 0.5):
    """u0 = c0 + sum of n_modes sines A_m sin(k_m pi x + phi_m), A_m ~ U(0, 0.5),
    k_m uniform in {1,2,3,4}, phi_m ~ U(0, 2 pi), periodic on [0, 2]."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(0.0, 0.5, n_modes)
    ks = rng.integers(1, 5, n_modes)
    phases = rng.uniform(0.0, 2 * np.pi, n_modes)
    fn = SineSum(c0, amps, ks * np.pi, phases)
    x = centers(x_left, x_right, N, N, 0)
    return taylor_scalar(fn, x, (x_right - x_left) / N, P), fn


# ---------------------------------------------------------------------------
# Piecewise Euler data: states (rho_s, u_s, p_s) with rho = rho_s*(1 + A sin(w x))
# ---------------------------------------------------------------------------
@dataclass
class EulerPiecewise:
    breaks: np.ndarray      # sorted jump positions inside the domain
    rho: np.ndarray         # per piece (len(breaks)+1)
    u: np.ndarray
    p: np.ndarray
    gamma: float = 1.4
    sine_amp: float = 0.2
    sine_w: float = 5.0
    period: tuple | None = None   # (x_left, x_right) when the data wraps around
    wrap_jump: bool = True        # periodic data: the state jumps at x_left == x_right
    piece_sine: np.ndarray | None = None   # per-piece factor on sine_amp (None: 1 everywhere)

    def piece(self, x: np.ndarray) -> np.ndarray:
        return np.searchsorted(self.breaks, x, side="right")

    def _wrap(self, x):
        if self.period is None:
            return x
        a, b = self.period
        return a + np.mod(x - a, b - a)

    def conserved_deriv(self, x: np.ndarray, k: int) -> np.ndarray:
        """k-th x-derivative of (rho, rho u, rho e) at x, shape (3, len(x))."""
        xw = self._wrap(np.asarray(x, dtype=np.float64))
        i = self.piece(xw)
        rs, us, ps = self.rho[i], self.u[i], self.p[i]
        w = self.sine_w
        amp = self.sine_amp if self.piece_sine is None else self.sine_amp * np.asarray(self.piece_sine)[i]
        if k == 0:
            rho = rs * (1.0 + amp * np.sin(w * xw))
            return np.stack([rho, rho * us, ps / (self.gamma - 1.0) + 0.5 * rho * us * us])
        drho = rs * amp * w ** k * np.sin(w * xw + k * np.pi / 2)
        return np.stack([drho, drho * us, 0.5 * drho * us * us])

    def cell_mean(self, xa: float, xb: float) -> np.ndarray:
        """Exact mean of the conserved variables over [xa, xb] (Gauss-Legendre
        on each smooth piece)."""
        pts = [xa]
        if self.period is None:
            inner = [b for b in self.breaks if xa < b < xb]
        else:
            a, b0 = self.period
            L = b0 - a
            inner = []
            cand = list(self.breaks) + ([a] if self.wrap_jump else [])
            for sh in (-L, 0.0, L):
                inner += [b + sh for b in cand if xa < b + sh < xb]
            inner = sorted(inner)
        pts += inner + [xb]
        tot = np.zeros(3)
        for lo, hi in zip(pts[:-1], pts[1:]):
            if hi <= lo:
                continue
            mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
            xs = mid + half * _GL_X
            # evaluate inside the piece: nudge the nodes away from the jump by construction
            vals = self.conserved_deriv(xs, 0)
            tot += half * (vals * _GL_W).sum(axis=1)
        return tot / (xb - xa)

    def jumps_in(self, xa: float, xb: float) -> bool:
        if self.period is None:
            return any(xa < b < xb for b in self.breaks)
        a, b0 = self.period
        L = b0 - a
        cand = list(self.breaks) + ([a] if self.wrap_jump else [])
        return any(xa < b + sh < xb for b in cand for sh in (-L, 0.0, L))


def euler_taylor(data: EulerPiecewise, x: np.ndarray, dx: float, P: int) -> np.ndarray:
    q = np.empty((3, P + 1, x.size), dtype=np.float64)
    for k in range(P + 1):
        q[:, k, :] = dx ** k * data.conserved_deriv(x, k)
    for j in jump_cells(data, x, dx):
        xa, xb = x[j] - 0.5 * dx, x[j] + 0.5 * dx
        q[:, 0, j] = data.cell_mean(xa, xb)
        q[:, 1:, j] = 0.0
    return q


def jump_cells(data: EulerPiecewise, x: np.ndarray, dx: float) -> list:
    """Indices of the cells (centres x, uniform spacing dx) whose open interval
    contains a jump of the data, found from the few jump positions."""
    if x.size == 0:
        return []
    cand = list(data.breaks)
    if data.period is not None:
        a, b0 = data.period
        L = b0 - a
        base = list(data.breaks) + ([a] if data.wrap_jump else [])
        cand = [b + sh for b in base for sh in (-L, 0.0, L)]
    out = set()
    x0 = x[0] - 0.5 * dx
    for b in cand:
        j = int(np.floor((b - x0) / dx))
        for jj in (j - 1, j, j + 1):
            if 0 <= jj < x.size and x[jj] - 0.5 * dx < b < x[jj] + 0.5 * dx:
                out.add(jj)
    return sorted(out)


def draw_state(rng: np.random.Generator):
    """(rho, u, p) with rho ~ U(0.1, 1), u ~ U(-1, 1), p ~ U(0.1, 1)."""
    return rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0)


def euler_riemann(seed: int, P: int, N: int, x_left: float = 0.0, x_right: float = 1.0,
                  x_jump: float = 0.5, gamma: float = 1.4, bc: str = "transmissive", parity: int = 0):
    """Seeded left/right states with a jump at x_jump and the density sine
    rho = rho_side*(1 + 0.2 sin 5x)."""
    rng = np.random.default_rng(seed)
    l, r = draw_state(rng), draw_state(rng)
    data = EulerPiecewise(np.array([x_jump]), np.array([l[0], r[0]]), np.array([l[1], r[1]]),
                          np.array([l[2], r[2]]), gamma=gamma,
                          period=(x_left, x_right) if bc == "periodic" else None)
    x = centers(x_left, x_right, N, n_cells(N, bc, parity), parity)
    return euler_taylor(data, x, (x_right - x_left) / N, P), data


def euler_multi_jump(seed: int, P: int, N: int, n_jumps: int = 8, x_left: float = 0.0,
                     x_right: float = 1.0, gamma: float = 1.4, bc: str = "periodic", parity: int = 0):
    """n_jumps sorted jump positions ~ U(0.05, 0.95), n_jumps+1 seeded states, density sine."""
    rng = np.random.default_rng(seed)
    breaks = np.sort(rng.uniform(0.05, 0.95, n_jumps))
    st = np.array([draw_state(rng) for _ in range(n_jumps + 1)])
    data = EulerPiecewise(x_left + (x_right - x_left) * breaks, st[:, 0], st[:, 1], st[:, 2], gamma=gamma,
                          period=(x_left, x_right) if bc == "periodic" else None)
    x = centers(x_left, x_right, N, n_cells(N, bc, parity), parity)
    return euler_taylor(data, x, (x_right - x_left) / N, P), data


def euler_uniform(N: int, P: int, rho: float, u: float, p: float, gamma: float = 1.4,
                  bc: str = "periodic", parity: int = 0) -> np.ndarray:
    n = n_cells(N, bc, parity)
    q = np.zeros((3, P + 1, n), dtype=np.float64)
    q[0, 0] = rho
    q[1, 0] = rho * u
    q[2, 0] = p / (gamma - 1.0) + 0.5 * rho * u * u
    return q


def euler_entropy_wave(P: int, N: int, x_left: float = 0.0, x_right: float = 2.0, amp: float = 0.2,
                       u: float = 1.0, p: float = 1.0, gamma: float = 1.4):
    """rho = 1 + amp sin(pi x), constant u and p, periodic on [0, 2]: the exact
    solution is the shifted density profile."""
    data = EulerPiecewise(np.array([]), np.array([1.0]), np.array([u]), np.array([p]), gamma=gamma,
                          sine_amp=amp, sine_w=np.pi, period=(x_left, x_right), wrap_jump=False)
    x = centers(x_left, x_right, N, N, 0)
    return euler_taylor(data, x, (x_right - x_left) / N, P), data


# ---------------------------------------------------------------------------
# Batched workload: independent Euler instances of uneven size and degree.
# ---------------------------------------------------------------------------
@dataclass
class BatchSpec:
    N: np.ndarray      # mesh intervals per instance
    P: np.ndarray      # degree per instance
    seeds: np.ndarray  # per-instance data seeds


def batch_spec(B: int, seed: int, n_lo: int = 256, n_hi: int = 65536, degrees=(1, 2, 3)) -> BatchSpec:
    """N_b = round(exp(U(ln n_lo, ln n_hi))), P_b uniform over degrees."""
    rng = np.random.default_rng(seed)
    N = np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), B))).astype(np.int64)
    P = rng.choice(np.asarray(degrees), B).astype(np.int32)
    seeds = rng.integers(0, 2 ** 31 - 1, B)
    return BatchSpec(N, P, seeds)


def batch_instance(spec: BatchSpec, b: int, gamma: float = 1.4):
    """Riemann problem with density sine on [0, 1], transmissive, for instance b."""
    return euler_riemann(int(spec.seeds[b]), int(spec.P[b]), int(spec.N[b]), gamma=gamma)[0]


# ---------------------------------------------------------------------------
# The 1D experiments of Section 5 (problem data only)
# ---------------------------------------------------------------------------
def sod(P: int, N: int, parity: int = 0):
    """Sod's shock tube (Section 5.2): [0, 2], (rho, u, p) = (1, 0, 1) for
    x < 1 and (0.125, 0, 0.1) otherwise, transmissive boundaries."""
    data = EulerPiecewise(np.array([1.0]), np.array([1.0, 0.125]), np.array([0.0, 0.0]), np.array([1.0, 0.1]),
                          sine_amp=0.0)
    x = centers(0.0, 2.0, N, n_cells(N, "transmissive", parity), parity)
    return euler_taylor(data, x, 2.0 / N, P), data


def shu_osher_tt(P: int, N: int, parity: int = 0):
    """Titarev and Toro's modified Shu-Osher problem (Section 5.2): [-5, 5],
    (1.515695, 0.523346, 1.805) for x < -4.5, else (1 + 0.1 sin(20 pi x), 0, 1),
    transmissive boundaries."""
    data = EulerPiecewise(np.array([-4.5]), np.array([1.515695, 1.0]), np.array([0.523346, 0.0]),
                          np.array([1.805, 1.0]), sine_amp=0.1, sine_w=20.0 * np.pi,
                          piece_sine=np.array([0.0, 1.0]))
    x = centers(-5.0, 5.0, N, n_cells(N, "transmissive", parity), parity)
    return euler_taylor(data, x, 10.0 / N, P), data


def jiang_shu_u0(x: np.ndarray) -> np.ndarray:
    """Jiang and Shu's composite profile on [-1, 1] (Section 5.1): Gaussians,
    a square wave, a sharp triangle and a half ellipse, zero elsewhere."""
    x = np.asarray(x, dtype=np.float64)
    a, z, dl, al = 0.5, -0.7, 0.005, 10.0
    be = np.log(2.0) / (36.0 * dl * dl)
    G = lambda zz: np.exp(-be * (x - zz) ** 2)
    F = lambda aa: np.sqrt(np.maximum(1.0 - al * al * (x - aa) ** 2, 0.0))
    u = np.zeros_like(x)
    m = (x >= -0.8) & (x <= -0.6)
    u = np.where(m, (G(z - dl) + 4.0 * G(z) + G(z + dl)) / 6.0, u)
    u = np.where((x >= -0.4) & (x <= -0.2), 1.0, u)
    u = np.where((x >= 0.0) & (x <= 0.2), 1.0 - 10.0 * np.abs(x - 0.1), u)
    u = np.where((x >= 0.4) & (x <= 0.6), (F(a - dl) + 4.0 * F(a) + F(a + dl)) / 6.0, u)
    return u


# points where the composite profile jumps or loses smoothness
JIANG_SHU_BREAKS = np.array([-0.8, -0.6, -0.4, -0.2, 0.0, 0.1, 0.2, 0.4, 0.405, 0.595, 0.6])


def projected_scalar(u0, breaks: np.ndarray, x: np.ndarray, dx: float, P: int) -> np.ndarray:
    """Degree-P L2 projection of u0 onto each cell (Gauss-Legendre quadrature,
    split at the given break points), returned as the point value and scaled
    derivatives at the cell centre -- the state convention of this module.
    Used for data that is not smooth enough for Taylor expansion."""
    n = x.size
    s_of = np.polynomial.legendre
    coef = np.zeros((P + 1, n))
    xa, xb = x - 0.5 * dx, x + 0.5 * dx

    def accumulate(j, lo, hi):
        mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
        xs = mid[:, None] + half[:, None] * _GL_X[None, :]
        sv = 2.0 * (xs - x[j][:, None]) / dx               # Legendre variable on [-1, 1]
        uv = u0(xs)
        wv = half[:, None] * _GL_W[None, :] / dx            # weights of the cell mean
        for m in range(P + 1):
            e = np.zeros(m + 1)
            e[m] = 1.0
            coef[m, j] += (2 * m + 1) * np.sum(wv * uv * s_of.legval(sv, e), axis=1)

    split = np.zeros(n, dtype=bool)
    for b in breaks:
        split |= (xa < b) & (b < xb)
    plain = np.nonzero(~split)[0]
    accumulate(plain, xa[plain], xb[plain])
    for j in np.nonzero(split)[0]:
        pts = [xa[j]] + sorted(b for b in breaks if xa[j] < b < xb[j]) + [xb[j]]
        for lo, hi in zip(pts[:-1], pts[1:]):
            accumulate(np.array([j]), np.array([lo]), np.array([hi]))
    q = np.empty((1, P + 1, n))
    for j in range(n):
        mono = s_of.leg2poly(coef[:, j])                    # coefficients of s^k, s = 2 xi
        for k in range(P + 1):
            ak = (mono[k] if k < mono.size else 0.0) * 2.0 ** k
            q[0, k, j] = ak * float(np.prod(np.arange(1, k + 1)))   # u_kx = k! a_k
    return q


def jiang_shu(P: int, N: int):
    """Projected Jiang-Shu composite on N periodic cells of [-1, 1]."""
    x = centers(-1.0, 1.0, N, N, 0)
    return projected_scalar(jiang_shu_u0, JIANG_SHU_BREAKS, x, 2.0 / N, P)


# ---------------------------------------------------------------------------
# 2D data (Section 3; Table 3's isentropic vortex).  States have shape
# (nc, ndof, Ny, Nx) with the DOFs u_{kx,ly} = dx^k dy^l d^{k+l}u0/dx^k dy^l
# at the cell centre in DOF order (k + l ascending, then l ascending).
# ---------------------------------------------------------------------------
def ndof2d(P: int) -> int:
    return (P + 1) * (P + 2) // 2


def dof2d(k: int, l: int) -> int:
    n = k + l
    return n * (n + 1) // 2 + l


def dof_pairs(P: int):
    """(k, l) in DOF order."""
    return [(n - l, l) for n in range(P + 1) for l in range(n + 1)]


def centers2d(x_left, x_right, y_left, y_right, Nx, Ny, parity, bc="periodic"):
    """Cell centres (X, Y) of the mesh of this parity (Section 3.1), per
    direction (`bc` a name or a pair (x, y) of names): periodic, N cells on
    both meshes, the staggered one shifted by half a cell; transmissive, the
    N+1 mesh points on parity 0 (edges included) and the N cells between them
    on parity 1.  Arrays of shape (rows, columns)."""
    bx, by = (bc, bc) if isinstance(bc, str) else bc
    x = centers(x_left, x_right, Nx, n_cells(Nx, bx, parity), parity)
    y = centers(y_left, y_right, Ny, n_cells(Ny, by, parity), parity)
    return np.meshgrid(x, y)


@dataclass
class Modes2D:
    """u0 = c0 + sum_m A_m sin(kx_m x + ky_m y + phi_m)."""
    c0: float
    amps: np.ndarray
    kx: np.ndarray
    ky: np.ndarray
    phases: np.ndarray

    def deriv(self, X, Y, k: int, l: int):
        out = np.full_like(X, self.c0 if k + l == 0 else 0.0, dtype=np.float64)
        for a, wx, wy, ph in zip(self.amps, self.kx, self.ky, self.phases):
            out = out + a * wx ** k * wy ** l * np.sin(wx * X + wy * Y + ph + (k + l) * np.pi / 2)
        return out

    def __call__(self, X, Y):
        return self.deriv(np.asarray(X, dtype=np.float64), np.asarray(Y, dtype=np.float64), 0, 0)


def taylor2d(fn: Modes2D, P: int, Nx: int, Ny: int, domain=(0.0, 2.0, 0.0, 2.0), parity: int = 0):
    x0, x1, y0, y1 = domain
    X, Y = centers2d(x0, x1, y0, y1, Nx, Ny, parity)
    dx, dy = (x1 - x0) / Nx, (y1 - y0) / Ny
    q = np.empty((1, ndof2d(P), Ny, Nx))
    for k, l in dof_pairs(P):
        q[0, dof2d(k, l)] = dx ** k * dy ** l * fn.deriv(X, Y, k, l)
    return q


def modes2d(seed: int, n_modes: int = 3, c0: float = 0.5, amp: float = 0.5, kmax: int = 3) -> Modes2D:
    """Seeded sum of sine modes periodic on [0, 2]^2: A ~ U(0, amp/n_modes),
    integer wavenumbers in [-kmax, kmax] (times pi), not both zero."""
    rng = np.random.default_rng(seed)
    kx, ky = [], []
    while len(kx) < n_modes:
        a, b = rng.integers(-kmax, kmax + 1, 2)
        if a or b:
            kx.append(a)
            ky.append(b)
    amps = rng.uniform(0.0, amp / n_modes, n_modes)
    phases = rng.uniform(0.0, 2 * np.pi, n_modes)
    return Modes2D(c0, amps, np.pi * np.array(kx, float), np.pi * np.array(ky, float), phases)


_VORTEX_CACHE: dict = {}


def _vortex_functions(P: int, gamma: float, psi: float):
    """Numerical functions d^{k+l}/dx^k dy^l of (rho, rho u, rho v, rho e) of
    the isentropic vortex (Section 5.3.1), from symbolic differentiation."""
    key = (P, gamma, psi)
    if key in _VORTEX_CACHE:
        return _VORTEX_CACHE[key]
    import sympy as sp
    x, y = sp.symbols("x y", real=True)
    g = sp.Rational(gamma).limit_denominator(1000) if isinstance(gamma, float) else gamma
    ps = sp.nsimplify(psi)
    e = sp.exp(sp.Rational(1, 2) * (1 - x * x - y * y))
    du, dv = ps / (2 * sp.pi) * e * (-y), ps / (2 * sp.pi) * e * x
    T = 1 - (g - 1) * ps ** 2 / (8 * g * sp.pi ** 2) * e ** 2
    rho = T ** (1 / (g - 1))
    p = rho * T
    u, v = 1 + du, 1 + dv
    U = [rho, rho * u, rho * v, p / (g - 1) + rho * (u * u + v * v) / 2]
    fns = {}
    for k, l in dof_pairs(P):
        fns[(k, l)] = [sp.lambdify((x, y), sp.diff(c, x, k, y, l) if k + l else c, "numpy") for c in U]
    _VORTEX_CACHE[key] = fns
    return fns


def vortex_state(X, Y, t: float = 0.0, gamma: float = 1.4, psi: float = 5.0, L: float = 10.0):
    """Conserved (rho, rho u, rho v, rho e) of the vortex moved by (t, t), the
    position wrapped into the periodic box [-L/2, L/2]^2 (the exact solution)."""
    fns = _vortex_functions(0, gamma, psi)[(0, 0)]
    xs = (X - t + L / 2) % L - L / 2
    ys = (Y - t + L / 2) % L - L / 2
    return np.stack([np.broadcast_to(f(xs, ys), X.shape) for f in fns])


def isentropic_vortex(P: int, N: int, parity: int = 0, gamma: float = 1.4, psi: float = 5.0):
    """Taylor data of the isentropic vortex on the periodic [-5, 5]^2 with
    N x N cells (Section 5.3.1): uniform rho = 1, p = 1, (u, v) = (1, 1) plus
    the isentropic perturbation of strength psi."""
    X, Y = centers2d(-5.0, 5.0, -5.0, 5.0, N, N, parity)
    h = 10.0 / N
    fns = _vortex_functions(P, gamma, psi)
    q = np.empty((4, ndof2d(P), N, N))
    for k, l in dof_pairs(P):
        for c in range(4):
            q[c, dof2d(k, l)] = h ** (k + l) * np.broadcast_to(fns[(k, l)][c](X, Y), X.shape)
    return q


# The two 2D Riemann problems of Section 5.3 (density, x- and y-velocity,
# pressure in the quadrants [-1,0]x[-1,0], [-1,0]x[0,1], [0,1]x[0,1],
# [0,1]x[-1,0]).
RIEMANN2D = {
    1: ((0.138, 1.206, 1.206, 0.029), (0.5323, 1.206, 0.0, 0.3), (1.5, 0.0, 0.0, 1.5), (0.5323, 0.0, 1.206, 0.3)),
    2: ((1.0, -0.75, 0.5, 1.0), (2.0, 0.75, 0.5, 1.0), (1.0, 0.75, -0.5, 1.0), (3.0, -0.75, -0.5, 1.0)),
}


def riemann2d(config: int, P: int, N: int, parity: int = 0, gamma: float = 1.4):
    """2D Riemann problem `config` on [-1, 1]^2 with N x N intervals,
    transmissive: every cell holds the exact mean of the conserved variables
    over the cell (area-weighted over the quadrants it overlaps) as its point
    value, derivatives zero (the piecewise-constant data have none)."""
    states = RIEMANN2D[config]
    h = 2.0 / N
    X, Y = centers2d(-1.0, 1.0, -1.0, 1.0, N, N, parity, "transmissive")

    def frac_neg(c):           # fraction of [c - h/2, c + h/2] below 0
        return np.clip((0.0 - (c - 0.5 * h)) / h, 0.0, 1.0)

    fx, fy = frac_neg(X), frac_neg(Y)
    weights = (fx * fy, fx * (1 - fy), (1 - fx) * (1 - fy), (1 - fx) * fy)
    q = np.zeros((4, ndof2d(P)) + X.shape)
    for w, (rho, u, v, p) in zip(weights, states):
        cons = (rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v))
        for c in range(4):
            q[c, 0] += w * cons[c]
    return q


def richtmyer_meshkov(P: int, Nx: int, Ny: int, parity: int = 0, gamma: float = 1.4, mach: float = 2.0,
                      quad: int = 8):
    """Single-mode Richtmyer-Meshkov set-up of Section 5.3 on [-0.5, 0.5] x
    [0, 5], periodic in x, transmissive in y: light gas (0.1, 0, 0, 1/gamma)
    above y = 1 - 0.3 cos(2 pi x), heavy gas (1, 0, 0, 1/gamma) below it down
    to y = 0.6, and below that the post-shock state of a Mach `mach` shock
    moving up into the heavy gas (normal-shock relations, as the paper writes
    them).  Each cell holds the mean of the conserved variables over the cell
    (a quad x quad Gauss-Legendre rule on each cell; the interfaces make the
    data piecewise constant) as its point value, derivatives zero."""
    r2, p2 = 1.0, 1.0 / gamma
    a2 = np.sqrt(gamma * p2 / r2)
    m2 = mach * mach
    rs = r2 * 0.5 * (gamma + 1.0) * m2 / (1.0 + 0.5 * (gamma - 1.0) * m2)
    vs = a2 * 2.0 * (m2 - 1.0) / ((gamma + 1.0) * mach)
    ps = p2 * (2.0 * gamma * m2 - gamma + 1.0) / (gamma + 1.0)
    states = {1: (0.1, 0.0, 0.0, 1.0 / gamma), 2: (r2, 0.0, 0.0, p2), 3: (rs, 0.0, vs, ps)}
    hx, hy = 1.0 / Nx, 5.0 / Ny
    X, Y = centers2d(-0.5, 0.5, 0.0, 5.0, Nx, Ny, parity, ("periodic", "transmissive"))
    g, w = np.polynomial.legendre.leggauss(quad)
    q = np.zeros((4, ndof2d(P)) + X.shape)
    for gi, wi in zip(g, w):
        for gj, wj in zip(g, w):
            xs, ys = X + 0.5 * hx * gi, Y + 0.5 * hy * gj
            region = np.where(ys >= 1.0 - 0.3 * np.cos(2 * np.pi * xs), 1, np.where(ys >= 0.6, 2, 3))
            for k, (rho, u, v, p) in states.items():
                cons = (rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v))
                m = (region == k) * (0.25 * wi * wj)
                for c in range(4):
                    q[c, 0] += m * cons[c]
    return q

