"""Closed-form and textbook solutions that pin the oracle independently of it.

* Burgers before the shock: method of characteristics, u = u0(xi) with
  x = xi + u0(xi) t.
* Burgers after the shock: Hopf-Lax / Lax-Oleinik formula for the convex flux
  u^2/2, u = (x - y*)/t with y* = argmin_y [(x-y)^2/(2t) + U0(y)].
* Euler Riemann problem: exact solution by the standard pressure-function
  Newton iteration for the star pressure and wave sampling (textbook method of
  Toro, Riemann Solvers and Numerical Methods for Fluid Dynamics, ch. 4).
* Euler isentropic flow with gamma = 3: the Riemann invariants w = u +- c move
  with speed w, so each obeys Burgers' equation and the method of
  characteristics gives an exact smooth solution of the full system.
"""
from __future__ import annotations

import numpy as np
import sympy as sp


# ---------------------------------------------------------------------------
# Burgers
# ---------------------------------------------------------------------------
def sine_sum_fn(fn):
    """Vectorised u0 and u0' of an inputs.SineSum."""
    def u0(x):
        return fn.deriv(np.asarray(x, dtype=np.float64), 0)

    def du0(x):
        return fn.deriv(np.asarray(x, dtype=np.float64), 1)
    return u0, du0


def breaking_time(fn, x_left=0.0, x_right=2.0) -> float:
    """t_b = 1 / max(-u0'), dense sampling refined by Newton on u0''."""
    x = np.linspace(x_left, x_right, 200001)
    d1 = fn.deriv(x, 1)
    i = int(np.argmin(d1))
    xs = x[i]
    for _ in range(50):
        g, h = fn.deriv(np.array([xs]), 2)[0], fn.deriv(np.array([xs]), 3)[0]
        if h == 0:
            break
        step = g / h
        xs -= step
        if abs(step) < 1e-15:
            break
    m = -fn.deriv(np.array([xs]), 1)[0]
    return 1.0 / m


def burgers_moc(fn, x: np.ndarray, t: float) -> np.ndarray:
    """Solve xi + u0(xi) t = x by Newton (valid before the breaking time)."""
    u0, du0 = sine_sum_fn(fn)
    xi = np.array(x, dtype=np.float64) - u0(x) * t
    for _ in range(100):
        g = xi + u0(xi) * t - x
        dg = 1.0 + du0(xi) * t
        step = g / dg
        xi = xi - step
        if np.max(np.abs(step)) < 1e-15:
            break
    return u0(xi)


def burgers_hopf_lax(fn, x: np.ndarray, t: float, n_grid: int = 4001) -> np.ndarray:
    """u(x,t) = (x - y*)/t, y* minimising (x-y)^2/(2t) + U0(y), U0' = u0."""
    c0, amps, ws, phs = fn.c0, fn.amps, fn.freqs, fn.phases

    def U0(y):
        s = c0 * y
        for a, w, ph in zip(amps, ws, phs):
            s = s + a / w * (np.cos(ph) - np.cos(w * y + ph))
        return s

    umax = c0 + np.sum(np.abs(amps))
    umin = c0 - np.sum(np.abs(amps))
    out = np.empty_like(x, dtype=np.float64)
    for i, xi in enumerate(x):
        lo, hi = xi - umax * t - 1e-3, xi - umin * t + 1e-3
        y = np.linspace(lo, hi, n_grid)
        obj = (xi - y) ** 2 / (2 * t) + U0(y)
        j = int(np.argmin(obj))
        a_, b_ = y[max(j - 1, 0)], y[min(j + 1, n_grid - 1)]
        # golden-section refinement on the bracket
        gr = (np.sqrt(5) - 1) / 2
        c_, d_ = b_ - gr * (b_ - a_), a_ + gr * (b_ - a_)
        for _ in range(80):
            fc = (xi - c_) ** 2 / (2 * t) + U0(c_)
            fd = (xi - d_) ** 2 / (2 * t) + U0(d_)
            if fc < fd:
                b_ = d_
            else:
                a_ = c_
            c_, d_ = b_ - gr * (b_ - a_), a_ + gr * (b_ - a_)
        ys = 0.5 * (a_ + b_)
        out[i] = (xi - ys) / t
    return out


# ---------------------------------------------------------------------------
# Euler exact Riemann solver (perfect gas)
# ---------------------------------------------------------------------------
def _f_k(p, rho_k, p_k, c_k, g):
    if p > p_k:
        A = 2.0 / ((g + 1) * rho_k)
        B = (g - 1) / (g + 1) * p_k
        q = np.sqrt(A / (p + B))
        return (p - p_k) * q, q * (1 - 0.5 * (p - p_k) / (B + p))
    r = p / p_k
    return 2 * c_k / (g - 1) * (r ** ((g - 1) / (2 * g)) - 1), 1.0 / (rho_k * c_k) * r ** (-(g + 1) / (2 * g))


def riemann_star(WL, WR, g=1.4):
    rl, ul, pl = WL
    rr, ur, pr = WR
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    p = max(1e-10, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dl = _f_k(p, rl, pl, cl, g)
        fr, dr = _f_k(p, rr, pr, cr, g)
        pn = p - (fl + fr + ur - ul) / (dl + dr)
        pn = max(pn, 1e-12)
        if abs(pn - p) / (0.5 * (pn + p)) < 1e-14:
            p = pn
            break
        p = pn
    fl, _ = _f_k(p, rl, pl, cl, g)
    fr, _ = _f_k(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(WL, WR, s: np.ndarray, g=1.4) -> np.ndarray:
    """Primitive (rho, u, p) at similarity coordinates s = (x - x0)/t."""
    rl, ul, pl = WL
    rr, ur, pr = WR
    cl, cr = np.sqrt(g * pl / rl), np.sqrt(g * pr / rr)
    ps, us = riemann_star(WL, WR, g)
    out = np.empty((3, s.size))
    for i, si in enumerate(s):
        if si <= us:
            if ps > pl:  # left shock
                sl = ul - cl * np.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                if si <= sl:
                    w = (rl, ul, pl)
                else:
                    rs = rl * (ps / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pl + 1)
                    w = (rs, us, ps)
            else:  # left rarefaction
                shl = ul - cl
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                stl = us - csl
                if si <= shl:
                    w = (rl, ul, pl)
                elif si >= stl:
                    w = (rl * (ps / pl) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + si)
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - si))
                    rho = rl * (c / cl) ** (2 / (g - 1))
                    w = (rho, u, pl * (c / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:  # right shock
                sr = ur + cr * np.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                if si >= sr:
                    w = (rr, ur, pr)
                else:
                    rs = rr * (ps / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / pr + 1)
                    w = (rs, us, ps)
            else:  # right rarefaction
                shr = ur + cr
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                str_ = us + csr
                if si >= shr:
                    w = (rr, ur, pr)
                elif si <= str_:
                    w = (rr * (ps / pr) ** (1 / g), us, ps)
                else:
                    u = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + si)
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - si))
                    rho = rr * (c / cr) ** (2 / (g - 1))
                    w = (rho, u, pr * (c / cr) ** (2 * g / (g - 1)))
        out[:, i] = w
    return out


# ---------------------------------------------------------------------------
# Euler, gamma = 3, isentropic simple waves: two decoupled Burgers problems
# ---------------------------------------------------------------------------
_xs = sp.Symbol("x", real=True)


class Gamma3Flow:
    """rho = c (p = rho^3/3, so c^2 = 3p/rho = rho^2), u0 and c0 given as sympy
    expressions of x; w+- = u +- c are constant along dx/dt = w+-."""

    def __init__(self, u0_expr, c0_expr):
        self.u0 = u0_expr
        self.c0 = c0_expr
        rho = c0_expr
        mom = rho * u0_expr
        ene = rho ** 3 / 6 + rho * u0_expr ** 2 / 2   # p/(gamma-1) + rho u^2/2 with p = rho^3/3
        self.U = [rho, mom, ene]
        self._wp = sp.lambdify(_xs, u0_expr + c0_expr, "numpy")
        self._wm = sp.lambdify(_xs, u0_expr - c0_expr, "numpy")
        self._dwp = sp.lambdify(_xs, sp.diff(u0_expr + c0_expr, _xs), "numpy")
        self._dwm = sp.lambdify(_xs, sp.diff(u0_expr - c0_expr, _xs), "numpy")
        self._derivs = {}

    def taylor_state(self, x: np.ndarray, dx: float, P: int) -> np.ndarray:
        q = np.empty((3, P + 1, x.size))
        for c in range(3):
            e = self.U[c]
            for k in range(P + 1):
                key = (c, k)
                if key not in self._derivs:
                    self._derivs[key] = sp.lambdify(_xs, sp.diff(e, _xs, k), "numpy")
                q[c, k] = dx ** k * np.broadcast_to(self._derivs[key](x), x.shape)
        return q

    @staticmethod
    def _moc(w, dw, x, t):
        xi = np.array(x, dtype=np.float64) - w(x) * t
        for _ in range(100):
            g = xi + w(xi) * t - x
            step = g / (1.0 + dw(xi) * t)
            xi = xi - step
            if np.max(np.abs(step)) < 1e-15:
                break
        return w(xi)

    def exact_conserved(self, x: np.ndarray, t: float) -> np.ndarray:
        wp = self._moc(self._wp, self._dwp, x, t)
        wm = self._moc(self._wm, self._dwm, x, t)
        u = 0.5 * (wp + wm)
        c = 0.5 * (wp - wm)
        rho = c
        return np.stack([rho, rho * u, rho ** 3 / 6 + 0.5 * rho * u * u])


def euler_jacobian(U, g=1.4) -> np.ndarray:
    """Analytic flux Jacobian dF/dU of the 1D Euler equations."""
    rho, mom, E = U
    u = mom / rho
    p = (g - 1) * (E - 0.5 * rho * u * u)
    H = (E + p) / rho
    return np.array([
        [0.0, 1.0, 0.0],
        [0.5 * (g - 3) * u * u, (3 - g) * u, g - 1],
        [u * (0.5 * (g - 1) * u * u - H), H - (g - 1) * u * u, g * u],
    ])


def euler_flux(U, g=1.4) -> np.ndarray:
    rho, mom, E = U
    u = mom / rho
    p = (g - 1) * (E - 0.5 * rho * u * u)
    return np.array([mom, mom * u + p, (E + p) * u])
