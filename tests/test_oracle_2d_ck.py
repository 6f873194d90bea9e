"""Pin of the 2D oracle's Cauchy-Kovalewski expansion (Section 3.1; the
system form of Section 4) against exact rational arithmetic.

For polynomial initial data, the space-time Taylor polynomial of the
solution truncated at total degree P is built here from the PDE alone: the
state as an exact-rational polynomial in (x, y, t), the fluxes evaluated on
it (the Euler velocities through the Neumann series of 1/rho), and the
coefficients of t^(m+1) from -(dF/dx + dG/dy) at t^m, level by level.  The
oracle's per-old-cell outputs that the expansion feeds must match it:

* the vertex values (Eq. SubEq:2DUij): the scaled derivatives at the cell
  centre expanded in time over the half-step, for k + l < P;
* the half-edge flux averages: F averaged over the half-step and over the
  upper (lower) half of the vertical line through the centre, G over the
  right (left) half of the horizontal one, by exact integration.

The test shares no arithmetic with the oracle: polynomial products and
derivatives come from sympy, the quotient from a geometric series, the
integrals from sympy's integrate.
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle

x, y, t = sp.symbols("x y t")
GAMMA = sp.Rational(7, 5)


def _poly(expr):
    return sp.Poly(expr, x, y, t, domain="QQ")


def _trunc(p, deg):
    return _poly(sum(c * x ** a * y ** b * t ** e for (a, b, e), c in p.terms() if a + b + e <= deg))


def space_time_solution(eq, U0, P):
    """Taylor polynomial of the solution in (x, y, t), total degree <= P, from
    initial polynomials U0 (one per component); returns (U, F, G)."""
    def mul(a, b):
        return _trunc(a * b, P)

    def inverse(r):
        r0 = r.coeff_monomial(1)
        d = (r - r0) * (-1 / r0)
        s = term = _poly(1)
        for _ in range(P):
            term = mul(term, d)
            s = s + term
        return s * (1 / r0)

    def fluxes(U):
        if eq == "burgers":
            h = mul(U[0], U[0]) * sp.Rational(1, 2)
            return [h], [h]
        r, m, n, E = U
        ir = inverse(r)
        u, v = mul(m, ir), mul(n, ir)
        p = (E - (mul(m, u) + mul(n, v)) * sp.Rational(1, 2)) * (GAMMA - 1)
        W = E + p
        return [m, mul(m, u) + p, mul(m, v), mul(W, u)], [n, mul(n, u), mul(n, v) + p, mul(W, v)]

    U = [_poly(u) for u in U0]
    for m in range(P):
        F, G = fluxes(U)
        nxt = []
        for c in range(len(U)):
            Fm = _poly(sum(co * x ** a * y ** b for (a, b, e), co in F[c].terms() if e == m)) * math.factorial(m)
            Gm = _poly(sum(co * x ** a * y ** b for (a, b, e), co in G[c].terms() if e == m)) * math.factorial(m)
            dU = -(Fm.diff(x) + Gm.diff(y))          # d^(m+1)U/dt^(m+1) at t = 0
            nxt.append(_trunc(U[c] + dU * _poly(t ** (m + 1)) * sp.Rational(1, math.factorial(m + 1)), P))
        U = nxt
    F, G = fluxes(U)
    return U, F, G


def random_data(eq, P, seed):
    rng = np.random.default_rng(seed)

    def rpoly(base, amp):
        s = sp.Rational(base)
        for n in range(1, P + 1):
            for l in range(n + 1):
                s += sp.Rational(int(rng.integers(-100, 101)), 1000) * amp * x ** (n - l) * y ** l
        return s

    if eq == "burgers":
        return [rpoly(sp.Rational(1, 2), 1)]
    return [rpoly(1, 1), rpoly(sp.Rational(1, 3), 1), rpoly(sp.Rational(-1, 4), 1), rpoly(3, 2)]


@pytest.mark.parametrize("eq,P", [("euler", 1), ("euler", 2), ("euler", 3), ("burgers", 3)])
def test_ck_expansion_matches_exact_rational_solution(eq, P):
    dx, dy, dt = 0.125, 0.0625, 0.03125
    U0 = random_data(eq, P, seed=10 + P)
    U, F, G = space_time_solution(eq, U0, P)
    nc = len(U0)
    pb = oracle.Problem2D(eq, P, 8, 8, limiter=False, x_right=8 * dx, y_right=8 * dy)
    # the oracle's cell state: point value and scaled derivatives dx^k dy^l d^(k+l)u at the centre
    q = np.zeros((nc, oracle.ndof2d(P)))
    U0p = [_poly(u) for u in U0]
    for c in range(nc):
        for n in range(P + 1):
            for l in range(n + 1):
                k = n - l
                q[c, oracle.dof2d(k, l)] = float(U0p[c].coeff_monomial(x ** k * y ** l)) * \
                    math.factorial(k) * math.factorial(l) * dx ** k * dy ** l
    o = oracle.old_cell2d(pb, q, dt)
    for c in range(nc):
        # vertex values: sum over m of dt^m/m! d^m/dt^m of the scaled derivative
        for n in range(P):
            for l in range(n + 1):
                k = n - l
                want = sum(float(U[c].coeff_monomial(x ** k * y ** l * t ** m)) * dt ** m
                           for m in range(P - n + 1)) * math.factorial(k) * math.factorial(l) * dx ** k * dy ** l
                got = o["V"][c][(k, l)]
                assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (c, k, l, got, want)
        # half-edge flux averages over the half-step
        Fc, Gc = F[c].as_expr(), G[c].as_expr()
        T = sp.Rational(dt).limit_denominator(10 ** 9)
        HX, HY = sp.Rational(dx) / 2, sp.Rational(dy) / 2
        fU = sp.integrate(Fc.subs(x, 0), (y, 0, HY), (t, 0, T)) / (HY * T)
        fD = sp.integrate(Fc.subs(x, 0), (y, -HY, 0), (t, 0, T)) / (HY * T)
        gR = sp.integrate(Gc.subs(y, 0), (x, 0, HX), (t, 0, T)) / (HX * T)
        gL = sp.integrate(Gc.subs(y, 0), (x, -HX, 0), (t, 0, T)) / (HX * T)
        for name, want in (("fU", fU), ("fD", fD), ("gR", gR), ("gL", gL)):
            want = float(want)
            got = o[name][c]
            assert abs(got - want) <= 1e-13 * max(1.0, abs(want)), (c, name, got, want)
