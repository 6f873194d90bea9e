"""Pin of the 1D oracle's Cauchy-Kovalewski expansion (Eq.
1DCauchy_Kovalewski; the Euler system of Section 4) at every level against
exact rational arithmetic.

In the cell's scaled variables (xi = (x - x_i)/dx, tau = (t - t^n)/dt) the
PDE reads u_tau + lam f(u)_xi = 0 with lam = dt/dx, and the oracle's triangle
T[c][k][m] is the coefficient of xi^k tau^m of the solution's Taylor
polynomial of total degree P.  That polynomial is built here from the PDE
alone, level by level: the state as an exact-rational polynomial in (xi, tau),
the flux evaluated on it (the Euler velocity through the geometric series of
1/rho), and the coefficients of tau^(m+1) from -lam d/dxi of the flux's tau^m
coefficients.  No arithmetic is shared with the oracle.
"""
import math

import numpy as np
import pytest
import sympy as sp

import oracle

xi, tau = sp.symbols("xi tau")
GAMMA = sp.Rational(7, 5)


def _poly(expr):
    return sp.Poly(expr, xi, tau, domain="QQ")


def exact_triangle(eq, U0, P, lam):
    def trunc(p):
        return _poly(sum(c * xi ** a * tau ** e for (a, e), c in p.terms() if a + e <= P))

    def mul(a, b):
        return trunc(a * b)

    def inverse(r):
        r0 = r.coeff_monomial(1)
        d = (r - r0) * (-1 / r0)
        s = term = _poly(1)
        for _ in range(P):
            term = mul(term, d)
            s = s + term
        return s * (1 / r0)

    def flux(U):
        if eq == "burgers":
            return [mul(U[0], U[0]) * sp.Rational(1, 2)]
        r, m, E = U
        u = mul(m, inverse(r))
        p = (E - mul(m, u) * sp.Rational(1, 2)) * (GAMMA - 1)
        return [m, mul(m, u) + p, mul(E + p, u)]

    U = [_poly(u) for u in U0]
    for m in range(P):
        F = flux(U)
        nxt = []
        for c in range(len(U)):
            Fm = _poly(sum(co * xi ** a for (a, e), co in F[c].terms() if e == m)) * math.factorial(m)
            dU = -lam * Fm.diff(xi)                  # d^(m+1)u/dtau^(m+1) at tau = 0
            nxt.append(trunc(U[c] + dU * _poly(tau ** (m + 1)) * sp.Rational(1, math.factorial(m + 1))))
        U = nxt
    return U


@pytest.mark.parametrize("eq,P", [("euler", 2), ("euler", 3), ("euler", 4), ("burgers", 4)])
def test_ck_triangle_matches_exact_rational_solution(eq, P):
    rng = np.random.default_rng(40 + P)
    lam = sp.Rational(3, 16)
    base = [sp.Rational(1, 2)] if eq == "burgers" else [sp.Rational(1), sp.Rational(-1, 3), sp.Rational(5, 2)]
    U0, q = [], np.zeros((len(base), P + 1))
    for c, b in enumerate(base):
        coef = [b] + [sp.Rational(int(rng.integers(-100, 101)), 500) for _ in range(P)]
        U0.append(sum(coef[k] * xi ** k for k in range(P + 1)))
        # the oracle's state: point value and scaled derivatives u_{kx} = k! (coefficient of xi^k)
        q[c] = [float(coef[k]) * math.factorial(k) for k in range(P + 1)]
    pb = oracle.Problem(eq, P, 8)
    T = oracle.ck_triangle(pb, q, float(lam))
    U = exact_triangle(eq, U0, P, lam)
    for c in range(len(base)):
        for k in range(P + 1):
            for m in range(P + 1 - k):
                want = float(U[c].coeff_monomial(xi ** k * tau ** m))
                assert abs(T[c, k, m] - want) <= 1e-14 * max(1.0, abs(want)), (c, k, m, T[c, k, m], want)
