"""Pins of the 2D oracle (Section 3, Appendix B; the 2D Euler step of
Section 4, unlimited and limited), each fixed by something other than the oracle's own formulas:

* Table 3 (Section 5.3.1): density errors of LCCS-2/3/4 and of WCCS-2/3/4
  (limiter on the characteristic fields of the rotated decomposition of
  Section 4) on the isentropic vortex at t = 2, mesh sizes 1/5 and 1/10
  (printed to 3 digits).
* Exactness for polynomial data of degree <= P under linear advection, on
  every cell outside the periodic seam's domain of dependence.
* P = 0 is the 2D staggered Lax-Friedrichs scheme.
* Data independent of y (or of x) reproduces the 1D oracle: advection,
  Burgers and Euler, limiter off.
* Symmetry under x <-> y for data and fluxes symmetric in x and y, limiter on.
* Conservation of the cell-average sum to round-off (periodic), limiter on.
* Linear data is kept by the limiter (all five candidates coincide).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2104_04347_amd import inputs

CFL = {1: 0.4, 2: 0.3, 3: 0.25}
DOF = inputs.dof2d


def averages2d(P, q):
    """Cell averages of a 2D state (Eq. SubEq:2DCellAVG, written out here from
    the integral of the cell polynomial over the unit square)."""
    out = q[:, 0].copy()
    for k, l in inputs.dof_pairs(P):
        if (k, l) != (0, 0) and k % 2 == 0 and l % 2 == 0:
            w = 1.0 / (math.factorial(k + 1) * 2 ** k * math.factorial(l + 1) * 2 ** l)
            out = out + w * q[:, DOF(k, l)]
    return out


# ---------------------------------------------------------------------------
# Table 3
# ---------------------------------------------------------------------------
TABLE3_LCCS = {  # (P, N): (L1, Linf) of density, mesh size 10/N
    (1, 50): (6.51e-4, 1.33e-2), (2, 50): (3.71e-4, 5.73e-3), (3, 50): (5.54e-5, 7.25e-4),
    (1, 100): (1.15e-4, 2.42e-3), (2, 100): (5.13e-5, 7.91e-4), (3, 100): (2.13e-6, 3.41e-5),
}


TABLE3_WCCS = {  # limited, rotated characteristic decomposition (Section 4)
    (1, 50): (1.69e-3, 3.77e-2), (2, 50): (4.09e-4, 6.91e-3), (3, 50): (5.70e-5, 7.25e-4),
    (1, 100): (2.75e-4, 9.63e-3), (2, 100): (5.26e-5, 9.30e-4), (3, 100): (2.16e-6, 3.41e-5),
}


def vortex_errors(P, N, limiter=False):
    q0 = inputs.isentropic_vortex(P, N)
    pb = oracle.Problem2D("euler", P, N, N, limiter=limiter, x_left=-5, x_right=5, y_left=-5, y_right=5)
    r = oracle.run2d(pb, q0, t_end=2.0, cfl=CFL[P])
    assert r.flags == 0 and r.t == 2.0
    X, Y = inputs.centers2d(-5, 5, -5, 5, N, N, r.parity)
    err = np.abs(r.q[0, 0] - inputs.vortex_state(X, Y, 2.0)[0])
    return err.mean(), err.max()


@pytest.mark.parametrize("P", [1, 2, 3])
def test_table3_lccs_mesh_1_5(P):
    l1, linf = vortex_errors(P, 50)
    p1, pinf = TABLE3_LCCS[(P, 50)]
    assert abs(l1 / p1 - 1) < 0.04, (l1, p1)
    assert abs(linf / pinf - 1) < 0.04, (linf, pinf)


@pytest.mark.slow
@pytest.mark.parametrize("P", [1, 2, 3])
def test_table3_lccs_mesh_1_10(P):
    l1, linf = vortex_errors(P, 100)
    p1, pinf = TABLE3_LCCS[(P, 100)]
    assert abs(l1 / p1 - 1) < 0.04, (l1, p1)
    assert abs(linf / pinf - 1) < 0.04, (linf, pinf)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_table3_wccs_mesh_1_5(P):
    l1, linf = vortex_errors(P, 50, limiter=True)
    p1, pinf = TABLE3_WCCS[(P, 50)]
    assert abs(l1 / p1 - 1) < 0.04, (l1, p1)
    assert abs(linf / pinf - 1) < 0.04, (linf, pinf)


@pytest.mark.slow
@pytest.mark.parametrize("P", [1, 2])
def test_table3_wccs_mesh_1_10(P):
    l1, linf = vortex_errors(P, 100, limiter=True)
    p1, pinf = TABLE3_WCCS[(P, 100)]
    assert abs(l1 / p1 - 1) < 0.04, (l1, p1)
    assert abs(linf / pinf - 1) < 0.04, (linf, pinf)


# ---------------------------------------------------------------------------
# Exactness, P = 0, reduction to 1D
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("P", [1, 2, 3])
def test_polynomial_exactness_advection(P):
    N, steps, a, b = 32, 6, 0.7, -0.4
    rng = np.random.default_rng(10 + P)
    pairs = inputs.dof_pairs(P)
    coef = {kl: rng.uniform(-1, 1) for kl in pairs}       # u0 = sum c_kl x^k y^l

    def deriv(X, Y, k, l):
        out = np.zeros_like(X)
        for (i, j), c in coef.items():
            if i >= k and j >= l:
                f = np.prod(np.arange(i - k + 1, i + 1)) * np.prod(np.arange(j - l + 1, j + 1))
                out = out + c * f * X ** (i - k) * Y ** (j - l)
        return out

    pb = oracle.Problem2D("advection", P, N, N, a=a, b=b)
    dx = dy = pb.dx
    X, Y = inputs.centers2d(0, 1, 0, 1, N, N, 0)
    q = np.stack([dx ** k * dy ** l * deriv(X, Y, k, l) for k, l in pairs])[None]
    dt = 0.2 * dx
    r = oracle.run2d(pb, q, dt_fixed=dt, max_half_steps=steps)
    X, Y = inputs.centers2d(0, 1, 0, 1, N, N, r.parity)
    inner = (slice(steps + 1, N - steps - 1), slice(steps + 1, N - steps - 1))
    for k, l in pairs:
        want = dx ** k * dy ** l * deriv(X - a * r.t, Y - b * r.t, k, l)
        np.testing.assert_allclose(r.q[0, DOF(k, l)][inner], want[inner], rtol=0, atol=1e-12, err_msg=str((k, l)))


@pytest.mark.parametrize("eq", ["advection", "burgers"])
@pytest.mark.parametrize("parity", [0, 1])
def test_p0_is_staggered_lax_friedrichs(eq, parity):
    N = 12
    rng = np.random.default_rng(5)
    u = rng.uniform(0.2, 1.0, (N, N))
    pb = oracle.Problem2D(eq, 0, N, N, a=0.8, b=-0.3)
    dt = 0.1 * pb.dx
    out, _, fl = oracle.half_step2d(pb, parity, u[None, None], dt)
    f = 0.8 * u if eq == "advection" else 0.5 * u * u
    g = -0.3 * u if eq == "advection" else 0.5 * u * u
    o = 0 if parity == 0 else -1
    # old cell (i + o + di, j + o + dj) of new cell (i, j); arrays are [j][i]
    sh = lambda z, di, dj: np.roll(np.roll(z, -(o + dj), 0), -(o + di), 1)
    uA, uB, uC, uD = sh(u, 0, 0), sh(u, 0, 1), sh(u, 1, 0), sh(u, 1, 1)
    fA, fB, fC, fD = sh(f, 0, 0), sh(f, 0, 1), sh(f, 1, 0), sh(f, 1, 1)
    gA, gB, gC, gD = sh(g, 0, 0), sh(g, 0, 1), sh(g, 1, 0), sh(g, 1, 1)
    lam = dt / pb.dx
    want = 0.25 * (uA + uB + uC + uD) + 0.5 * lam * (fA + fB - fC - fD) + 0.5 * lam * (gA + gC - gB - gD)
    assert fl == 0
    np.testing.assert_allclose(out[0, 0], want, rtol=1e-14, atol=1e-15)


def _one_d(eq, P, N, q1, t_end, cfl, axis_x=True):
    pb = oracle.Problem(eq, P, N, bc="periodic", limiter=False, x_left=0.0, x_right=2.0, a=0.7)
    return oracle.run(pb, q1, t_end=t_end, cfl=cfl)


@pytest.mark.parametrize("eq", ["advection", "burgers"])
@pytest.mark.parametrize("P", [1, 2, 3])
@pytest.mark.parametrize("direction", ["x", "y"])
def test_reduces_to_1d_scalar(eq, P, direction):
    """u0 depending on x only (or y only): every row (column) follows the 1D
    scheme.  The 2D time step uses s_x/dx + s_y/dy; with the transverse speed
    zero (advection) or the step fixed (Burgers), both take the same dt."""
    N, M = 48, 4
    q1, _ = inputs.sine_wave(P, N, 0.0, 2.0, c0=0.6, amp=0.3, w=np.pi, phase=0.4)
    pb1 = oracle.Problem(eq, P, N, bc="periodic", limiter=False, x_left=0.0, x_right=2.0, a=0.7)
    dt = 0.2 * pb1.dx
    r1 = oracle.run(pb1, q1, dt_fixed=dt, max_half_steps=9)
    if direction == "x":
        pb2 = oracle.Problem2D(eq, P, N, M, x_right=2.0, y_right=2.0 * M / N, a=0.7, b=0.0)
        q2 = np.zeros((1, inputs.ndof2d(P), M, N))
        for k in range(P + 1):
            q2[0, DOF(k, 0)] = q1[0, k][None, :]
    else:
        pb2 = oracle.Problem2D(eq, P, M, N, x_right=2.0 * M / N, y_right=2.0, a=0.0, b=0.7)
        q2 = np.zeros((1, inputs.ndof2d(P), N, M))
        for k in range(P + 1):
            q2[0, DOF(0, k)] = q1[0, k][:, None]
    r2 = oracle.run2d(pb2, q2, dt_fixed=dt, max_half_steps=9)
    assert r2.parity == r1.parity == 1
    for k in range(P + 1):
        got = r2.q[0, DOF(k, 0)] if direction == "x" else r2.q[0, DOF(0, k)].T
        np.testing.assert_allclose(got, np.broadcast_to(r1.q[0, k], got.shape), rtol=0, atol=1e-13)
    for k, l in inputs.dof_pairs(P):
        if (direction == "x" and l > 0) or (direction == "y" and k > 0):
            assert np.all(r2.q[0, DOF(k, l)] == 0.0)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_reduces_to_1d_euler(P):
    """Euler data depending on x only with v = 0: rows follow the 1D Euler
    oracle and rho v stays zero."""
    N, M = 40, 3
    data = inputs.EulerPiecewise(np.array([]), np.array([0.8]), np.array([0.3]), np.array([0.9]),
                                 sine_amp=0.2, sine_w=np.pi, period=(0.0, 2.0), wrap_jump=False)
    x = inputs.centers(0.0, 2.0, N, N, 0)
    q1 = inputs.euler_taylor(data, x, 2.0 / N, P)
    pb1 = oracle.Problem("euler", P, N, bc="periodic", limiter=False, x_left=0.0, x_right=2.0)
    dt = 0.1 * pb1.dx
    r1 = oracle.run(pb1, q1, dt_fixed=dt, max_half_steps=7)
    pb2 = oracle.Problem2D("euler", P, N, M, x_right=2.0, y_right=2.0 * M / N)
    q2 = np.zeros((4, inputs.ndof2d(P), M, N))
    for k in range(P + 1):
        q2[0, DOF(k, 0)] = q1[0, k]
        q2[1, DOF(k, 0)] = q1[1, k]
        q2[3, DOF(k, 0)] = q1[2, k]
    r2 = oracle.run2d(pb2, q2, dt_fixed=dt, max_half_steps=7)
    for c1, c2 in ((0, 0), (1, 1), (2, 3)):
        for k in range(P + 1):
            got = r2.q[c2, DOF(k, 0)]
            np.testing.assert_allclose(got, np.broadcast_to(r1.q[c1, k], got.shape), rtol=0,
                                       atol=2e-13 * max(1.0, np.abs(r1.q[c1, k]).max()))
    assert np.all(r2.q[2] == 0.0)


# ---------------------------------------------------------------------------
# Invariants with the limiter on
# ---------------------------------------------------------------------------
def _transpose_state(P, q):
    """Swap x and y: DOF (k, l) <- (l, k), grid transposed."""
    out = np.empty_like(q.transpose(0, 1, 3, 2))
    for k, l in inputs.dof_pairs(P):
        out[:, DOF(l, k)] = q[:, DOF(k, l)].transpose(0, 2, 1)
    return out


@pytest.mark.parametrize("P", [1, 2, 3])
def test_xy_symmetry_burgers_limited(P):
    N = 24
    fn = inputs.Modes2D(0.3, np.array([0.4, 0.25]), np.pi * np.array([1.0, 2.0]), np.pi * np.array([2.0, 1.0]),
                        np.array([0.3, 0.3]))
    q = inputs.taylor2d(fn, P, N, N)
    q = 0.5 * (q + _transpose_state(P, q))        # symmetric data
    pb = oracle.Problem2D("burgers", P, N, N, limiter=True, x_right=2.0, y_right=2.0)
    r = oracle.run2d(pb, q, cfl=CFL[P], max_half_steps=40)
    assert r.flags == 0
    np.testing.assert_allclose(r.q, _transpose_state(P, r.q), rtol=0, atol=1e-12)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_conservation_burgers_limited(P):
    N = 20
    q = inputs.taylor2d(inputs.modes2d(P), P, N, N)
    pb = oracle.Problem2D("burgers", P, N, N, limiter=True, x_right=2.0, y_right=2.0)
    s0 = averages2d(P, q).sum()
    r = oracle.run2d(pb, q, cfl=CFL[P], max_half_steps=120)   # well past shock formation
    assert r.flags == 0
    s1 = averages2d(P, r.q).sum()
    assert abs(s1 - s0) < 1e-12 * np.abs(averages2d(P, q)).sum()


@pytest.mark.parametrize("P", [1, 2, 3])
def test_limiter_keeps_linear_data(P):
    """u0 = c + alpha x + beta y: every candidate has the exact slopes, so the
    limited polynomial is the data (weights sum to one).  a = b = 0 and
    dt = 0; cells next to the periodic seam (where the plane wraps) excluded."""
    N = 16
    pb = oracle.Problem2D("advection", P, N, N, limiter=True, a=0.0, b=0.0)
    J, I = np.mgrid[0:N, 0:N].astype(float)
    q = np.zeros((1, inputs.ndof2d(P), N, N))
    q[0, 0] = 0.3 + 0.02 * I - 0.05 * J
    q[0, DOF(1, 0)] = 0.02
    q[0, DOF(0, 1)] = -0.05
    out, _, _ = oracle.half_step2d(pb, 0, q, 0.0)
    inner = (slice(0, N - 1), slice(0, N - 1))
    np.testing.assert_allclose(out[0, DOF(1, 0)][inner], 0.02, rtol=0, atol=1e-15)
    np.testing.assert_allclose(out[0, DOF(0, 1)][inner], -0.05, rtol=0, atol=1e-15)
    np.testing.assert_allclose(out[0, 0][inner], (0.3 + 0.02 * (I + 0.5) - 0.05 * (J + 0.5))[inner], rtol=0,
                               atol=1e-14)
    for k, l in inputs.dof_pairs(P):
        if k + l >= 2:
            assert np.all(np.abs(out[0, DOF(k, l)][inner]) < 1e-15)


# ---------------------------------------------------------------------------
# Smoothness indicator (closed forms) and the limiter at a discontinuity
# ---------------------------------------------------------------------------
def _js_sympy(P, terms):
    """Eq. 2DSmoothIndicator integrated symbolically for p = sum c xi^a eta^b."""
    import sympy as sp
    xi, eta = sp.symbols("xi eta")
    p = sum(sp.Rational(c) * xi ** a * eta ** b for (a, b), c in terms.items())
    tot = 0
    for k, l in inputs.dof_pairs(P):
        if k + l == 0:
            continue
        d = sp.diff(p, xi, k, eta, l) if k and l else (sp.diff(p, xi, k) if k else sp.diff(p, eta, l))
        tot += sp.integrate(sp.integrate(d * d, (xi, -sp.Rational(1, 2), sp.Rational(1, 2))),
                            (eta, -sp.Rational(1, 2), sp.Rational(1, 2)))
    return float(tot)


@pytest.mark.parametrize("P,terms", [
    (1, {(1, 0): 3, (0, 1): -2}),
    (2, {(1, 1): 1}),
    (2, {(2, 0): 1, (0, 1): 1}),
    (3, {(2, 1): 1, (0, 3): -1, (1, 0): 2}),
    (3, {(3, 0): 1, (1, 2): 2, (0, 2): -1, (1, 1): 3}),
    (4, {(2, 2): 1, (4, 0): -1, (3, 1): 2, (1, 0): 1}),
])
def test_js_indicator_closed_form(P, terms):
    d = np.zeros(inputs.ndof2d(P))
    for (a, b), c in terms.items():
        d[DOF(a, b)] = c * math.factorial(a) * math.factorial(b)   # u_{ax,by} = a! b! coefficient
    want = _js_sympy(P, terms)
    assert oracle.js_indicator2d(P, d) == pytest.approx(want, rel=1e-14)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_limiter_tames_square_wave(P):
    """A square wave advected diagonally: unlimited, the high-order scheme
    rings well past the jump; limited, the solution stays within a small
    margin of [0, 1] (Section 3.2's purpose)."""
    N = 40
    X, Y = inputs.centers2d(0, 1, 0, 1, N, N, 0)
    q = np.zeros((1, inputs.ndof2d(P), N, N))
    q[0, 0] = ((np.abs(X - 0.5) < 0.2) & (np.abs(Y - 0.5) < 0.2)).astype(float)
    out = {}
    for lim in (False, True):
        pb = oracle.Problem2D("advection", P, N, N, limiter=lim, a=1.0, b=0.5)
        r = oracle.run2d(pb, q, cfl=CFL[P], t_end=0.25)
        out[lim] = (r.q[0, 0].min(), r.q[0, 0].max())
    assert out[False][0] < -0.08 or out[False][1] > 1.08
    assert out[True][0] > -0.01 and out[True][1] < 1.01


# ---------------------------------------------------------------------------
# 2D Burgers along the diagonal: u0 = w(x + y) gives w_t + (w^2)_s = 0 in
# s = x + y, i.e. 1D Burgers at twice the speed, solved exactly by the
# method of characteristics before the shock.
# ---------------------------------------------------------------------------
def burgers_diagonal_error(P, N, t_frac=0.5):
    import exact
    fn1 = inputs.SineSum(0.5, np.array([0.3]), np.array([np.pi]), np.array([0.7]))
    fn2 = inputs.Modes2D(0.5, np.array([0.3]), np.array([np.pi]), np.array([np.pi]), np.array([0.7]))
    t_end = t_frac * exact.breaking_time(fn1) / 2.0
    q = inputs.taylor2d(fn2, P, N, N)
    pb = oracle.Problem2D("burgers", P, N, N, limiter=False, x_right=2.0, y_right=2.0)
    r = oracle.run2d(pb, q, cfl=CFL[P], t_end=t_end)
    assert r.flags == 0 and r.t == t_end
    X, Y = inputs.centers2d(0, 2, 0, 2, N, N, r.parity)
    s = np.mod(X + Y, 2.0)
    want = exact.burgers_moc(fn1, s.ravel(), 2.0 * t_end).reshape(s.shape)
    return np.abs(r.q[0, 0] - want).mean()


@pytest.mark.parametrize("P", [1, 2, 3])
def test_burgers_diagonal_order(P):
    e1, e2 = burgers_diagonal_error(P, 32), burgers_diagonal_error(P, 64)
    order = np.log2(e1 / e2)
    assert order > P + 1 - 0.35, (P, e1, e2, order)


# ---------------------------------------------------------------------------
# Appendix B directly: for linear advection of a polynomial of degree <= P
# the expansion is exact, so every per-cell quantity equals its defining
# integral of u(x, y, t) = u0(x - a t, y - b t), evaluated symbolically.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_appendix_b_integrals_exact(P):
    import sympy as sp
    x, y, t = sp.symbols("x y t")
    a, b = sp.Rational(7, 10), sp.Rational(-3, 10)
    dx, dy, dt = sp.Rational(1, 8), sp.Rational(1, 4), sp.Rational(1, 40)
    rng = np.random.default_rng(40 + P)
    coef = {kl: sp.Rational(int(rng.integers(-9, 10)), 8) for kl in inputs.dof_pairs(P)}
    u0 = sum(c * x ** k * y ** l for (k, l), c in coef.items())        # cell centred at the origin
    u = u0.subs({x: x - a * t, y: y - b * t}, simultaneous=True)
    q = np.array([[float(sp.diff(u0, x, k, y, l).subs({x: 0, y: 0}) * dx ** k * dy ** l) if k + l else
                   float(u0.subs({x: 0, y: 0})) for k, l in inputs.dof_pairs(P)]])
    pb = oracle.Problem2D("advection", P, 8, 4, x_right=1.0, y_right=1.0, a=0.7, b=-0.3)
    got = oracle.old_cell2d(pb, q, float(dt))
    hx, hy = dx / 2, dy / 2
    avg = lambda x0, x1, y0, y1: sp.integrate(u0, (x, x0, x1), (y, y0, y1)) / ((x1 - x0) * (y1 - y0))
    want = {"RU": avg(0, hx, 0, hy), "RD": avg(0, hx, -hy, 0), "LU": avg(-hx, 0, 0, hy), "LD": avg(-hx, 0, -hy, 0)}
    f, g = a * u, b * u
    want["fU"] = sp.integrate(f.subs(x, 0), (y, 0, hy), (t, 0, dt)) / (hy * dt)
    want["fD"] = sp.integrate(f.subs(x, 0), (y, -hy, 0), (t, 0, dt)) / (hy * dt)
    want["gR"] = sp.integrate(g.subs(y, 0), (x, 0, hx), (t, 0, dt)) / (hx * dt)
    want["gL"] = sp.integrate(g.subs(y, 0), (x, -hx, 0), (t, 0, dt)) / (hx * dt)
    for name, w in want.items():
        assert got[name][0] == pytest.approx(float(w), rel=1e-13, abs=1e-15), name
    ut = u.subs(t, dt)                                                    # Eq. SubEq:2DUij
    for (k, l), v in got["V"][0].items():
        w = (sp.diff(ut, x, k, y, l) if k + l else ut).subs({x: 0, y: 0}) * dx ** k * dy ** l
        assert v == pytest.approx(float(w), rel=1e-13, abs=1e-15), (k, l)
