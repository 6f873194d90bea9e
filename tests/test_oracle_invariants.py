"""Pins of the oracle by invariants and special cases the paper and the
mathematics fix.

* P = 0 reduces to the staggered Lax-Friedrichs scheme (abstract; Eq.
  SubEq:1DIntegral with no derivative terms) -- bitwise, for scalars.
* Uniform states are preserved bitwise by every equation, degree and limiter
  setting.
* Conservation of the cell-average sum under periodic boundaries (Section 2.1
  remarks; the limiter keeps the average, Eq. 1DLimitedPolynomial).
* Mirror symmetry x -> -x of the PDEs.
* Limiter: the Jiang-Shu indicator (Eq. 1DSmoothIndicator) equals its closed
  form; constants untouched; smooth data at P >= 2 left (almost) untouched
  (Section 5.1: the limiter has no effect on the 3rd/4th-order schemes);
  the smooth side wins at a jump.
* Euler eigenvectors: L R = I and L A R = diag(u-c, u, u+c) with the analytic
  flux Jacobian (Section 4).
"""
from fractions import Fraction

import numpy as np
import pytest

import exact
import oracle
from paper_2104_04347_amd import inputs


def exact_fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


@pytest.mark.parametrize("eq", ["advection", "burgers"])
@pytest.mark.parametrize("parity", [0, 1])
def test_p0_is_staggered_lax_friedrichs(eq, parity):
    N = 37
    rng = np.random.default_rng(5)
    pb = oracle.Problem(eq, 0, N, a=-0.6, x_left=0.0, x_right=2.0)
    q = rng.uniform(-1.0, 1.0, (1, 1, N))
    dt = 0.37 * pb.dx
    qn, _, _ = oracle.half_step(pb, parity, q, dt)
    u = q[0, 0]
    lam = dt / pb.dx
    f = (lambda v: pb.a * v) if eq == "advection" else (lambda v: 0.5 * (v * v))
    for j in range(N):
        jl, jr = (j, (j + 1) % N) if parity == 0 else ((j - 1) % N, j)
        want = exact_fma(lam, f(u[jl]) - f(u[jr]), 0.5 * (u[jl] + u[jr]))
        assert qn[0, 0, j] == want


def test_p0_euler_lax_friedrichs():
    N = 20
    pb = oracle.Problem("euler", 0, N, x_left=0.0, x_right=1.0)
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.5, 1.0, N)
    u = rng.uniform(-0.5, 0.5, N)
    p = rng.uniform(0.5, 1.0, N)
    q = np.stack([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])[:, None, :]
    dt = 0.2 * pb.dx
    qn, _, _ = oracle.half_step(pb, 0, q, dt)
    lam = dt / pb.dx
    for j in range(N):
        L, R = q[:, 0, j], q[:, 0, (j + 1) % N]
        want = 0.5 * (L + R) + lam * (exact.euler_flux(L) - exact.euler_flux(R))
        np.testing.assert_allclose(qn[:, 0, j], want, rtol=4e-16, atol=4e-16)


CASES = [(eq, P, lim) for eq in ("advection", "burgers", "euler") for P in range(5) for lim in (False, True)]


@pytest.mark.parametrize("eq,P,lim", CASES)
@pytest.mark.parametrize("bc", ["periodic", "transmissive"])
def test_uniform_state_bitwise(eq, P, lim, bc):
    N = 16
    pb = oracle.Problem(eq, P, N, bc=bc, limiter=lim)
    if eq == "euler":
        q = inputs.euler_uniform(N, P, 0.7, -0.3, 0.45, bc=bc)
    else:
        q = np.zeros((1, P + 1, pb.ncells(0)))
        q[0, 0] = 0.83
    r = oracle.run(pb, q, t_end=0.3, cfl=0.25)
    assert r.flags == 0 and r.half_steps > 2
    n = pb.ncells(r.parity)
    assert np.array_equal(r.q, q[:, :, :1].repeat(n, axis=2) if n == q.shape[2] else
                          np.broadcast_to(q[:, :, :1], (pb.nc, P + 1, n)))


def cell_average(q, P):
    """Eq. SubEq:1DCellAVG: average = sum over even k of u_kx/((k+1)! 2^k)."""
    from math import factorial
    avg = q[:, 0].copy()
    for k in range(2, P + 1, 2):
        avg = avg + q[:, k] / (factorial(k + 1) * 2 ** k)
    return avg


@pytest.mark.parametrize("eq,P,lim", [("advection", 3, True), ("burgers", 2, True), ("burgers", 4, True),
                                      ("euler", 1, True), ("euler", 3, True), ("euler", 4, False)])
def test_conservation_periodic(eq, P, lim):
    N = 128
    if eq == "euler":
        q, _ = inputs.euler_multi_jump(3, P, N, n_jumps=3, bc="periodic")
        pb = oracle.Problem(eq, P, N, limiter=lim)
    elif eq == "burgers":
        q, _ = inputs.burgers_modes(4, P, N)
        pb = oracle.Problem(eq, P, N, limiter=lim, x_left=0.0, x_right=2.0)
    else:
        q, _ = inputs.sine_wave(P, N, 0.0, 1.0, c0=1.0, amp=0.2, w=2 * np.pi)
        pb = oracle.Problem(eq, P, N, limiter=lim)
    tot0 = cell_average(q, P).sum(axis=1)
    scale = np.abs(cell_average(q, P)).sum(axis=1)
    steps = 300
    r = oracle.run(pb, q, cfl=0.2, max_half_steps=steps)
    assert r.flags == 0
    tot = cell_average(r.q, P).sum(axis=1)
    assert np.all(np.abs(tot - tot0) <= 10 * 2.2e-16 * scale * np.sqrt(steps))


@pytest.mark.parametrize("eq,P,lim", [("advection", 3, False), ("advection", 2, True), ("burgers", 3, True),
                                      ("burgers", 1, True), ("euler", 2, True), ("euler", 4, True)])
def test_mirror_symmetry(eq, P, lim):
    """Reflect x -> -x: cell j -> -j (original mesh), odd derivatives change
    sign, and so do the advection speed, Burgers' u and the momentum."""
    N = 40
    if eq == "euler":
        q, _ = inputs.euler_multi_jump(7, P, N, n_jumps=2, bc="periodic")
        field_sign = np.array([1.0, -1.0, 1.0])
    elif eq == "burgers":
        q, _ = inputs.burgers_modes(1, P, N)
        field_sign = np.array([-1.0])
    else:
        q, _ = inputs.sine_wave(P, N, 0.0, 1.0, c0=0.3, amp=1.0, w=2 * np.pi, phase=0.4)
        field_sign = np.array([1.0])
    a = 0.8
    pb = oracle.Problem(eq, P, N, limiter=lim, a=a)
    pbm = oracle.Problem(eq, P, N, limiter=lim, a=-a)
    ksign = np.array([(-1.0) ** k for k in range(P + 1)])

    def mirror(qq, parity):
        idx = (-np.arange(N)) % N if parity == 0 else (N - 1 - np.arange(N))
        return qq[:, :, idx] * field_sign[:, None, None] * ksign[None, :, None]

    dt = 0.2 * pb.dx
    r = oracle.run(pb, q, dt_fixed=dt, max_half_steps=7)
    rm = oracle.run(pbm if eq == "advection" else pb, mirror(q, 0), dt_fixed=dt, max_half_steps=7)
    # Round-off differs between the two orientations and the limiter weights
    # amplify it near jumps; a sign or index mistake shows up at 1e-3 and above.
    np.testing.assert_allclose(rm.q, mirror(r.q, r.parity), rtol=0, atol=1e-11 * np.abs(r.q).max())


def test_js_indicator_closed_forms():
    """Eq. 1DSmoothIndicator in scaled derivatives; closed forms worked out by
    hand: P=2 gives the familiar 13/12."""
    rng = np.random.default_rng(0)
    for _ in range(50):
        d = rng.uniform(-2, 2, 5)
        d1, d2, d3, d4 = d[1:]
        js = {
            1: d1 * d1,
            2: d1 * d1 + 13 / 12 * d2 * d2,
            3: d1 * d1 + d1 * d3 / 12 + 13 / 12 * d2 * d2 + 1043 / 960 * d3 * d3,
        }
        js[4] = js[3] + 7 / 80 * d2 * d4 + 87617 / 80640 * d4 * d4
        for P in (1, 2, 3, 4):
            got = oracle.js_indicator(P, d[: P + 1])
            assert abs(got - js[P]) <= 1e-14 * max(1.0, abs(js[P]))


def test_js_indicator_by_quadrature():
    """Brute force: integrate the squared derivatives of the polynomial on a
    fine Gauss grid."""
    from math import factorial
    xg, wg = np.polynomial.legendre.leggauss(20)
    xg, wg = 0.5 * xg, 0.5 * wg
    rng = np.random.default_rng(1)
    for P in (1, 2, 3, 4):
        d = rng.uniform(-1, 1, P + 1)
        beta = 0.0
        for k in range(1, P + 1):
            vals = sum(d[j] * xg ** (j - k) / factorial(j - k) for j in range(k, P + 1))
            beta += np.sum(wg * vals * vals)
        assert abs(oracle.js_indicator(P, d) - beta) <= 1e-14


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_limiter_constants_untouched(P):
    d = np.zeros(P + 1)
    out = oracle.limit_field(P, 0.4, d, 0.4, 0.4)
    assert np.array_equal(out[1:], d[1:])


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_limiter_linear_data_untouched(P):
    """A linear polynomial whose vertex values match it exactly is a fixed
    point: s1 = s2 = d1; for P >= 2 sigma = tau = 0 so w0 = 1."""
    d = np.zeros(P + 1)
    d[1] = 0.25
    out = oracle.limit_field(P, 1.0, d, 1.0 - 0.125, 1.0 + 0.125)
    assert np.array_equal(out, d)


@pytest.mark.parametrize("P", [2, 3, 4])
def test_limiter_picks_smooth_side_at_jump(P):
    """Oscillatory u0 next to a jump: the limited slope ends near the smooth
    one-sided slope and higher derivatives are damped."""
    d = np.zeros(P + 1)
    d[1], d[2] = 1.0, 0.8
    if P >= 3:
        d[3] = -0.7
    if P >= 4:
        d[4] = 0.5      # tau = (u_Px)^2 must not vanish, else w0 = 1 (Eq. 1DHighOrderWeights)
    abar, vl, vr = 0.0, -0.01, 0.9      # smooth on the left, jump on the right
    out = oracle.limit_field(P, abar, d, vl, vr)
    s1 = 2 * (abar - vl)
    assert abs(out[1] - s1) < 0.05 * abs(d[1])
    assert np.all(np.abs(out[2:]) < 0.05 * np.abs(d[2:]) + 1e-30)


@pytest.mark.parametrize("P,N", [(2, 100), (3, 100), (4, 64)])
def test_limiter_no_effect_on_smooth_data(P, N):
    """Section 5.1 observes that the limiter has no effect on the 3rd- and
    4th-order schemes for a smooth wave: |WCC - LCC| far below the error."""
    nu = {2: 0.3, 3: 0.25, 4: 0.25}[P]
    q, _ = inputs.sine_wave(P, N, -1.0, 1.0)
    res = {}
    for lim in (False, True):
        pb = oracle.Problem("advection", P, N, x_left=-1.0, x_right=1.0, limiter=lim)
        res[lim] = oracle.run(pb, q, t_end=1.0, cfl=nu)
    x = oracle.Problem("advection", P, N, x_left=-1.0, x_right=1.0).centers(res[False].parity)
    err = np.abs(res[False].q[0, 0] - np.sin(np.pi * (x - 1.0))).max()
    diff = np.abs(res[True].q[0, 0] - res[False].q[0, 0]).max()
    assert diff <= 1e-3 * err


def test_euler_eigenvectors():
    rng = np.random.default_rng(3)
    for g in (1.4, 5 / 3, 3.0):
        for _ in range(20):
            rho, u, p = rng.uniform(0.1, 2), rng.uniform(-2, 2), rng.uniform(0.1, 2)
            U = np.array([rho, rho * u, p / (g - 1) + 0.5 * rho * u * u])
            L, R = oracle.euler_eigen(g, U)
            np.testing.assert_allclose(L @ R, np.eye(3), atol=1e-13)
            A = exact.euler_jacobian(U, g)
            c = np.sqrt(g * p / rho)
            np.testing.assert_allclose(L @ A @ R, np.diag([u - c, u, u + c]), atol=1e-12 * (1 + abs(u) + c) ** 2)


def test_euler_ck_first_level_matches_jacobian():
    """U_t = -A(U) U_x: first CK level of the Euler triangle, scaled by lam."""
    rng = np.random.default_rng(9)
    pb = oracle.Problem("euler", 3, 8)
    for _ in range(10):
        rho, u, p = rng.uniform(0.3, 1.5), rng.uniform(-1, 1), rng.uniform(0.3, 1.5)
        U = np.array([rho, rho * u, p / 0.4 + 0.5 * rho * u * u])
        qc = np.zeros((3, 4))
        qc[:, 0] = U
        qc[:, 1:] = rng.uniform(-0.3, 0.3, (3, 3))
        lam = 0.13
        T = oracle.ck_triangle(pb, qc, lam)
        want = -lam * exact.euler_jacobian(U) @ qc[:, 1]
        np.testing.assert_allclose(T[:, 0, 1], want, rtol=1e-13, atol=1e-14)


def test_dirichlet_ghost_uniform():
    """Dirichlet ghosts holding the interior constant state keep it exactly."""
    N, P = 12, 2
    pb = oracle.Problem("burgers", P, N, bc="dirichlet", limiter=True, left_state=(0.6,), right_state=(0.6,))
    q = np.zeros((1, P + 1, N + 1))
    q[0, 0] = 0.6
    r = oracle.run(pb, q, t_end=0.2, cfl=0.3)
    assert r.flags == 0 and np.all(r.q[0, 0] == 0.6) and np.all(r.q[0, 1:] == 0.0)


def test_nonfinite_and_positivity_flags():
    N, P = 16, 2
    pb = oracle.Problem("euler", P, N, limiter=True)
    q = inputs.euler_uniform(N, P, 1.0, 0.0, 1.0)
    q[0, 0, 5] = np.nan
    _, _, f = oracle.half_step(pb, 0, q, 0.1 * pb.dx)
    assert f & 1
    q = inputs.euler_uniform(N, P, 1.0, 0.0, 1.0)
    q[2, 0, 5:7] = 0.1     # energy below the kinetic energy: p < 0 in the new cell 5
    q[1, 0, 5:7] = 1.0
    _, _, f = oracle.half_step(pb, 0, q, 0.1 * pb.dx)
    assert f & 2


def brute_force_limited(P, abar, d, vl, vr, eps=1e-40):
    """Eq. 1D_U012 / 1DLimitedPolynomial / 1D2ndOrderWeights /
    1DHighOrderWeights with every ingredient computed by brute force:
    smoothness indicators and tau by Gauss quadrature of squared derivatives,
    the polynomial's edge values by direct evaluation, the candidates' average
    by quadrature of the polynomial."""
    from math import factorial
    xg, wg = np.polynomial.legendre.leggauss(20)
    xg, wg = 0.5 * xg, 0.5 * wg

    def deriv_poly(coef, k, x):   # k-th xi-derivative of sum_j coef_j xi^j / j!
        return sum(coef[j] * x ** (j - k) / factorial(j - k) for j in range(k, len(coef)))

    def js(coef):
        return sum(np.sum(wg * deriv_poly(coef, k, xg) ** 2) for k in range(1, len(coef)))

    pc = abar - sum(d[k] / (factorial(k + 1) * 2 ** k) for k in range(2, P + 1, 2))
    u0 = np.array([pc] + list(d[1:P + 1]))
    assert abs(np.sum(wg * deriv_poly(u0, 0, xg)) - abar) < 1e-13   # u0 has average abar
    s1, s2 = 2 * (abar - vl), 2 * (vr - abar)
    b = [js(u0), js(np.array([abar, s1])), js(np.array([abar, s2]))]
    if P == 1:
        wh = [(1.0 / (bm + eps)) ** 2 for bm in b]
    else:
        sigma = (deriv_poly(u0, 0, 0.5) - vr) ** 2 + (deriv_poly(u0, 0, -0.5) - vl) ** 2
        tau = np.sum(wg * deriv_poly(u0, P, xg) ** 2)
        r = [sigma * tau / (bm * bm + eps) for bm in b]
        wh = [1 + r[0] ** 2, r[1] ** 2, r[2] ** 2]
    w = np.array(wh) / sum(wh)
    out = np.zeros(P + 1)
    out[1] = w[0] * d[1] + w[1] * s1 + w[2] * s2
    out[2:] = w[0] * np.asarray(d[2:P + 1])
    return out


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_limiter_brute_force(P):
    rng = np.random.default_rng(100 + P)
    for _ in range(200):
        d = np.zeros(P + 1)
        d[1:] = rng.normal(0, 1, P) * rng.choice([1e-3, 1e-1, 1.0], P)
        abar = rng.uniform(-1, 1)
        vl = abar - 0.5 * d[1] + rng.normal(0, 1) * rng.choice([1e-4, 1e-2, 0.5])
        vr = abar + 0.5 * d[1] + rng.normal(0, 1) * rng.choice([1e-4, 1e-2, 0.5])
        got = oracle.limit_field(P, abar, d, vl, vr)
        want = brute_force_limited(P, abar, d, vl, vr)
        np.testing.assert_allclose(got[1:], want[1:], rtol=1e-9, atol=1e-13)
