"""Pins of two oracle branches that the other pins leave open: the Dirichlet
ghost cells and the wave speed behind the CFL time step.

* Dirichlet ghosts (problem statement Eq. 1DHCL with boundary values u_L(t),
  u_R(t); the ghost staggered cells centred at x_L - dx/2 and x_R + dx/2 of
  the mesh in Section 2.1).  The reading taken: the ghost beside x_L holds the
  left boundary state, the one beside x_R the right state, both as constant
  polynomials (zero derivatives).  Pinned by
  - the end cells of one odd->even half-step of linear advection against the
    paper's own matrices: q_new = M1 q_left_parent + M2 q_right_parent
    (Eq. 1DSchemeMatrixForm, Appendix A) with q_ghost = (state, 0, ..., 0);
  - P = 0 against the staggered Lax-Friedrichs formula, bitwise;
  - a stationary Euler contact between two different states, whose uniform
    ends are kept bit for bit only if each ghost holds its own side's state;
  - a smooth advected profile whose inflow state enters through the left
    ghost, against the exact shifted solution u0(x - a t).
* Wave speed (Section 5 preamble: nu = max|wave speed| dt / dx): |a| for
  advection, |u| for Burgers and |u| + c for the Euler equations, from the
  cell averages.  Pinned with negative velocities, where a dropped absolute
  value changes the time step.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import sympy as sp

import oracle

from test_oracle_linear import _mat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _appendix(P, nu):
    gold = json.load(open(os.path.join(GOLDEN, "appendix_a_matrices.json")))[f"P{P}"]
    return _mat(gold["M01"], nu), _mat(gold["M02"], nu)


def dirichlet_end_cells_match_appendix(P, nu, seed=3):
    """One odd->even half-step of u_t + u_x = 0 with distinct Dirichlet
    states; returns the largest deviation of the two end cells from
    M1 q_L + M2 q_R with the ghost as the missing parent."""
    N = 10
    left, right = 0.9, -0.35
    pb = oracle.Problem("advection", P, N, bc="dirichlet", a=1.0, left_state=(left,), right_state=(right,))
    rng = np.random.default_rng(seed)
    q = rng.uniform(-1.0, 1.0, (1, P + 1, pb.ncells(1)))
    qn, _, _ = oracle.half_step(pb, 1, q, nu * pb.dx)
    M1, M2 = _appendix(P, nu)
    gl = np.zeros(P + 1)
    gl[0] = left
    gr = np.zeros(P + 1)
    gr[0] = right
    want0 = M1 @ gl + M2 @ q[0, :, 0]          # new cell at x_L: ghost, old cell 0
    wantN = M1 @ q[0, :, N - 1] + M2 @ gr      # new cell at x_R: old cell N-1, ghost
    return max(np.max(np.abs(qn[0, :, 0] - want0)), np.max(np.abs(qn[0, :, N] - wantN)))


@pytest.mark.parametrize("P", [1, 2, 3])
@pytest.mark.parametrize("nu", [0.1, 0.2371, 0.4])
def test_dirichlet_end_cells_appendix_a(P, nu):
    assert dirichlet_end_cells_match_appendix(P, nu) < 4e-15


def test_dirichlet_interior_unchanged_by_ghosts():
    """Cells whose parents are both interior do not see the ghosts: same new
    state as the transmissive run, bit for bit."""
    P, N = 2, 12
    rng = np.random.default_rng(4)
    q = rng.uniform(-1.0, 1.0, (1, P + 1, N))
    a = oracle.Problem("advection", P, N, bc="dirichlet", left_state=(0.3,), right_state=(-0.8,))
    b = oracle.Problem("advection", P, N, bc="transmissive")
    qa, _, _ = oracle.half_step(a, 1, q, 0.3 * a.dx)
    qb, _, _ = oracle.half_step(b, 1, q, 0.3 * b.dx)
    assert np.array_equal(qa[:, :, 1:N], qb[:, :, 1:N])
    assert not np.array_equal(qa[:, :, 0], qb[:, :, 0]) and not np.array_equal(qa[:, :, N], qb[:, :, N])


@pytest.mark.parametrize("eq", ["advection", "burgers"])
def test_dirichlet_p0_lax_friedrichs_ends(eq):
    """P = 0: the end cells are the staggered Lax-Friedrichs update with the
    boundary state as the outer parent, bit for bit."""
    N = 9
    left, right = 0.7, -0.45
    pb = oracle.Problem(eq, 0, N, bc="dirichlet", a=0.8, left_state=(left,), right_state=(right,))
    rng = np.random.default_rng(6)
    q = rng.uniform(-1.0, 1.0, (1, 1, N))
    dt = 0.31 * pb.dx
    qn, _, _ = oracle.half_step(pb, 1, q, dt)
    lam = dt / pb.dx
    f = (lambda v: pb.a * v) if eq == "advection" else (lambda v: 0.5 * (v * v))

    def lf(uL, uR):
        # one correctly rounded fused multiply-add, as the canonical order writes it
        return float(Fraction(lam) * Fraction(f(uL) - f(uR)) + Fraction(0.5 * (uL + uR)))

    assert qn[0, 0, 0] == lf(left, q[0, 0, 0])
    assert qn[0, 0, N] == lf(q[0, 0, N - 1], right)


def dirichlet_contact_ends_kept(P, limiter, half_steps=10):
    """A stationary contact (u = 0, p equal, rho different) between the two
    Dirichlet states; True if the cells outside the jump's numerical domain of
    dependence still hold their side's state bit for bit."""
    N, g = 64, 1.4
    rhoL, rhoR, p = 1.0, 0.3, 0.7
    UL = (rhoL, 0.0, p / (g - 1.0))
    UR = (rhoR, 0.0, p / (g - 1.0))
    pb = oracle.Problem("euler", P, N, bc="dirichlet", limiter=limiter, left_state=UL, right_state=UR)
    n0 = pb.ncells(0)
    q = np.zeros((3, P + 1, n0))
    for c in range(3):
        q[c, 0, : n0 // 2] = UL[c]
        q[c, 0, n0 // 2:] = UR[c]
    r = oracle.run(pb, q, cfl=0.25, max_half_steps=half_steps)
    keep = half_steps // 2 + 2
    n = r.q.shape[2]
    left_ok = all(np.all(r.q[c, 0, : n // 2 - keep] == UL[c]) for c in range(3))
    right_ok = all(np.all(r.q[c, 0, n // 2 + keep:] == UR[c]) for c in range(3))
    return r.flags == 0 and left_ok and right_ok and np.all(r.q[:, 1:, : n // 2 - keep] == 0.0)


@pytest.mark.parametrize("P", [0, 1, 2, 3])
@pytest.mark.parametrize("limiter", [False, True])
def test_dirichlet_euler_contact_ends_bitwise(P, limiter):
    assert dirichlet_contact_ends_kept(P, limiter)


def _smooth_step_fn():
    """C-infinity step from 0 (s <= 0) to 1 (s >= 1) and its derivatives."""
    s = sp.Symbol("s", real=True)
    h0, h1 = sp.exp(-1 / s), sp.exp(-1 / (1 - s))
    S = h0 / (h0 + h1)
    return [sp.lambdify(s, sp.diff(S, s, k), "numpy") for k in range(5)]


def dirichlet_inflow_errors(P, Ns=(100, 200), t_end=0.25):
    """u_t + u_x = 0 on [0, 1], u0 = cL + (cR - cL) S((x - 0.35)/0.3) with the
    Dirichlet states cL (inflow) and cR; L_inf error against u0(x - t) for
    each N (Taylor initial data, CFL per half-step 0.25, limiter off)."""
    cL, cR, x0, w = 0.8, -0.4, 0.35, 0.3
    dS = _smooth_step_fn()

    def u0_deriv(x, k):
        s = (x - x0) / w
        inside = (s > 0) & (s < 1)
        out = np.zeros_like(x)
        if k == 0:
            out[s >= 1] = 1.0
        with np.errstate(all="ignore"):
            out[inside] = dS[k](s[inside])
        scale = (cR - cL) / w ** k
        return (cL if k == 0 else 0.0) + scale * out

    errs = []
    for N in Ns:
        pb = oracle.Problem("advection", P, N, bc="dirichlet", a=1.0, left_state=(cL,), right_state=(cR,))
        x = pb.centers(0)
        q = np.stack([u0_deriv(x, k) * pb.dx ** k for k in range(P + 1)])[None]
        r = oracle.run(pb, q, t_end=t_end, cfl=0.25)
        xe = pb.centers(r.parity)
        exact = u0_deriv(xe - r.t, 0)
        errs.append(float(np.max(np.abs(r.q[0, 0] - exact))))
    return errs


@pytest.mark.parametrize("P", [1, 2, 3])
def test_dirichlet_inflow_exact_shift(P):
    e100, e200 = dirichlet_inflow_errors(P)
    assert e200 < {1: 2e-3, 2: 1e-4, 3: 1e-5}[P]
    assert math.log2(e100 / e200) > P + 1 - 0.6


def _euler_state(rho, u, p, g=1.4):
    return (rho, rho * u, p / (g - 1.0) + 0.5 * rho * u * u)


def wave_speed_time_steps_ok():
    """Uniform states with negative velocity: two CFL half-steps must each
    take dt = (cfl dx)/s with s = |a|, |u| or |u| + c."""
    cfl = 0.3
    cases = []
    N, P = 16, 2
    # advection, a < 0
    pb = oracle.Problem("advection", P, N, a=-0.7)
    q = np.zeros((1, P + 1, N))
    q[0, 0] = 0.25
    cases.append((pb, q, 0.7))
    # Burgers, u < 0
    pb = oracle.Problem("burgers", P, N, limiter=True)
    q = np.zeros((1, P + 1, N))
    q[0, 0] = -0.6
    cases.append((pb, q, 0.6))
    # Euler, u < 0 with |u| < c (u + c > 0, so a dropped |.| still gives a positive speed)
    rho, u, p, g = 0.8, -0.5, 0.6, 1.4
    pb = oracle.Problem("euler", P, N, limiter=True)
    q = np.zeros((3, P + 1, N))
    for c_, v in enumerate(_euler_state(rho, u, p, g)):
        q[c_, 0] = v
    cases.append((pb, q, abs(u) + math.sqrt(g * p / rho)))
    for pb, q, s in cases:
        s0 = oracle.max_speed(pb, 0, q)
        r = oracle.run(pb, q, cfl=cfl, max_half_steps=2)
        dt = (cfl * pb.dx) / s
        if not (abs(s0 - s) <= 1e-14 * s and abs(r.smax - s) <= 1e-14 * s and abs(r.t - 2 * dt) <= 1e-14 * dt):
            return False
    return True


def test_wave_speed_negative_velocity():
    assert wave_speed_time_steps_ok()


def test_euler_speed_matches_characteristic_speeds():
    """|u| + c is the largest |eigenvalue| of the flux Jacobian (u - c, u, u + c)."""
    rng = np.random.default_rng(12)
    g = 1.4
    for _ in range(20):
        rho, u, p = rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0)
        pb = oracle.Problem("euler", 0, 4, gamma=g)
        q = np.zeros((3, 1, 4))
        for c_, v in enumerate(_euler_state(rho, u, p, g)):
            q[c_, 0] = v
        c = math.sqrt(g * p / rho)
        want = max(abs(u - c), abs(u), abs(u + c))
        assert abs(oracle.max_speed(pb, 0, q) - want) <= 1e-14 * want


def transmissive_outflow_errors(P, Ns=(100, 200, 400), t_end=0.45):
    """u_t + u_x = 0 on [0, 1], transmissive ends, a Gaussian bump
    1 + 0.2 exp(-((x - 0.75)/0.08)^2) that leaves through x = 1; L_inf error
    against u0(x - t) for each N (Taylor data, CFL per half-step 0.25)."""
    s = sp.Symbol("s", real=True)
    f = 1 + sp.Rational(1, 5) * sp.exp(-((s - sp.Rational(3, 4)) / sp.Rational(2, 25)) ** 2)
    fs = [sp.lambdify(s, sp.diff(f, s, k), "numpy") for k in range(P + 1)]
    errs = []
    for N in Ns:
        pb = oracle.Problem("advection", P, N, bc="transmissive", a=1.0)
        x = pb.centers(0)
        q = np.stack([np.asarray(fs[k](x), dtype=float) * pb.dx ** k for k in range(P + 1)])[None]
        r = oracle.run(pb, q, t_end=t_end, cfl=0.25)
        exact = np.asarray(fs[0](pb.centers(r.parity) - r.t), dtype=float)
        errs.append(float(np.max(np.abs(r.q[0, 0] - exact))))
    return errs


@pytest.mark.parametrize("P", [1, 2, 3])
def test_transmissive_outflow_non_reflecting(P):
    """The paper names the outer boundary "non-reflection" and says nothing
    more.  A wave that leaves through a transmissive end must leave no
    reflection beyond what vanishes under refinement (at least first order:
    the ghost is a copy of the adjacent cell).  The choice of copying all
    DOFs rather than only the average is a reading the paper does not fix;
    both satisfy this property."""
    e = transmissive_outflow_errors(P)
    assert e[-1] < 1e-5
    assert math.log2(e[0] / e[-1]) > 2 * 0.9
