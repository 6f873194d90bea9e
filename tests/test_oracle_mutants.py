"""The pins must catch plausible mistakes in the oracle.

Each case copies the oracle source, plants one mistake (a dropped term, a wrong
sign, index or operand, a wrong loop order), builds the copy on the CPU and
checks that a quick selection of the pins fails on it.  The real oracle must
pass the same selection.
"""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest
import sympy as sp

import exact
import oracle
from oracle import build as obuild
from paper_2104_04347_amd import inputs

from test_oracle_linear import _mat, oracle_matrices
import test_oracle_boundary_speed as tbs
import test_oracle_ck_exact as tce
import test_oracle_euler_limiter as tel

import json

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MUTANTS = {
    "characteristic vertex operand": ("mat3(e.L, vl, cl);", "mat3(e.L, vr, cl);"),
    "back-projection matrix": ("mat3(e.Rm, cd[k], y);", "mat3(e.L, cd[k], y);"),
    "derivative correction sign": ("NCO[k] = (k % 2 == 1) ? -(2.0", "NCO[k] = (k % 2 == 1) ? (2.0"),
    "left half-average sign": ("SCA[k] = (k % 2 == 0) ? CA[k] : -CA[k];", "SCA[k] = CA[k];"),
    "CK factor (k+1)/m": ("CKR[k][m] = (m > 0) ? (double)(k + 1) / (double)m", "CKR[k][m] = (m > 0) ? (double)(k + 1) / (double)(m + 1)"),
    "Taylor product index": ("s = fmaR(X[a][b], Y[k - a][m - b], s);", "s = fmaR(X[a][b], Y[k - a][b], s);"),
    "Taylor quotient sign": ("s = fmaR(-Rho[a][b], V[k - a][m - b], s);", "s = fmaR(Rho[a][b], V[k - a][m - b], s);"),
    "pressure kinetic factor": ("gm1 * (ene[k][j] - half * w.Kin[k][j])", "gm1 * (ene[k][j] - w.Kin[k][j])"),
    "energy flux operand": ("G[2][k][j] = tprod(w.W, w.v, k, j);", "G[2][k][j] = tprod(ene, w.v, k, j);"),
    "limiter slope sign": ("R s1 = (abar - vl) * R(2.0);", "R s1 = (vl - abar) * R(2.0);"),
    "residual vertex swapped": ("R rp = ep - vr, rm = em - vl;", "R rp = ep - vl, rm = em - vr;"),
    "JS square index": ("sq = fmaR(cpoly[n], cpoly[s - n], sq);", "sq = fmaR(cpoly[n], cpoly[n], sq);"),
    "eigenvector entry": ("e.L[0][1] = R(-0.5) * (b1u + ic);", "e.L[0][1] = R(-0.5) * (b1u - ic);"),
    "vertex value factorial": ("out.V[c][k] = (k <= 1) ? s : R(K.fact[k]) * s;", "out.V[c][k] = s;"),
    "flux integral weight": ("RM[k] = 1.0 / (double)(k + 1);", "RM[k] = 1.0 / (double)(k + 2);"),
    "flux difference sign": ("abar[c] = fmaR(lam, Lc.fbar[c] - Rc.fbar[c], h);", "abar[c] = fmaR(lam, Rc.fbar[c] - Lc.fbar[c], h);"),
    "transmissive ghost side": ("oc[0] = oc[1];", "oc[0] = oc[(size_t)n_old];"),
    "derivative loop order": ("for (int k = P - 1; k >= 0; --k) {\n      R s = Rc.V[c][k] - Lc.V[c][k];",
                              "for (int k = 0; k < P; ++k) {\n      R s = Rc.V[c][k] - Lc.V[c][k];"),
    "point value sign": ("for (int k = 2; k <= P; k += 2) p = fmaR(R(K.NCA[k]), d[c][k], p);",
                         "for (int k = 2; k <= P; k += 2) p = fmaR(R(K.CA[k]), d[c][k], p);"),
    "weight normalisation term": ("R inv = R(1.0) / ((wh0 + wh1) + wh2);", "R inv = R(1.0) / (wh0 + wh1);"),
    "high-order weight +1 dropped": ("wh0 = fmaR(r0, r0, R(1.0));", "wh0 = r0 * r0;"),
    "tau from d1": ("R tau = d[P] * d[P];", "R tau = d[1] * d[1];"),
    "Dirichlet side swap": ("const double* st = side == 0 ? pb.left_state : pb.right_state;",
                            "const double* st = side == 0 ? pb.right_state : pb.left_state;"),
    "Dirichlet ghost keeps derivatives": (
        "q[c][k] = (k == 0) ? st[c] : 0.0;",
        "q[c][k] = (k == 0) ? st[c] : old_dofs[((int64_t)c * (P + 1) + k) * n_old + (side == 0 ? 0 : n_old - 1)];"),
    "speed without |u| (new cells)": ("speed = absR(eu) + ec;", "speed = eu + ec;"),
    "speed without |u| (state)": ("return absR(u) + c;", "return u + c;"),
    "Burgers speed without |u|": ("if (pb.equation == EQ_BURGERS) return absR(abar[0]);",
                                  "if (pb.equation == EQ_BURGERS) return abar[0];"),
    "advection speed without |a|": ("if (pb.equation == EQ_ADVECTION) return absR(R(pb.a));",
                                    "if (pb.equation == EQ_ADVECTION) return R(pb.a);"),
}


def quick_pins(first_only: bool = False) -> list:
    """A fast subset of the pins; returns the names of those that fail
    (first_only: stop at the first failing pin)."""
    failed = []

    def check(name, fn):
        if first_only and failed:
            return
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            failed.append(name)

    gold = json.load(open(os.path.join(GOLDEN, "appendix_a_matrices.json")))

    def appendix():
        for P in (1, 2, 3):
            got = oracle_matrices(P, 0.2371)
            for k, m in gold[f"P{P}"].items():
                if not np.allclose(got[k], _mat(m, 0.2371), rtol=0, atol=1e-14):
                    return False
        return True

    def table1():
        t1 = json.load(open(os.path.join(GOLDEN, "table1_advection.json")))
        for P, sch in ((1, "WCCS"), (3, "LCCS"), (3, "WCCS")):
            pb = oracle.Problem("advection", P, 50, x_left=-1.0, x_right=1.0, limiter=(sch == "WCCS"))
            q, _ = inputs.sine_wave(P, 50, -1.0, 1.0)
            r = oracle.run(pb, q, t_end=2.0, cfl=t1["cfl"][str(P)])
            err = np.abs(r.q[0, 0] - np.sin(np.pi * (pb.centers(r.parity) - 2.0)))
            if not (abs(err.mean() / t1[sch][str(P)]["L1"][0] - 1) < 0.03 and
                    abs(err.max() / t1[sch][str(P)]["Linf"][0] - 1) < 0.03):
                return False
        return True

    def gamma3():
        x = sp.Symbol("x", real=True)
        flow = exact.Gamma3Flow(0.1 * sp.sin(sp.pi * x + 1), 1 + 0.1 * sp.sin(sp.pi * x))
        errs = []
        for N in (40, 80):
            pb = oracle.Problem("euler", 3, N, x_left=0.0, x_right=2.0, gamma=3.0)
            r = oracle.run(pb, flow.taylor_state(pb.centers(0), pb.dx, 3), t_end=0.2, cfl=0.2)
            errs.append(np.abs(r.q[:, 0] - flow.exact_conserved(pb.centers(r.parity), r.t)).mean())
        return np.log2(errs[0] / errs[1]) > 3.5

    def eigen():
        U = np.array([0.8, 0.8 * 0.3, 0.6 / 0.4 + 0.5 * 0.8 * 0.09])
        L, R = oracle.euler_eigen(1.4, U)
        return np.allclose(L @ R, np.eye(3), atol=1e-13)

    def js():
        d = np.array([0.0, 0.3, -0.7, 0.4])
        d1, d2, d3 = d[1:]
        return abs(oracle.js_indicator(3, d) - (d1 * d1 + d1 * d3 / 12 + 13 / 12 * d2 * d2 + 1043 / 960 * d3 * d3)) < 1e-14

    def limiter_jump():
        d = np.array([0.0, 1.0, 0.8, -0.7])
        out = oracle.limit_field(3, 0.0, d, -0.01, 0.9)
        return abs(out[1] - 0.02) < 0.05 and np.all(np.abs(out[2:]) < 0.05)

    def sod():
        pb = oracle.Problem("euler", 2, 200, bc="transmissive", x_left=0.0, x_right=2.0, limiter=True)
        data = inputs.EulerPiecewise(np.array([1.0]), np.array([1.0, 0.125]), np.array([0.0, 0.0]),
                                     np.array([1.0, 0.1]), sine_amp=0.0)
        r = oracle.run(pb, inputs.euler_taylor(data, pb.centers(0), pb.dx, 2), t_end=0.4, cfl=0.3)
        x = pb.centers(r.parity)
        ex = exact.riemann_sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (x - 1.0) / r.t)
        return r.flags == 0 and np.abs(r.q[0, 0] - ex[0]).mean() < 8e-3

    def riemann_transmissive():
        # an asymmetric Riemann problem whose waves reach both ends
        q, _ = inputs.euler_riemann(11, 2, 64)
        pb = oracle.Problem("euler", 2, 64, bc="transmissive", limiter=True)
        r = oracle.run(pb, q, t_end=0.6, cfl=0.3)
        q2, _ = inputs.euler_riemann(11, 2, 128)
        pb2 = oracle.Problem("euler", 2, 128, bc="transmissive", limiter=True)
        r2 = oracle.run(pb2, q2, t_end=0.6, cfl=0.3)
        # consistency between resolutions at the left end cell (the data there is uniform)
        return r.flags == 0 and r2.flags == 0 and np.allclose(r.q[:, 0, 0], r2.q[:, 0, 0], rtol=0.02)

    def limiter_brute():
        from test_oracle_invariants import brute_force_limited
        rng = np.random.default_rng(7)
        for P in (1, 2, 3):
            for _ in range(20):
                d = np.zeros(P + 1)
                d[1:] = rng.normal(0, 1, P)
                abar = rng.uniform(-1, 1)
                vl, vr = abar - 0.5 * d[1] + rng.normal(0, 0.3), abar + 0.5 * d[1] + rng.normal(0, 0.3)
                if not np.allclose(oracle.limit_field(P, abar, d, vl, vr)[1:],
                                   brute_force_limited(P, abar, d, vl, vr)[1:], rtol=1e-9, atol=1e-13):
                    return False
        return True

    def dirichlet_ends():
        return (dirichlet_appendix() and tbs.dirichlet_contact_ends_kept(2, True)
                and tbs.dirichlet_inflow_errors(3, Ns=(100,))[0] < 1e-4)

    def dirichlet_appendix():
        return all(tbs.dirichlet_end_cells_match_appendix(P, 0.2371) < 4e-15 for P in (1, 2, 3))

    def euler_limiter():
        worst, acted = tel.euler_limiter_deviation(2, 96, steps=6)
        return worst <= tel.TOL[2] and acted >= 5

    def ck_exact():
        tce.test_ck_triangle_matches_exact_rational_solution("euler", 3)
        return True

    check("appendix A", appendix)
    check("CK exact", ck_exact)
    check("Euler characteristic limiter", euler_limiter)
    check("Dirichlet ghosts", dirichlet_ends)
    check("wave speed", tbs.wave_speed_time_steps_ok)
    check("limiter brute force", limiter_brute)
    check("table 1", table1)
    check("gamma=3 order", gamma3)
    check("eigenvectors", eigen)
    check("JS closed form", js)
    check("limiter at jump", limiter_jump)
    check("Sod", sod)
    check("transmissive ends", riemann_transmissive)
    return failed


def test_real_oracle_passes_quick_pins():
    assert quick_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
    mut = tmp_path / "mut.cpp"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["g++", *obuild.CXXFLAGS, "-o", str(lib), str(mut)], check=True)
    with oracle.use_library(str(lib)):
        failed = quick_pins(first_only=True)
    assert failed, f"mutation '{name}' survived every pin"
