"""The 2D pins must catch plausible mistakes in the 2D oracle (on the periodic
and on the transmissive meshes): each case plants one mistake in a copy of
wcc2d_oracle.cpp, builds it with the real 1D source, and checks that a quick
selection of the 2D pins fails on it."""
import subprocess

import pytest

import oracle
from oracle import build as obuild

import test_oracle_2d as t2
import test_oracle_2d_ck as t2ck
import test_oracle_2d_limiter as t2l
import test_oracle_2d_transmissive as t2t

MUTANTS = {
    "LD quarter-average sign": ("ld = std::fma(((k + l) % 2) ? -qa : qa, x, ld);",
                                "ld = std::fma((k % 2) ? -qa : qa, x, ld);"),
    "flux integral 2^s dropped": ("FI[k][l] = 1.0 / ((double)(k + 1) * std::ldexp(1.0, k) * (double)(l + 1));",
                                  "FI[k][l] = 1.0 / ((double)(k + 1) * (double)(l + 1));"),
    "CK y factor index": ("std::fma(cy[l][m], G[c][k][l + 1][m - 1]", "std::fma(cy[k][m], G[c][k][l + 1][m - 1]"),
    "cross derivative not averaged": ("D[c][k][l] = (k >= 1 && l >= 1) ? 0.5 * (X + Y)",
                                      "D[c][k][l] = (k >= 1 && l >= 1) ? X"),
    "y correction index": ("Y = std::fma(K.CX2[t][s], D[c][k + s][lb + t], Y);",
                           "Y = std::fma(K.CX2[t][s], D[c][k + t][lb + s], Y);"),
    "vertex value factorial": ("o.V[c][k][l] = (k <= 1 && l <= 1) ? s : K.FF[k][l] * s;", "o.V[c][k][l] = s;"),
    "candidate slope vertex": ("a2 - (vld + vrd), vru - vrd", "a2 - (vld + vru), vru - vrd"),
    "sigma vertex sign": ("const int sx[4] = {-1, 1, 1, -1}", "const int sx[4] = {1, 1, 1, -1}"),
    "tau only one term": ("for (int k = 1; k <= P; ++k) tau = std::fma(D[k][P - k], D[k][P - k], tau);", ""),
    "indicator weight index": ("K.W2[cs[i] + cs[j]][ct[i] + ct[j]]", "K.W2[cs[i] + ct[j]][ct[i] + cs[j]]"),
    "Euler pressure drops rho v^2": ("(E[k][l][m] - 0.5 * (kx + ky))", "(E[k][l][m] - 0.5 * kx)"),
    "Euler energy flux velocity": ("G[3][k][l][m] = tprod3(w.W, w.v, k, l, m);",
                                   "G[3][k][l][m] = tprod3(w.W, w.u, k, l, m);"),
    "balance factor 1/2 dropped": ("hx = 0.5 * lamx", "hx = lamx"),
    "lower flux sign": ("fd = std::fma((s % 2) ? -fi : fi, F[c][0][s][m], fd);", "fd = std::fma(fi, F[c][0][s][m], fd);"),
    "point value sign": ("NQA[k][l] = (k % 2 == 0 && l % 2 == 0) ? -QA[k][l] : 0.0;",
                         "NQA[k][l] = (k % 2 == 0 && l % 2 == 0) ? QA[k][l] : 0.0;"),
    "limited x slope candidate": ("dx1 = std::fma(w[m], ux[m], dx1);", "dx1 = std::fma(w[m], uy[m], dx1);"),
    "rotated direction from rho": ("const double gx = D[3][1][0] / dx, gy = D[3][0][1] / dy;",
                                   "const double gx = D[0][1][0] / dx, gy = D[0][0][1] / dy;"),
    "rotated direction swapped": ("nx = gx / gn;\n    ny = gy / gn;", "nx = gy / gn;\n    ny = gx / gn;"),
    "left eigenvector sign": ("{-ut, -ny, nx, 0.0}", "{ut, -ny, nx, 0.0}"),
    "right eigenvector energy entry": ("{1.0, u, vv, 0.5 * q2}", "{1.0, u, vv, q2}"),
    "tangential velocity sign": ("ut = std::fma(vv, nx, -(u * ny))", "ut = std::fma(vv, nx, u * ny)"),
    "Taylor product time index": ("s = std::fma(X[a][b][c], Y[k - a][l - b][m - c], s);",
                                  "s = std::fma(X[a][b][c], Y[k - a][l - b][m], s);"),
    "Taylor quotient y index": ("s = std::fma(-Rho[a][b][c], V[k - a][l - b][m - c], s);",
                                "s = std::fma(-Rho[a][b][c], V[k - a][l][m - c], s);"),
    "candidate weights unsquared": ("      wh[m] = rm * rm;", "      wh[m] = rm;"),
    "back-projection with the left eigenvectors": ("out[r][k][l] = (f == 0) ? R[f][r] * cD[k][l] : std::fma(R[f][r], cD[k][l], out[r][k][l]);",
                                                   "out[r][k][l] = (f == 0) ? L[f][r] * cD[k][l] : std::fma(L[f][r], cD[k][l], out[r][k][l]);"),
    "vertex values projected from one vertex": ("for (int r = 0; r < 4; ++r) x[r] = v[r][vtx];",
                                                "for (int r = 0; r < 4; ++r) x[r] = v[r][0];"),
    "transmissive ghost wraps in x": ("    return i < 0 ? 0 : (i >= nx ? nx - 1 : i);", "    return (i % nx + nx) % nx;"),
    "transmissive edge mesh missing": ("ex = (px || parity == 1) ? 0 : 1", "ex = (px || parity == 0) ? 0 : 1"),
    "y edges follow x": ("const bool px = pb.bc == 0, py = bc_y_of(pb) == 0;",
                         "const bool px = pb.bc == 0, py = px;"),
}


def _brute_ok(eq):
    worst, acted = t2l.limiter_deviation(eq, 2, N=12)
    assert worst <= t2l.TOL[2] and acted >= 10


def quick_pins(first_only: bool = False) -> list:
    checks = [
        ("table3 P2", lambda: t2.test_table3_lccs_mesh_1_5(2)),
        ("table3 WCCS P1", lambda: t2.test_table3_wccs_mesh_1_5(1)),
        ("table3 WCCS P2", lambda: t2.test_table3_wccs_mesh_1_5(2)),
        ("exactness P3", lambda: t2.test_polynomial_exactness_advection(3)),
        ("LxF", lambda: [t2.test_p0_is_staggered_lax_friedrichs(e, p) for e in ("advection", "burgers") for p in (0, 1)]),
        ("1D x", lambda: t2.test_reduces_to_1d_scalar("burgers", 3, "x")),
        ("1D y", lambda: t2.test_reduces_to_1d_scalar("burgers", 3, "y")),
        ("1D Euler", lambda: t2.test_reduces_to_1d_euler(3)),
        ("symmetry", lambda: [t2.test_xy_symmetry_burgers_limited(P) for P in (2, 3)]),
        ("linear", lambda: t2.test_limiter_keeps_linear_data(2)),
        ("JS", lambda: [t2.test_js_indicator_closed_form(P, tm) for P, tm in
                        [(2, {(1, 1): 1}), (3, {(2, 1): 1, (0, 3): -1, (1, 0): 2})]]),
        ("square", lambda: [t2.test_limiter_tames_square_wave(P) for P in (2, 3)]),
        ("Appendix B", lambda: [t2.test_appendix_b_integrals_exact(P) for P in (2, 3)]),
        ("Burgers diagonal", lambda: t2.test_burgers_diagonal_order(2)),
        ("transmissive 1D Euler", lambda: t2t.test_reduces_to_1d_euler_transmissive(2)),
        ("transmissive interior", lambda: t2t.test_interior_equals_periodic("burgers", 3)),
        ("mixed edges 1D", lambda: t2t.test_periodic_x_transmissive_y_reduces_to_1d(2)),
        ("limiter brute force", lambda: [_brute_ok(eq) for eq in ("burgers", "euler")]),
        ("CK exact", lambda: [t2ck.test_ck_expansion_matches_exact_rational_solution(e, p)
                              for e, p in (("euler", 2), ("euler", 3))]),
    ]
    failed = []
    for name, fn in checks:
        try:
            fn()
        except Exception:       # a failed assertion or a rejected problem
            failed.append(name)
            if first_only:
                break
    return failed


def test_real_oracle_passes_quick_pins():
    assert quick_pins() == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(obuild.SRC2D).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {old!r}"
    mut = tmp_path / "mut2d.cpp"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut2d.so"
    subprocess.run(["g++", *obuild.CXXFLAGS, "-o", str(lib), obuild.SRC, str(mut)], check=True)
    with oracle.use_library(str(lib)):
        failed = quick_pins(first_only=True)
    assert failed, f"mutation '{name}' survived every pin"
