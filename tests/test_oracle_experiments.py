"""The 1D experiments of Section 5 on the oracle: regression against the
values of tests/golden/experiments_1d.json (written from the oracle by
tests/golden/write_experiments_1d.py) and the qualitative statements the
paper makes about them:

* Section 5.1, Jiang-Shu composite: WCCS-3 and WCCS-4 are much better than
  WCCS-2 for every kind of profile; WCCS-4 is best on the smooth Gaussians.
* Section 5.2, Sod: WCCS-3 and WCCS-4 are clearly better than WCCS-2,
  especially at the contact; WCCS-3 and WCCS-4 perform alike.
* Section 5.2, modified Shu-Osher: WCCS-2 damps the entropy waves strongly;
  WCCS-4 is the best of the three.

The paper's further remark that WCCS-3 resolves discontinuities more
sharply than WCCS-4 is not reproduced (square-wave transitions of 5 and 4
cells); that reading is recorded in the design notes, not pinned here.
"""
import base64
import hashlib
import json
import os

import numpy as np
import pytest

import exact
import oracle
from paper_2104_04347_amd import inputs

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "experiments_1d.json")))
CFL = {1: 0.4, 2: 0.3, 3: 0.25}


def sha(q):
    return hashlib.sha256(np.ascontiguousarray(q, dtype=np.float64).tobytes()).hexdigest()


@pytest.mark.parametrize("P", [1, 2, 3])
def test_jiang_shu_regression(P):
    g = GOLD["jiang_shu"][f"P{P}"]
    pb = oracle.Problem("advection", P, 400, bc="periodic", limiter=True, x_left=-1.0, x_right=1.0)
    r = oracle.run(pb, inputs.jiang_shu(P, 400), t_end=12.0, cfl=CFL[P])
    assert (r.half_steps, r.parity, r.flags) == (g["half_steps"], g["parity"], 0)
    assert sha(r.q) == g["sha256"]
    x = inputs.centers(-1.0, 1.0, 400, 400, r.parity)
    err = np.abs(r.q[0, 0] - inputs.jiang_shu_u0(x))
    assert err.mean() == pytest.approx(g["L1"], rel=1e-12)


def test_jiang_shu_paper_statements():
    js = GOLD["jiang_shu"]
    for reg in ("gauss", "square", "triangle", "ellipse"):
        e1, e2, e3 = (js[f"P{P}"]["regions"][reg] for P in (1, 2, 3))
        assert e2 < e1 and e3 < e1, reg
    g1, g2, g3 = (js[f"P{P}"]["regions"]["gauss"] for P in (1, 2, 3))
    assert g3 < g2 < g1
    assert js["P3"]["L1"] < js["P2"]["L1"] < 0.5 * js["P1"]["L1"]


@pytest.mark.parametrize("P", [1, 2, 3])
def test_sod_regression_and_exact(P):
    g = GOLD["sod"][f"P{P}"]
    pb = oracle.Problem("euler", P, 200, bc="transmissive", limiter=True, x_left=0.0, x_right=2.0)
    r = oracle.run(pb, inputs.sod(P, 200)[0], t_end=0.4, cfl=CFL[P])
    assert (r.half_steps, r.parity, r.flags, r.t) == (g["half_steps"], g["parity"], 0, 0.4)
    assert sha(r.q) == g["sha256"]
    x = inputs.centers(0.0, 2.0, 200, pb.ncells(r.parity), r.parity)
    W = exact.riemann_sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (x - 1.0) / 0.4)
    err = np.abs(r.q[0, 0] - W[0])
    assert err.mean() == pytest.approx(g["L1_rho"], rel=1e-12)
    assert err.mean() < 5e-3          # a few cells of smearing at shock and contact on dx = 1/100


def test_sod_paper_statements():
    s = GOLD["sod"]
    c1, c2, c3 = (s[f"P{P}"]["contact_L1_rho"] for P in (1, 2, 3))
    assert c2 < 0.75 * c1 and c3 < 0.75 * c1
    l2, l3 = s["P2"]["L1_rho"], s["P3"]["L1_rho"]
    assert abs(l2 - l3) < 0.25 * max(l2, l3)


def _tt_reference():
    ref = GOLD["titarev_toro"]["reference"]
    rho = np.frombuffer(base64.b64decode(ref["rho_f32_b64"]), dtype="<f4").astype(np.float64)
    x = inputs.centers(-5.0, 5.0, ref["N"], rho.size, ref["parity"])
    return x, rho


@pytest.mark.slow
@pytest.mark.parametrize("P", [1, 2, 3])
def test_titarev_toro_regression(P):
    g = GOLD["titarev_toro"][f"P{P}"]
    pb = oracle.Problem("euler", P, 2000, bc="transmissive", limiter=True, x_left=-5.0, x_right=5.0)
    r = oracle.run(pb, inputs.shu_osher_tt(P, 2000)[0], t_end=5.0, cfl=CFL[P])
    assert (r.half_steps, r.parity, r.flags) == (g["half_steps"], g["parity"], 0)
    assert sha(r.q) == g["sha256"]
    xf, rf = _tt_reference()
    x = inputs.centers(-5.0, 5.0, 2000, pb.ncells(r.parity), r.parity)
    err = np.abs(r.q[0, 0] - np.interp(x, xf, rf))
    assert err.mean() == pytest.approx(g["L1_rho"], rel=1e-4)     # reference stored in float32


def test_titarev_toro_paper_statements():
    t = GOLD["titarev_toro"]
    w1, w2, w3 = (t[f"P{P}"]["waves_L1_rho"] for P in (1, 2, 3))
    assert w3 < w2 < w1
    assert w1 > 2.0 * w3                # WCCS-2 damps the compressed entropy waves
    assert t["reference"]["flags"] == 0 and t["reference"]["t"] == 5.0
