"""The OpenMP build of the oracle (the same source with its cell loops split
over threads) gives the serial build's results bit for bit: every cell is
computed by the same operations, and the only reduction (largest wave speed,
NaN if any is NaN; status bits OR-ed) does not depend on the visiting order.
It exists to time the oracle on all host cores."""
import numpy as np
import pytest

import oracle
from oracle import build as obuild
from paper_2104_04347_amd import inputs


def _run(lib, pb, q0, **kw):
    with oracle.use_library(lib):
        return oracle.run(pb, q0, **kw), oracle.threads()


CASES = [
    ("euler", 3, 3001, "transmissive", True),
    ("euler", 4, 2048, "periodic", True),
    ("burgers", 2, 4097, "periodic", True),
    ("advection", 3, 1500, "dirichlet", False),
]


@pytest.mark.parametrize("eq,P,N,bc,lim", CASES)
def test_openmp_build_bitwise(eq, P, N, bc, lim):
    if eq == "euler":
        q0, _ = inputs.euler_riemann(3, P, N, bc=bc) if bc != "periodic" else inputs.euler_multi_jump(
            1, P, N, n_jumps=4, bc="periodic")
    else:
        pb0 = oracle.Problem(eq, P, N, bc=bc)
        rng = np.random.default_rng(8)
        q0 = np.zeros((1, P + 1, pb0.ncells(0)))
        q0[0, 0] = 0.5 + 0.3 * np.sin(2 * np.pi * pb0.centers(0)) + 0.05 * rng.standard_normal(pb0.ncells(0))
        q0[0, 1:] = 0.01 * rng.standard_normal((P, pb0.ncells(0)))
    pb = oracle.Problem(eq, P, N, bc=bc, limiter=lim, left_state=(0.4, 0, 0), right_state=(0.9, 0, 0))
    serial, n1 = _run(obuild.LIB, pb, q0, cfl=0.25, max_half_steps=9)
    par, nt = _run(obuild.LIB_OMP, pb, q0, cfl=0.25, max_half_steps=9)
    assert n1 == 1
    assert nt >= 1
    assert par.half_steps == serial.half_steps and par.parity == serial.parity
    assert par.t == serial.t and par.smax == serial.smax and par.flags == serial.flags
    assert np.array_equal(par.q, serial.q)


def test_openmp_build_flags_and_nan_speed():
    P, N = 2, 4000
    q0 = inputs.euler_uniform(N, P, 1.0, 0.0, 1.0)
    q0[0, 0, 2500] = np.nan
    pb = oracle.Problem("euler", P, N, limiter=True)
    outs = []
    for lib in (obuild.LIB, obuild.LIB_OMP):
        with oracle.use_library(lib):
            outs.append(oracle.half_step(pb, 0, q0, 0.1 * pb.dx))
    (qa, sa, fa), (qb, sb, fb) = outs
    assert fa == fb and fa & 1
    assert np.isnan(sa) and np.isnan(sb)
    assert np.array_equal(qa, qb, equal_nan=True)
