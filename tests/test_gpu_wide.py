"""GPU parity of the second tile shape (launch variant 4: wave tiles of 128
old cells, two per lane, 127 new cells per tile) against the FP64 oracle,
bit for bit: every equation and degree, every boundary condition, mesh sizes
at the 127/128-cell tile edges, launch shapes with ragged block ranges, and
the benchmark size.  The per-cell arithmetic is that of the 64-cell tiles;
only the work decomposition and the lane exchange differ."""
import numpy as np
import pytest

import oracle
from paper_2104_04347_amd import binding, inputs

from test_gpu_parity import assert_bitwise, gpu_run, oracle_run, scalar_data, _c3_reference

pytestmark = pytest.mark.gpu

WIDE = (256, 0, 4)


@pytest.mark.parametrize("eq", ["advection", "burgers"])
@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("lim", [False, True])
def test_wide_scalar_periodic(eq, P, lim):
    N = 1000
    q0, kw = scalar_data(eq, P, N)
    t_end = 0.15 if eq == "advection" else 0.6
    q, info, taken = gpu_run(eq, P, N, "periodic", q0, limiter=lim, t_end=t_end, cfl=0.3, launch=WIDE, **kw)
    ref = oracle_run(eq, P, N, "periodic", q0, limiter=lim, t_end=t_end, cfl=0.3, **kw)
    assert_bitwise(q, info, taken, ref, f"wide {eq} P={P} lim={lim}")


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
def test_wide_euler_transmissive(P, precision):
    N = 500
    q0, _ = inputs.euler_riemann(3, P, N)
    q, info, taken = gpu_run("euler", P, N, "transmissive", q0, limiter=True, t_end=0.12, cfl=0.25, launch=WIDE,
                             precision=precision)
    if precision == "fp64":
        ref = oracle_run("euler", P, N, "transmissive", q0, limiter=True, t_end=0.12, cfl=0.25)
        assert_bitwise(q, info, taken, ref, f"wide euler P={P}")
    else:   # same kernels' arithmetic as the 64-cell tiles: identical results
        q1, info1, taken1 = gpu_run("euler", P, N, "transmissive", q0, limiter=True, t_end=0.12, cfl=0.25,
                                    launch=(256, 0, 0), precision=precision)
        assert taken == taken1 and info.t == info1.t and np.array_equal(q, q1)


@pytest.mark.parametrize("P", [1, 2, 3])
def test_wide_dirichlet(P):
    N = 300
    x = inputs.centers(0.0, 2.0, N, N + 1, 0)
    _, fn = inputs.burgers_modes(0, P, N)
    q0 = np.stack([(2.0 / N) ** k * fn.deriv(x, k) for k in range(P + 1)])[None]
    kw = dict(x_left=0.0, x_right=2.0, left_state=(0.9, 0, 0), right_state=(0.2, 0, 0))
    q, info, taken = gpu_run("burgers", P, N, "dirichlet", q0, limiter=True, t_end=0.3, cfl=0.3, launch=WIDE, **kw)
    ref = oracle_run("burgers", P, N, "dirichlet", q0, limiter=True, t_end=0.3, cfl=0.3, **kw)
    assert_bitwise(q, info, taken, ref, f"wide dirichlet P={P}")


@pytest.mark.parametrize("N", [2, 3, 63, 64, 65, 126, 127, 128, 129, 190, 253, 254, 255, 256, 381, 382])
@pytest.mark.parametrize("case", ["euler-T", "adv-P"])
def test_wide_tile_edges(N, case):
    if case == "euler-T":
        q0, _ = inputs.euler_riemann(1, 2, N)
        args = ("euler", 2, N, "transmissive")
        kw = {}
    else:
        q0, kw = scalar_data("advection", 3, N)
        args = ("advection", 3, N, "periodic")
    q, info, taken = gpu_run(*args, q0, limiter=True, steps=9, cfl=0.2, launch=WIDE, **kw)
    ref = oracle_run(*args, q0, limiter=True, steps=9, cfl=0.2, **kw)
    assert_bitwise(q, info, taken, ref, f"wide {case} N={N}")


@pytest.mark.parametrize("shape", [(64, 1, 4), (64, 3, 4), (128, 5, 4), (192, 7, 4), (256, 2, 4), (256, 1000, 4)])
def test_wide_block_ranges(shape):
    """Grids whose blocks own ragged ranges of tiles (and more blocks than tiles)."""
    N = 2000
    q0, _ = inputs.euler_riemann(2, 3, N)
    q, info, taken = gpu_run("euler", 3, N, "transmissive", q0, limiter=True, steps=11, cfl=0.25, launch=shape)
    ref = oracle_run("euler", 3, N, "transmissive", q0, limiter=True, steps=11, cfl=0.25)
    assert_bitwise(q, info, taken, ref, f"wide shape {shape}")


@pytest.mark.parametrize("P", [2, 3])
@pytest.mark.parametrize("shape", [(256, 0, 4), (128, 0, 4), (256, 1024, 4)], ids=lambda s: f"t{s[0]}b{s[1]}")
def test_wide_c3_full_size(P, shape):
    """The benchmark size, N = 1,048,576, 6 half-steps in graph-replayed runs."""
    N = 1 << 20
    q0, ref = _c3_reference(P, 6)
    q, info, taken = gpu_run("euler", P, N, "transmissive", q0, limiter=True, steps=6, cfl=0.25, launch=shape)
    assert_bitwise(q, info, taken, ref, f"wide Euler N=2^20 P={P} launch {shape}")


def test_wide_long_run_graphs():
    """100 half-steps (two 48-step graphs and 4 single launches) equal
    100 single wcc_step calls and the oracle."""
    P, N = 3, 3001
    q0, _ = inputs.euler_riemann(5, P, N)
    a = binding.Solver("euler", P, N, "transmissive", limiter=True)
    a.set_launch(*WIDE)
    a.write(q0)
    a.run(100, 0.25)
    qa, ia = a.read()
    b = binding.Solver("euler", P, N, "transmissive", limiter=True)
    b.set_launch(*WIDE)
    b.write(q0)
    for _ in range(100):
        b.step(0.25)
    qb, ib = b.read()
    ref = oracle_run("euler", P, N, "transmissive", q0, limiter=True, steps=100, cfl=0.25)
    assert ia.t == ib.t == ref.t and np.array_equal(qa, qb) and np.array_equal(qa, ref.q)
