"""GPU parity of the staged (line-aligned store) kernel variants.

The staged variants compute every new cell exactly as the direct-store
kernels do and only change how the new cells reach memory: through LDS, in
whole 64-cell groups, with a group that straddles two iterations of a block
carried between them.  Bar: bit-identical states against the FP64 oracle
(binary64) and against the direct-store kernels (both precisions), over tile
edges, launch shapes whose block ranges end anywhere inside a group, every
boundary kind, and batches whose runs of tiles change instance in the middle
of a block iteration."""
import numpy as np
import pytest

import oracle
from paper_2104_04347_amd import binding, inputs

pytestmark = pytest.mark.gpu

STAGED = [2, 3]          # variant bits: 2 = staged stores, 3 = staged + prefetch


def run_gpu(eq, P, N, bc, q0, steps, cfl, *, variant, threads=256, blocks=0, precision="fp64", limiter=True, **kw):
    print(f"staged: {eq} P={P} N={N} {bc} variant={variant} threads={threads} blocks={blocks} {precision}",
          flush=True)
    s = binding.Solver(eq, P, N, bc, limiter=limiter, precision=precision, **kw)
    try:
        s.set_launch(threads, blocks, variant)
        s.write(q0)
        s.run(steps, cfl)
        q, info = s.read()
    finally:
        s.close()
    return q, info


def check_oracle(q, info, eq, P, N, bc, q0, steps, cfl, limiter=True, **kw):
    ref = oracle.run(oracle.Problem(eq, P, N, bc=bc, limiter=limiter, **kw), q0, cfl=cfl, max_half_steps=steps)
    assert info.flags & 3 == 0 and ref.flags == 0
    assert info.parity == ref.parity and info.t == ref.t
    if not np.array_equal(q, ref.q):
        bad = np.argwhere(q != ref.q)
        raise AssertionError(f"{len(bad)} values differ, first at {tuple(bad[0])}")


@pytest.mark.parametrize("variant", STAGED)
@pytest.mark.parametrize("N", [2, 3, 62, 63, 64, 65, 125, 126, 127, 128, 189, 190, 255, 256, 257, 4031, 4033])
def test_tile_edges_euler_transmissive(N, variant):
    q0, _ = inputs.euler_riemann(1, 2, N)
    q, info = run_gpu("euler", 2, N, "transmissive", q0, 9, 0.2, variant=variant)
    check_oracle(q, info, "euler", 2, N, "transmissive", q0, 9, 0.2)


@pytest.mark.parametrize("variant", STAGED)
@pytest.mark.parametrize("eq", ["advection", "burgers"])
@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
def test_scalar_periodic(eq, P, variant):
    N = 1000
    if eq == "advection":
        q0, _ = inputs.sine_wave(P, N, 0.0, 1.0, c0=1.0, amp=0.2, w=2 * np.pi)
        kw = dict(x_left=0.0, x_right=1.0, a=1.0)
    else:
        q0, _ = inputs.burgers_modes(0, P, N)
        kw = dict(x_left=0.0, x_right=2.0)
    lim = P > 0
    q, info = run_gpu(eq, P, N, "periodic", q0, 12, 0.25, variant=variant, limiter=lim, **kw)
    check_oracle(q, info, eq, P, N, "periodic", q0, 12, 0.25, limiter=lim, **kw)


@pytest.mark.parametrize("variant", STAGED)
@pytest.mark.parametrize("P", [1, 3])
def test_dirichlet(P, variant):
    N = 700
    q0, _ = inputs.euler_riemann(2, P, N)
    kw = dict(x_left=0.0, x_right=1.0, left_state=[1.0, 0.0, 2.5], right_state=[0.125, 0.0, 0.25])
    q, info = run_gpu("euler", P, N, "dirichlet", q0, 10, 0.2, variant=variant, **kw)
    check_oracle(q, info, "euler", P, N, "dirichlet", q0, 10, 0.2, **kw)


@pytest.mark.parametrize("variant", STAGED)
@pytest.mark.parametrize("threads,blocks", [(64, 1), (64, 7), (128, 3), (192, 5), (192, 64), (256, 1), (256, 9),
                                            (256, 4096)])
def test_launch_shapes(threads, blocks, variant):
    """Block ranges of every length, one to four waves per block, more blocks
    than tiles."""
    N = 5001
    q0, _ = inputs.euler_riemann(3, 3, N)
    q, info = run_gpu("euler", 3, N, "transmissive", q0, 7, 0.25, variant=variant, threads=threads, blocks=blocks)
    check_oracle(q, info, "euler", 3, N, "transmissive", q0, 7, 0.25)


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("variant", STAGED)
def test_full_size_equals_direct(precision, variant):
    """N = 2^20 Euler P = 3 (the benchmark workload): staged == direct stores,
    bit for bit, in the library's default launch shape."""
    N = 1 << 20
    q0, _ = inputs.euler_riemann(0, 3, N)
    q, info = run_gpu("euler", 3, N, "transmissive", q0, 8, 0.25, variant=variant, threads=0, precision=precision)
    r, rinfo = run_gpu("euler", 3, N, "transmissive", q0, 8, 0.25, variant=0, threads=0, precision=precision)
    assert info.t == rinfo.t and info.parity == rinfo.parity
    assert np.array_equal(q, r)


def _batch(precision, mode, spec, qs, steps, threads=256, blocks=0):
    print(f"staged batch: mode={mode} threads={threads} blocks={blocks} {precision} B={spec.P.size}", flush=True)
    cfl = [0.4, 0.4, 0.3, 0.25, 0.25]
    bt = binding.Batch("euler", spec.P, spec.N, "transmissive", limiter=True, precision=precision)
    try:
        bt.set_schedule(threads, blocks, mode)
        for b, q in enumerate(qs):
            bt.write(b, q)
        bt.prepare()
        bt.run(steps, cfl)
        return [bt.read(b) for b in range(spec.P.size)]
    finally:
        bt.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("mode", [3, 4, 5, 6])
@pytest.mark.parametrize("threads,blocks", [(256, 0), (64, 5), (192, 3), (128, 40)])
def test_batch_staged_equals_direct(precision, mode, threads, blocks):
    """Batches with instances of every degree and sizes around the tile and
    group edges (a block iteration's waves cross instance boundaries)."""
    spec = inputs.batch_spec(14, 11, n_lo=40, n_hi=900)
    spec.N[:6] = [2, 62, 63, 64, 126, 127]
    qs = [inputs.batch_instance(spec, b) for b in range(spec.P.size)]
    got = _batch(precision, mode, spec, qs, 21, threads, blocks)
    ref = _batch(precision, 2, spec, qs, 21)
    for b in range(spec.P.size):
        assert got[b][1].t == ref[b][1].t, b
        assert np.array_equal(got[b][0], ref[b][0]), f"instance {b} (P={spec.P[b]}, N={spec.N[b]})"


def test_batch_staged_fp64_matches_oracle():
    spec = inputs.batch_spec(7, 12, n_lo=40, n_hi=700)
    qs = [inputs.batch_instance(spec, b) for b in range(spec.P.size)]
    got = _batch("fp64", 4, spec, qs, 15)
    cfl = [0.4, 0.4, 0.3, 0.25, 0.25]
    for b, q in enumerate(qs):
        P, N = int(spec.P[b]), int(spec.N[b])
        ref = oracle.run(oracle.Problem("euler", P, N, bc="transmissive", limiter=True), q, cfl=cfl[P],
                         max_half_steps=15)
        assert got[b][1].t == ref.t and np.array_equal(got[b][0], ref.q), b


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("mode", [1, 3, 4, 5, 6])
def test_batch_graphs_equal_direct(precision, mode):
    """50 half-steps: two captured 24-half-step graphs (with one branch per
    degree in modes 5 and 6) and two enqueued half-steps, against the
    grouped direct schedule run the same way, and each instance's time
    against its single-instance run."""
    spec = inputs.batch_spec(12, 13, n_lo=40, n_hi=1500)
    spec.N[:4] = [2, 63, 64, 127]
    qs = [inputs.batch_instance(spec, b) for b in range(spec.P.size)]
    got = _batch(precision, mode, spec, qs, 50)
    ref = _batch(precision, 2, spec, qs, 50)
    cfl = [0.4, 0.4, 0.3, 0.25, 0.25]
    for b in range(spec.P.size):
        assert got[b][1].half_steps == 50 and got[b][1].t == ref[b][1].t, b
        assert np.array_equal(got[b][0], ref[b][0]), f"instance {b} (P={spec.P[b]}, N={spec.N[b]})"
    # one instance of every degree against its own single-instance run
    for P in (1, 2, 3):
        b = int(np.flatnonzero(spec.P == P)[0])
        s = binding.Solver("euler", P, int(spec.N[b]), "transmissive", limiter=True, precision=precision)
        try:
            s.write(qs[b])
            s.run(50, cfl[P])
            q1, i1 = s.read()
        finally:
            s.close()
        assert i1.t == got[b][1].t and np.array_equal(q1, got[b][0]), f"instance {b} vs single"


@pytest.mark.parametrize("mode", [5, 6])
def test_batch_branches_single_degree(mode):
    """Parallel degree branches with only one degree present (one branch)."""
    spec = inputs.batch_spec(6, 14, n_lo=40, n_hi=900, degrees=(2,))
    qs = [inputs.batch_instance(spec, b) for b in range(spec.P.size)]
    got = _batch("fp64", mode, spec, qs, 30)
    ref = _batch("fp64", 2, spec, qs, 30)
    for b in range(spec.P.size):
        assert got[b][1].t == ref[b][1].t and np.array_equal(got[b][0], ref[b][0]), b


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("variant", STAGED)
def test_graph_replay_equals_direct(precision, variant):
    """100 half-steps: two captured 48-half-step graphs and four enqueued
    launches in a staged variant, bit for bit against variant 0 run the
    same way, on a mesh whose block ranges end inside 64-cell groups."""
    N = 20011
    q0, _ = inputs.euler_riemann(5, 3, N)
    q, info = run_gpu("euler", 3, N, "transmissive", q0, 100, 0.25, variant=variant, threads=192, blocks=37,
                      precision=precision)
    r, rinfo = run_gpu("euler", 3, N, "transmissive", q0, 100, 0.25, variant=0, threads=192, blocks=37,
                       precision=precision)
    assert info.half_steps == 100 and info.t == rinfo.t and info.parity == rinfo.parity
    assert np.array_equal(q, r)


@pytest.mark.parametrize("mode", [4, 6])
def test_batch_periodic_staged(mode):
    """Periodic instances (N cells on both meshes), 30 half-steps (one graph
    chunk + 6 launches): staged schedules against the grouped direct one and
    an instance of every degree against its single-instance run."""
    spec = inputs.batch_spec(9, 15, n_lo=40, n_hi=1200)
    spec.N[:3] = [2, 63, 65]
    qs = [inputs.euler_riemann(int(spec.seeds[b]), int(spec.P[b]), int(spec.N[b]), bc="periodic")[0]
          for b in range(spec.P.size)]
    cfl = [0.4, 0.4, 0.3, 0.25, 0.25]

    def run(m):
        bt = binding.Batch("euler", spec.P, spec.N, "periodic", limiter=True, precision="fp64")
        try:
            bt.set_schedule(256, 0, m)
            for b, q in enumerate(qs):
                bt.write(b, q)
            bt.prepare()
            bt.run(30, cfl)
            return [bt.read(b) for b in range(spec.P.size)]
        finally:
            bt.close()

    got, ref = run(mode), run(2)
    for b in range(spec.P.size):
        assert got[b][1].t == ref[b][1].t and np.array_equal(got[b][0], ref[b][0]), b
    for P in (1, 2, 3):
        b = int(np.flatnonzero(spec.P == P)[0])
        s = binding.Solver("euler", P, int(spec.N[b]), "periodic", limiter=True, precision="fp64")
        try:
            s.write(qs[b])
            s.run(30, cfl[P])
            q1, i1 = s.read()
        finally:
            s.close()
        assert i1.t == got[b][1].t and np.array_equal(q1, got[b][0]), f"instance {b} vs single"
