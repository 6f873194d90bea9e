"""GPU parity at the full sizes of the benchmarked workloads, in the launch
configurations the benchmark times:

* the large 1D Euler run: N = 16,777,216, P = 4, eight seeded jumps with the
  density sine, periodic, CFL 0.20 per half-step -- binary64 bit for bit
  against the FP64 oracle over two half-steps (both mesh parities), and the
  FP32-mixed mode against the same oracle result within the stated
  tolerance, with its conserved totals at binary64 round-off; with direct
  and with staged stores (the autotuner picks staged at this size);
* the batched workload: 4096 instances, N log-uniform in [256, 65536],
  P in {1, 2, 3} -- sampled instances (the smallest, the largest, every
  degree) of the FP32-mixed batch bit for bit against single-instance runs,
  and of a binary64 batch bit for bit against the oracle, in every schedule
  (fused / grouped, direct / staged stores, degrees in sequence or as
  parallel graph branches);
* the 2D legs: Burgers with the limiter on 2048 x 2048, the Euler vortex on
  1024 x 1024 unlimited and limited, and the first 2D Riemann problem on
  1200 x 1200 intervals with transmissive edges (P = 3), bit for bit against
  the 2D oracle over two half-steps.
"""
import numpy as np
import pytest

import oracle
from paper_2104_04347_amd import binding, inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
CFL_BY_P = [0.4, 0.4, 0.3, 0.25, 0.25]


def _bitwise(q, info, ref, label):
    print(label, flush=True)
    assert info.flags & 3 == 0 and ref.flags == 0, (label, info.flags, ref.flags)
    assert info.parity == ref.parity and info.t == ref.t, (label, info.t, ref.t)
    if not np.array_equal(q, ref.q):
        bad = np.argwhere(q != ref.q)
        raise AssertionError(f"{label}: {len(bad)} of {q.size} values differ; first at {tuple(bad[0])}")


# ---------------------------------------------------------------------------
# Large 1D Euler, N = 2^24, P = 4
# ---------------------------------------------------------------------------
LARGE_N, LARGE_P, LARGE_CFL, LARGE_STEPS = 1 << 24, 4, 0.20, 2


@pytest.fixture(scope="module")
def large_case():
    q0, _ = inputs.euler_multi_jump(0, LARGE_P, LARGE_N, n_jumps=8, bc="periodic")
    print("large: oracle, 2 half-steps", flush=True)
    pb = oracle.Problem("euler", LARGE_P, LARGE_N, bc="periodic", limiter=True)
    ref = oracle.run(pb, q0, cfl=LARGE_CFL, max_half_steps=LARGE_STEPS)
    return q0, ref


def _large_gpu(q0, precision, variant=0):
    s = binding.Solver("euler", LARGE_P, LARGE_N, "periodic", limiter=True, precision=precision)
    try:
        s.set_launch(0, 0, variant)
        s.write(q0)
        tot0 = s.totals()
        s.run(LARGE_STEPS, LARGE_CFL)
        tot = s.totals()
        q, info = s.read()
    finally:
        s.close()
    return q, info, tot0, tot


# launch variants: 0 direct stores, 2 staged stores, 3 staged + prefetch (the
# autotuner's choice at this size)
@pytest.mark.timeout(600)
@pytest.mark.parametrize("variant", [0, 2, 3])
def test_large_fp64_bitwise(large_case, variant):
    q0, ref = large_case
    q, info, _, _ = _large_gpu(q0, "fp64", variant)
    assert info.half_steps == LARGE_STEPS
    _bitwise(q, info, ref, f"large fp64 variant {variant}")


@pytest.mark.timeout(600)
@pytest.mark.parametrize("variant", [0, 3])
def test_large_mixed_within_tolerance(large_case, variant):
    """Two half-steps in FP32-mixed against the FP64 oracle: point-value L1
    within 4 sqrt(n) u32 S, Linf within n C u32 S with C = 128 (the bound on
    binary32 roundings along the longest dependent chain to a new DOF, as in
    test_gpu_parity.MIXED_LINF_C), conserved totals within the round-off of
    their own binary64 evaluation."""
    q0, ref = large_case
    q, info, tot0, tot = _large_gpu(q0, "fp32_mixed", variant)
    print(f"large mixed variant {variant}", flush=True)
    assert info.flags & 3 == 0 and info.parity == ref.parity
    n = LARGE_STEPS
    assert abs(info.t - ref.t) <= n * U32 * ref.t
    for c in range(3):
        S = np.abs(ref.q[c, 0]).max()
        err = np.abs(q[c, 0] - ref.q[c, 0])
        print(f"large mixed v{variant} c={c}: Linf/S {err.max() / S:.3e} L1/S {err.mean() / S:.3e}", flush=True)
        assert err.mean() <= 4 * np.sqrt(n) * U32 * S, (c, err.mean() / S)
        assert err.max() <= n * 128 * U32 * S, (c, err.max() / S)
    # the totals are sequential binary64 sums over N cells: each evaluation
    # carries round-off of about sqrt(N) u64 sum|u| (random-walk estimate, a
    # factor 4 above it allowed); binary32 averages would drift by ~1e-8
    avg_abs = np.abs(q[:, 0]).sum(axis=1) * info.dx
    bound = 2 * 4 * np.sqrt(LARGE_N) * 2.0 ** -53 * avg_abs
    assert np.all(np.abs(tot - tot0) <= bound), (tot - tot0, bound)


# ---------------------------------------------------------------------------
# Batched workload, 4096 instances
# ---------------------------------------------------------------------------
BATCH_B, BATCH_STEPS = 4096, 6


def _samples(spec):
    idx = {int(np.argmin(spec.N)), int(np.argmax(spec.N))}
    for P in (1, 2, 3):
        idx.add(int(np.flatnonzero(spec.P == P)[0]))
    return sorted(idx)


def _batch_run(spec, precision, mode):
    bt = binding.Batch("euler", spec.P, spec.N, "transmissive", limiter=True, precision=precision)
    try:
        for b in range(spec.P.size):
            bt.write(b, inputs.batch_instance(spec, b))
        bt.prepare()
        bt.set_schedule(256, 0, mode)
        bt.run(BATCH_STEPS, CFL_BY_P)
        out = {b: bt.read(b) for b in _samples(spec)}
    finally:
        bt.close()
    return out


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", [1, 2, 3, 4, 5, 6])   # fused / grouped, direct / staged, branches
def test_batch_full_mixed_equals_single(mode):
    spec = inputs.batch_spec(BATCH_B, 0)
    got = _batch_run(spec, "fp32_mixed", mode)
    for b, (qb, ib) in got.items():
        P, N = int(spec.P[b]), int(spec.N[b])
        print(f"batch mixed mode={mode} instance {b} P={P} N={N}", flush=True)
        s = binding.Solver("euler", P, N, "transmissive", limiter=True, precision="fp32_mixed")
        s.write(inputs.batch_instance(spec, b))
        s.run(BATCH_STEPS, CFL_BY_P[P])
        qs, is_ = s.read()
        s.close()
        assert ib.flags & 3 == 0 and ib.t == is_.t and ib.half_steps == BATCH_STEPS, (b, ib.t, is_.t)
        assert np.array_equal(qb, qs), f"instance {b} (P={P}, N={N})"


@pytest.mark.timeout(600)
@pytest.mark.parametrize("mode", [2, 4, 6])
def test_batch_full_fp64_matches_oracle(mode):
    spec = inputs.batch_spec(BATCH_B, 0)
    got = _batch_run(spec, "fp64", mode)
    for b, (qb, ib) in got.items():
        P, N = int(spec.P[b]), int(spec.N[b])
        ref = oracle.run(oracle.Problem("euler", P, N, bc="transmissive", limiter=True),
                         inputs.batch_instance(spec, b), cfl=CFL_BY_P[P], max_half_steps=BATCH_STEPS)
        _bitwise(qb, ib, ref, f"batch fp64 mode {mode} instance {b} P={P} N={N}")


# ---------------------------------------------------------------------------
# 2D legs
# ---------------------------------------------------------------------------
_REF2D = {}


# launch shapes the benchmark's autotuner may pick for these legs: row
# marching with prefetch (2) or with band-major items (3), on the
# device-filling grid (0) or one block per compute unit (256)
SHAPES_2D = [(256, 0, 2), (256, 256, 2), (256, 0, 3), (256, 256, 3)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("shape", SHAPES_2D, ids=lambda s: f"b{s[1]}v{s[2]}")
@pytest.mark.parametrize("case", ["burgers_lim_P3_2048", "euler_vortex_P3_1024", "euler_vortex_lim_P3_1024",
                                  "riemann2d_1_lim_P3_1200"])
def test_2d_bench_size_bitwise(case, shape):
    """Every 2D benchmark leg at its benchmark size, two half-steps, in each
    launch shape the benchmark may time."""
    P, lim, bc = 3, "_lim_" in case, "periodic"
    if case.startswith("burgers"):
        eq, N, dom = "burgers", 2048, (0.0, 2.0, 0.0, 2.0)
        q0 = inputs.taylor2d(inputs.modes2d(0), P, N, N)
    elif case.startswith("euler_vortex"):
        eq, N, dom = "euler", 1024, (-5.0, 5.0, -5.0, 5.0)
        q0 = inputs.isentropic_vortex(P, N)
    else:
        eq, N, dom, bc = "euler", 1200, (-1.0, 1.0, -1.0, 1.0), "transmissive"
        q0 = inputs.riemann2d(1, P, N)
    kw = dict(x_left=dom[0], x_right=dom[1], y_left=dom[2], y_right=dom[3])
    s = binding.Solver2D(eq, P, N, N, limiter=lim, bc=bc, **kw)
    try:
        s.set_launch(*shape)
        s.write(q0)
        s.run(2, 0.25)
        q, info = s.read()
    finally:
        s.close()
    if case not in _REF2D:
        print(f"{case}: oracle", flush=True)
        _REF2D[case] = oracle.run2d(oracle.Problem2D(eq, P, N, N, limiter=lim, bc=bc, **kw), q0, cfl=0.25,
                                    max_half_steps=2)
    _bitwise(q, info, _REF2D[case], f"{case} launch {shape}")
