"""GPU parity: the gfx950 half-step kernels (through the C ABI) against the FP64
CPU oracle on the same seeded inputs.

Bar (binary64 mode): bit-identical states, time, mesh parity and half-step
counts.  The FP32-mixed mode is compared against the FP64 oracle with the
tolerances written in each test.
"""
import numpy as np
import pytest

import exact
import oracle
from paper_2104_04347_amd import binding, inputs

pytestmark = pytest.mark.gpu


def gpu_run(eq, P, N, bc, q0, *, limiter, t_end=None, cfl=0.25, steps=None, precision="fp64", launch=None, **kw):
    s = binding.Solver(eq, P, N, bc, limiter=limiter, precision=precision, **kw)
    if launch is not None:
        s.set_launch(*launch)
    s.write(q0)
    if t_end is not None:
        taken = s.advance(t_end, cfl)
    else:
        s.run(steps, cfl)
        taken = steps
    q, info = s.read()
    s.close()
    return q, info, taken


def oracle_run(eq, P, N, bc, q0, *, limiter, t_end=None, cfl=0.25, steps=None, **kw):
    pb = oracle.Problem(eq, P, N, bc=bc, limiter=limiter, **kw)
    if t_end is not None:
        return oracle.run(pb, q0, t_end=t_end, cfl=cfl)
    return oracle.run(pb, q0, cfl=cfl, max_half_steps=steps)


def assert_bitwise(q, info, taken, ref, label=""):
    assert info.flags & 3 == 0 and ref.flags == 0, (label, info.flags, ref.flags)
    assert taken == ref.half_steps, (label, taken, ref.half_steps)
    assert info.parity == ref.parity and info.t == ref.t, (label, info.parity, ref.parity, info.t, ref.t)
    assert q.shape == ref.q.shape, (label, q.shape, ref.q.shape)
    if not np.array_equal(q, ref.q):
        bad = np.argwhere(q != ref.q)
        c, k, j = bad[0]
        raise AssertionError(f"{label}: {len(bad)} of {q.size} values differ; first at c={c} k={k} j={j}: "
                             f"gpu {q[c, k, j]!r} oracle {ref.q[c, k, j]!r}")


def scalar_data(eq, P, N, seed=0):
    if eq == "advection":
        q, _ = inputs.sine_wave(P, N, 0.0, 1.0, c0=1.0, amp=0.2, w=2 * np.pi)
        return q, dict(x_left=0.0, x_right=1.0, a=1.0)
    q, _ = inputs.burgers_modes(seed, P, N)
    return q, dict(x_left=0.0, x_right=2.0)


@pytest.mark.parametrize("eq", ["advection", "burgers"])
@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("lim", [False, True])
def test_scalar_periodic_bitwise(eq, P, lim):
    N = 1000  # 15 full wave tiles and a ragged one
    q0, kw = scalar_data(eq, P, N)
    t_end = 0.15 if eq == "advection" else 0.6   # Burgers: past the first shock for seed 0
    q, info, taken = gpu_run(eq, P, N, "periodic", q0, limiter=lim, t_end=t_end, cfl=0.3, **kw)
    ref = oracle_run(eq, P, N, "periodic", q0, limiter=lim, t_end=t_end, cfl=0.3, **kw)
    assert_bitwise(q, info, taken, ref, f"{eq} P={P} lim={lim}")


@pytest.mark.parametrize("P", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("lim", [False, True])
def test_euler_transmissive_bitwise(P, lim):
    N = 500
    q0, _ = inputs.euler_riemann(3, P, N)
    q, info, taken = gpu_run("euler", P, N, "transmissive", q0, limiter=lim, t_end=0.12, cfl=0.25)
    ref = oracle_run("euler", P, N, "transmissive", q0, limiter=lim, t_end=0.12, cfl=0.25)
    assert_bitwise(q, info, taken, ref, f"euler P={P} lim={lim}")


@pytest.mark.parametrize("P", [1, 3, 4])
def test_euler_periodic_multijump_bitwise(P):
    N = 700
    q0, _ = inputs.euler_multi_jump(5, P, N, n_jumps=8, bc="periodic")
    q, info, taken = gpu_run("euler", P, N, "periodic", q0, limiter=True, t_end=0.05, cfl=0.2)
    ref = oracle_run("euler", P, N, "periodic", q0, limiter=True, t_end=0.05, cfl=0.2)
    assert_bitwise(q, info, taken, ref, f"euler periodic P={P}")


@pytest.mark.parametrize("P", [1, 2, 3])
def test_dirichlet_bitwise(P):
    N = 300
    q0, kw = scalar_data("burgers", P, N)
    # non-periodic mesh: N+1 cells on the original mesh
    x = inputs.centers(0.0, 2.0, N, N + 1, 0)
    _, fn = inputs.burgers_modes(0, P, N)
    q0 = np.stack([(2.0 / N) ** k * fn.deriv(x, k) for k in range(P + 1)])[None]
    kw.update(left_state=(0.9, 0, 0), right_state=(0.2, 0, 0))
    q, info, taken = gpu_run("burgers", P, N, "dirichlet", q0, limiter=True, t_end=0.3, cfl=0.3, **kw)
    ref = oracle_run("burgers", P, N, "dirichlet", q0, limiter=True, t_end=0.3, cfl=0.3, **kw)
    assert_bitwise(q, info, taken, ref, f"dirichlet P={P}")


@pytest.mark.parametrize("N", [2, 3, 62, 63, 64, 65, 125, 126, 127, 189, 190])
@pytest.mark.parametrize("case", ["euler-T", "adv-P"])
def test_tile_edges(N, case):
    if case == "euler-T":
        q0, _ = inputs.euler_riemann(1, 2, N)
        args = ("euler", 2, N, "transmissive")
        kw = {}
    else:
        q0, kw = scalar_data("advection", 3, N)
        args = ("advection", 3, N, "periodic")
    q, info, taken = gpu_run(*args, q0, limiter=True, steps=9, cfl=0.2, **kw)
    ref = oracle_run(*args, q0, limiter=True, steps=9, cfl=0.2, **kw)
    assert_bitwise(q, info, taken, ref, f"{case} N={N}")


def test_step_by_step_euler():
    """Every half-step of a limited Euler run, read back one at a time."""
    P, N = 3, 300
    q0, _ = inputs.euler_riemann(7, P, N)
    s = binding.Solver("euler", P, N, "transmissive", limiter=True)
    s.write(q0)
    pb = oracle.Problem("euler", P, N, bc="transmissive", limiter=True)
    ref = oracle.RunResult(q0, 0, 0.0, oracle.max_speed(pb, 0, q0), 0, 0)
    for n in range(12):
        s.step(0.25)
        q, info = s.read()
        ref = oracle.run(pb, ref.q, parity=ref.parity, t=ref.t, cfl=0.25, max_half_steps=1, smax=ref.smax)
        assert info.t == ref.t and info.parity == ref.parity
        assert np.array_equal(q, ref.q), f"half-step {n}"


@pytest.mark.parametrize("P", [1, 2, 3])
def test_fixed_dt_linear(P):
    """Fixed time step (the Appendix A setting: nu = a dt/dx)."""
    N = 130
    q0, kw = scalar_data("advection", P, N)
    dt = 0.2371 / N
    s = binding.Solver("advection", P, N, "periodic", limiter=False, **kw)
    s.write(q0)
    for _ in range(7):
        s.step(0.0, dt)
    q, info = s.read()
    ref = oracle.run(oracle.Problem("advection", P, N, limiter=False, **kw), q0, dt_fixed=dt, max_half_steps=7)
    assert info.t == ref.t and np.array_equal(q, ref.q)


def test_c1_advection_full():
    """u_t + u_x = 0, u0 = 1 + 0.2 sin(pi x) on [0, 2], P = 2, N = 200, t = 2,
    CFL 0.25 per half-step, limiter off: bitwise over the whole run, and the
    error against the exact shift is the third-order one."""
    P, N = 2, 200
    q0, fn = inputs.sine_wave(P, N, 0.0, 2.0, c0=1.0, amp=0.2)
    kw = dict(x_left=0.0, x_right=2.0, a=1.0)
    q, info, taken = gpu_run("advection", P, N, "periodic", q0, limiter=False, t_end=2.0, cfl=0.25, **kw)
    ref = oracle_run("advection", P, N, "periodic", q0, limiter=False, t_end=2.0, cfl=0.25, **kw)
    assert_bitwise(q, info, taken, ref, "advection N=200 t=2")
    x = inputs.centers(0.0, 2.0, N, N, info.parity)
    assert np.abs(q[0, 0] - fn(x - 2.0)).mean() < 2e-6


def test_c2_burgers_full_size():
    """Burgers, three seeded sine modes on [0, 2], P = 3, N = 12800, limiter on:
    bitwise for 1500 half-steps."""
    P, N = 3, 12800
    q0, _ = inputs.burgers_modes(0, P, N)
    kw = dict(x_left=0.0, x_right=2.0)
    q, info, taken = gpu_run("burgers", P, N, "periodic", q0, limiter=True, steps=1500, cfl=0.25, **kw)
    ref = oracle_run("burgers", P, N, "periodic", q0, limiter=True, steps=1500, cfl=0.25, **kw)
    assert_bitwise(q, info, taken, ref, "Burgers N=12800")


_C3_REF = {}


def _c3_reference(P, steps):
    if (P, steps) not in _C3_REF:
        q0, _ = inputs.euler_riemann(0, P, 1 << 20)
        _C3_REF[(P, steps)] = (q0, oracle_run("euler", P, 1 << 20, "transmissive", q0, limiter=True, steps=steps,
                                              cfl=0.25))
    return _C3_REF[(P, steps)]


# every launch shape the benchmark's autotuner can pick at this size: kernel
# variant (bit 1 prefetch, bit 2 staged stores), threads per block and grid
# (0 = device-filling default)
C3_SHAPES = [(256, 0, v) for v in (0, 1, 2, 3)] + [(256, 768, 0), (256, 768, 1), (128, 1536, 3), (64, 0, 1)]


@pytest.mark.parametrize("P", [2, 3])
@pytest.mark.parametrize("shape", C3_SHAPES, ids=lambda s: f"t{s[0]}b{s[1]}v{s[2]}")
def test_c3_euler_full_size(P, shape):
    """1D Euler at the benchmark size N = 1,048,576, seeded Riemann data with
    the density sine, transmissive, limiter on, FP64: bitwise for 6 half-steps
    (graph-replayed wcc_run) in each launch shape the benchmark may time."""
    N = 1 << 20
    q0, ref = _c3_reference(P, 6)
    q, info, taken = gpu_run("euler", P, N, "transmissive", q0, limiter=True, steps=6, cfl=0.25, launch=shape)
    assert_bitwise(q, info, taken, ref, f"Euler N=2^20 P={P} launch {shape}")


@pytest.mark.parametrize("P", [2, 3])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_c3_mixed_full_size_vs_oracle(P, variant):
    """FP32-mixed at the benchmark size against the FP64 oracle after n = 6
    half-steps, in each kernel variant, with the tolerances of MIXED_LINF_C
    (Linf within n C u32 S) and the mean within 4 sqrt(n) u32 S."""
    n, N = 6, 1 << 20
    q0, ref = _c3_reference(P, n)
    q, info, taken = gpu_run("euler", P, N, "transmissive", q0, limiter=True, steps=n, cfl=0.25,
                             precision="fp32_mixed", launch=(256, 0, variant))
    assert info.flags & 3 == 0 and info.parity == ref.parity
    assert abs(info.t - ref.t) <= n * U32 * ref.t
    for c in range(3):
        S = np.abs(ref.q[c, 0]).max()
        err = np.abs(q[c, 0] - ref.q[c, 0])
        print(f"C3 mixed P={P} v{variant} c={c}: Linf/S {err.max() / S:.3e} L1/S {err.mean() / S:.3e}", flush=True)
        assert err.max() <= n * MIXED_LINF_C * U32 * S, (c, err.max() / S)
        assert err.mean() <= 4 * np.sqrt(n) * U32 * S, (c, err.mean() / S)


def test_graph_replay_equals_single_steps():
    P, N = 3, 2000
    q0, _ = inputs.euler_riemann(2, P, N)
    a = binding.Solver("euler", P, N, "transmissive", limiter=True)
    a.write(q0)
    a.run(100, 0.25)   # two 48-step graphs and 4 single launches
    qa, ia = a.read()
    b = binding.Solver("euler", P, N, "transmissive", limiter=True)
    b.write(q0)
    for _ in range(100):
        b.step(0.25)
    qb, ib = b.read()
    assert ia.t == ib.t and np.array_equal(qa, qb)
    # graphs are replayed: run again from the same state
    a.write(q0)
    a.run(100, 0.25)
    qc, _ = a.read()
    assert np.array_equal(qa, qc)


def test_determinism_repeat():
    P, N = 3, 100000
    q0, _ = inputs.euler_riemann(4, P, N)
    outs = []
    for prec in ("fp64", "fp32_mixed", "fp64", "fp32_mixed"):
        s = binding.Solver("euler", P, N, "transmissive", limiter=True, precision=prec)
        s.write(q0)
        s.run(200, 0.25)
        outs.append(s.read()[0])
    assert np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[1], outs[3])


U32 = 2.0 ** -24   # binary32 unit round-off
# Linf tolerance of the FP32-mixed mode against the FP64 oracle, from the
# arithmetic: one half-step perturbs a new DOF by at most C u32 S (S the
# field's scale), C bounding the binary32 roundings along the longest
# dependent chain from the stored DOFs to a new DOF -- for Euler at P = 3
# about 60 in the expansion (Taylor products and the series quotient, four
# time levels) and about 50 in the characteristic limiter (projection,
# indicator, sigma and tau, ratio, square, normalisation, back-projection):
# C = 128.  The perturbations pass through the scheme without growth (a
# stable step; the limited polynomial is a convex combination of candidates
# with weights of bounded sensitivity), so after n half-steps they add up to
# at most n C u32 S.  Where the rounding errors are independent (everywhere
# but at the few cells of a jump) the mean error grows like their random
# walk: within 4 sqrt(n) u32 S.
MIXED_LINF_C = 128


@pytest.mark.parametrize("P", [1, 2, 3, 4])
def test_mixed_precision_smooth(P):
    """FP32-mixed on smooth Euler data (entropy wave, limiter on) against the
    FP64 oracle after n = 400 half-steps.

    Tolerance from the arithmetic: every half-step rounds the binary32 flux
    integral and the binary32 vertex values once relative to the state scale S
    (the scaled derivatives are differences of O(S) vertex values, so their
    error is absolute in S, not relative to their own O(dx^k) size); the
    rounding errors accumulate at most linearly, so every DOF must stay within
    n * u32 * S and the mean point-value error within 4 sqrt(n) u32 S."""
    N, n = 2000, 400
    q0, _ = inputs.euler_entropy_wave(P, N)
    kw = dict(x_left=0.0, x_right=2.0)
    q, info, taken = gpu_run("euler", P, N, "periodic", q0, limiter=True, steps=n, cfl=0.25,
                             precision="fp32_mixed", **kw)
    ref = oracle_run("euler", P, N, "periodic", q0, limiter=True, steps=n, cfl=0.25, **kw)
    assert taken == ref.half_steps and info.parity == ref.parity
    assert abs(info.t - ref.t) <= n * U32 * ref.t
    for c in range(3):
        S = np.abs(ref.q[c, 0]).max()
        err = np.abs(q[c] - ref.q[c])
        assert err.max() <= n * U32 * S, (c, err.max() / S)
        assert err[0].mean() <= 4 * np.sqrt(n) * U32 * S, (c, err[0].mean() / S)


@pytest.mark.parametrize("P", [2, 3])
def test_mixed_precision_riemann(P):
    """FP32-mixed on a seeded Riemann problem (limiter active at the waves)
    against the FP64 oracle after n = 300 half-steps: density Linf within
    n C u32 S and mean within 4 sqrt(n) u32 S (MIXED_LINF_C)."""
    N = 4000
    q0, _ = inputs.euler_riemann(0, P, N)
    q, info, taken = gpu_run("euler", P, N, "transmissive", q0, limiter=True, steps=300, cfl=0.25,
                             precision="fp32_mixed")
    ref = oracle_run("euler", P, N, "transmissive", q0, limiter=True, steps=300, cfl=0.25)
    scale = np.abs(ref.q[0, 0]).max()
    err = np.abs(q[0, 0] - ref.q[0, 0])
    print(f"Riemann mixed P={P}: Linf/S {err.max() / scale:.3e} L1/S {err.mean() / scale:.3e}", flush=True)
    n = 300
    assert err.mean() <= 4 * np.sqrt(n) * U32 * scale, err.mean() / scale
    assert err.max() <= n * MIXED_LINF_C * U32 * scale, err.max() / scale


def test_mixed_conservation_periodic():
    """FP32-mixed keeps the binary64 average accumulation: the conserved
    totals drift only at binary64 round-off over 2000 half-steps."""
    P, N = 3, 20000
    q0, _ = inputs.euler_multi_jump(9, P, N, n_jumps=8, bc="periodic")
    s = binding.Solver("euler", P, N, "periodic", limiter=True, precision="fp32_mixed")
    s.write(q0)
    tot0 = s.totals()
    s.run(2000, 0.2)
    tot = s.totals()
    q, info = s.read()
    assert info.flags & 3 == 0
    # sum of |average| bounds the round-off of the total
    avg_abs = np.abs(q[:, 0]).sum(axis=1) * info.dx
    assert np.all(np.abs(tot - tot0) <= 200 * 2.2e-16 * avg_abs * np.sqrt(2000)), (tot - tot0, avg_abs)


def _batch_case(seed=3, B=10):
    spec = inputs.batch_spec(B, seed, n_lo=40, n_hi=3000)
    return spec, [inputs.batch_instance(spec, b) for b in range(B)]


@pytest.mark.parametrize("precision", ["fp64", "fp32_mixed"])
@pytest.mark.parametrize("mode", [1, 2])
def test_batch_equals_single(precision, mode):
    """Batched persistent kernels reproduce single-instance runs bit for bit
    (same arithmetic, different scheduling), for both schedules."""
    spec, qs = _batch_case()
    cfl = [0.4, 0.4, 0.3, 0.25, 0.25]
    bt = binding.Batch("euler", spec.P, spec.N, "transmissive", limiter=True, precision=precision)
    bt.set_schedule(256, 0, mode)
    for b, q in enumerate(qs):
        bt.write(b, q)
    bt.prepare()
    bt.run(30, cfl)
    for b, q in enumerate(qs):
        qb, ib = bt.read(b)
        P, N = int(spec.P[b]), int(spec.N[b])
        s = binding.Solver("euler", P, N, "transmissive", limiter=True, precision=precision)
        s.write(q)
        s.run(30, cfl[P])
        qs_, is_ = s.read()
        assert ib.t == is_.t and ib.half_steps == 30, (b, ib.t, is_.t)
        assert np.array_equal(qb, qs_), f"instance {b} (P={P}, N={N})"


def test_batch_fp64_matches_oracle():
    spec, qs = _batch_case(seed=8, B=6)
    cfl = [0.4, 0.4, 0.3, 0.25, 0.25]
    bt = binding.Batch("euler", spec.P, spec.N, "transmissive", limiter=True, precision="fp64")
    for b, q in enumerate(qs):
        bt.write(b, q)
    bt.prepare()
    bt.run(25, cfl)
    for b, q in enumerate(qs):
        qb, ib = bt.read(b)
        P, N = int(spec.P[b]), int(spec.N[b])
        ref = oracle.run(oracle.Problem("euler", P, N, bc="transmissive", limiter=True), q, cfl=cfl[P],
                         max_half_steps=25)
        assert ib.t == ref.t and np.array_equal(qb, ref.q), b


def test_error_paths():
    s = binding.Solver("euler", 2, 64, "transmissive")
    with pytest.raises(binding.WccError) as e:
        s.step(0.25)
    assert e.value.code == binding.WCC_ESTATE
    q0, _ = inputs.euler_riemann(0, 2, 64)
    bad = q0.copy()
    bad[0, 0, 10] = np.nan
    with pytest.raises(binding.WccError) as e:
        s.write(bad)
    assert e.value.code == binding.WCC_ENONFINITE
    short = np.ascontiguousarray(q0[:, :, :10])
    rc = binding.load().wcc_write_dofs(s.h, binding._dptr(short), 10, 0, 0.0)
    assert rc == binding.WCC_ESIZE
    s.write(q0)
    with pytest.raises(binding.WccError) as e:
        s.step(1.5)
    assert e.value.code == binding.WCC_EINVAL
    with pytest.raises(binding.WccError) as e:
        s.advance(-1.0, 0.25)
    assert e.value.code == binding.WCC_EINVAL


def test_blowup_is_flagged_and_kept():
    """An unstable fixed time step drives Burgers to overflow; the run stops at
    the flagged step, keeps that state and refuses to go on."""
    P, N = 2, 256
    q0, kw = scalar_data("burgers", P, N)
    s = binding.Solver("burgers", P, N, "periodic", limiter=False, **kw)
    s.write(q0)
    for _ in range(400):
        s.step(0.0, 40.0 * (2.0 / N))
    q, info = s.read()
    assert info.flags & 1
    n_done = info.half_steps
    s.step(0.0, 40.0 * (2.0 / N))
    _, info2 = s.read()
    assert info2.half_steps == n_done and info2.flags & 1
    with pytest.raises(binding.WccError) as e:
        s.advance(1e9, 0.3)
    assert e.value.code == binding.WCC_ENONFINITE


def test_context_managers_release_the_workspace():
    """`with` blocks destroy the contexts and drop their device workspaces."""
    q0, kw = scalar_data("advection", 2, 64)
    with binding.Solver("advection", 2, 64, "periodic", limiter=False, **kw) as s:
        s.write(q0)
        s.run(4, 0.25)
        q, info = s.read()
    assert s.h is None and s.workspace is None and info.half_steps == 4
    s.close()                                  # idempotent
    spec = inputs.batch_spec(3, 1, n_lo=40, n_hi=100)
    with binding.Batch("euler", spec.P, spec.N, "transmissive", limiter=True) as bt:
        bt.write(0, inputs.batch_instance(spec, 0))
    assert bt.h is None and bt.workspace is None
    with binding.Solver2D("burgers", 1, 8, 8, limiter=True) as s2:
        pass
    assert s2.h is None and s2.workspace is None


def test_degenerate_calls():
    """Zero half-steps leave the state, time and parity as written; an
    advance to the current time takes no step; the smallest mesh (N = 2)
    runs in every boundary condition."""
    P, N = 2, 300
    q0, _ = inputs.euler_riemann(6, P, N)
    s = binding.Solver("euler", P, N, "transmissive", limiter=True)
    s.write(q0, t=0.125)
    s.run(0, 0.25)
    q, info = s.read()
    assert np.array_equal(q, q0) and info.t == 0.125 and info.parity == 0 and info.half_steps == 0
    assert s.advance(0.125, 0.25) == 0
    q, info = s.read()
    assert np.array_equal(q, q0) and info.t == 0.125
    s.close()
    for bc in ("periodic", "transmissive", "dirichlet"):
        kw = dict(x_left=0.0, x_right=2.0)
        n0 = 2 if bc == "periodic" else 3
        q0 = np.full((1, 2, n0), 0.4)
        q0[0, 1] = 0.0
        kw.update(left_state=(0.4, 0, 0), right_state=(0.4, 0, 0))
        q, info, taken = gpu_run("burgers", 1, 2, bc, q0, limiter=True, steps=5, cfl=0.3, **kw)
        ref = oracle_run("burgers", 1, 2, bc, q0, limiter=True, steps=5, cfl=0.3, **kw)
        assert_bitwise(q, info, taken, ref, f"N=2 {bc}")


def test_batch_single_instance_and_degree_zero():
    """A batch of one instance, and instances of degree 0, equal
    single-instance runs bit for bit."""
    for P_list, N_list in (([3], [1000]), ([0, 1, 0], [300, 65, 2])):
        P = np.array(P_list, dtype=np.int32)
        N = np.array(N_list, dtype=np.int64)
        bt = binding.Batch("euler", P, N, "transmissive", limiter=True, precision="fp64")
        qs = [inputs.euler_riemann(10 + b, int(P[b]), int(N[b]))[0] for b in range(P.size)]
        for b in range(P.size):
            bt.write(b, qs[b])
        bt.prepare()
        bt.advance(13, [0.4, 0.4, 0.3, 0.25, 0.25])
        for b in range(P.size):
            qb, ib = bt.read(b)
            q, info, _ = gpu_run("euler", int(P[b]), int(N[b]), "transmissive", qs[b], limiter=True, steps=13,
                                 cfl=[0.4, 0.4, 0.3, 0.25, 0.25][int(P[b])])
            assert ib.t == info.t and np.array_equal(qb, q), (P_list, b)
        bt.close()
