"""GPU parity at the largest meshes the library accepts (32-bit cell and byte
offsets): 1D with N = 2^28 cells, 2D with (Nx+1) x (Ny+1) = 2^28 cells on
the transmissive mesh-point mesh; and 2D Euler on both sides of the 2 GiB
state size up to which the row kernels use 32-bit buffer offsets.  Seeded random states (the limiter acts
everywhere), one half-step; sampled windows of new cells are checked bit for
bit against the oracle run on the window's own old cells with the GPU's dt
(a new cell depends only on its parents and dt; the mesh widths are powers
of two, so a window's dx is the full mesh's dx exactly)."""
import numpy as np
import pytest

import oracle
from paper_2104_04347_amd import binding

pytestmark = pytest.mark.gpu


@pytest.mark.timeout(900)
@pytest.mark.parametrize("variant", [0, 3])      # direct stores; staged stores + prefetch
def test_1d_max_cells_burgers(variant):
    P, N = 3, 1 << 28
    dx = 2.0 ** -20
    rng = np.random.default_rng(21)
    q0 = np.empty((1, P + 1, N))
    q0[0, 0] = 0.5 + 0.3 * rng.random(N)
    for k in range(1, P + 1):
        q0[0, k] = (0.1 / k) * (rng.random(N) - 0.5)
    s = binding.Solver("burgers", P, N, "periodic", limiter=True, x_left=0.0, x_right=N * dx)
    try:
        s.set_launch(0, 0, variant)
        s.write(q0)
        s.step(0.25)
        q, info = s.read()
    finally:
        s.close()
    print(f"1D max, variant {variant}: GPU step done", flush=True)
    assert info.flags & 3 == 0 and info.parity == 1 and q.shape == (1, P + 1, N)
    dt = info.t
    W = 256
    starts = [0, 1 << 20, (1 << 27) + 12345, N - 2 * W] + list(rng.integers(0, N - W, 8))
    for a in starts:
        a = int(a)
        pb = oracle.Problem("burgers", P, W, bc="periodic", limiter=True, x_left=0.0, x_right=W * dx)
        r = oracle.run(pb, q0[:, :, a:a + W], dt_fixed=dt, max_half_steps=1)
        got = q[:, :, a:a + W - 1]
        assert np.array_equal(got, r.q[:, :, :W - 1]), f"window at {a}"
    # the last new cell wraps to the first old one
    pb = oracle.Problem("burgers", P, 2, bc="periodic", limiter=True, x_left=0.0, x_right=2 * dx)
    r = oracle.run(pb, np.concatenate([q0[:, :, N - 1:], q0[:, :, :1]], axis=2), dt_fixed=dt, max_half_steps=1)
    assert np.array_equal(q[:, :, N - 1], r.q[:, :, 0])


@pytest.mark.timeout(900)
def test_2d_max_cells_transmissive_burgers():
    P, Nx, Ny = 1, 16383, 16383            # (Nx+1) (Ny+1) = 2^28 cells on parity 0
    h = 2.0 ** -10
    rng = np.random.default_rng(22)
    q0 = np.empty((1, 3, Ny + 1, Nx + 1))
    q0[0, 0] = 0.5 + 0.3 * rng.random((Ny + 1, Nx + 1))
    q0[0, 1] = 0.05 * (rng.random((Ny + 1, Nx + 1)) - 0.5)
    q0[0, 2] = 0.05 * (rng.random((Ny + 1, Nx + 1)) - 0.5)
    s = binding.Solver2D("burgers", P, Nx, Ny, limiter=True, bc="transmissive", x_right=Nx * h, y_right=Ny * h)
    try:
        s.write(q0)
        s.step(cfl=0.25)
        q, info = s.read()
    finally:
        s.close()
    print("2D max: GPU step done", flush=True)
    assert info.flags & 3 == 0 and info.parity == 1 and q.shape == (1, 3, Ny, Nx)
    dt = info.t
    W = H = 48
    corners = [(0, 0), (Nx + 1 - W, Ny + 1 - H), (8191, 100), (1000, 16000 - H)]
    corners += [(int(rng.integers(0, Nx + 1 - W)), int(rng.integers(0, Ny + 1 - H))) for _ in range(6)]
    for a, b in corners:
        pb = oracle.Problem2D("burgers", P, W, H, limiter=True, x_right=W * h, y_right=H * h)
        r = oracle.run2d(pb, np.ascontiguousarray(q0[:, :, b:b + H, a:a + W]), dt_fixed=dt, max_half_steps=1)
        got = q[:, :, b:b + H - 1, a:a + W - 1]
        assert np.array_equal(got, r.q[:, :, :H - 1, :W - 1]), f"window at ({a}, {b})"


# The prefetching row kernels (variants 2 and 3) address the state through
# buffer resources with 32-bit offsets while one state buffer is below 2 GiB,
# and through 64-bit plane pointers above.  Limited Euler, P = 3 (40 planes):
# 2560^2 cells -> 40 x 6,553,600 x 8 B = 2.097e9 B, just below 2^31 (the last
# planes' offsets near the top of the 32-bit range); 2600^2 -> 2.163e9 B, the
# pointer form.
@pytest.mark.timeout(900)
@pytest.mark.parametrize("N,variant", [(2560, 3), (2560, 2), (2600, 3), (2600, 2)])
def test_2d_euler_at_the_buffer_offset_limit(N, variant):
    P = 3
    h = 2.0 ** -9
    rng = np.random.default_rng(23)
    q0 = np.empty((4, 10, N, N))
    rho = 1.0 + 0.2 * rng.random((N, N))
    u = 0.2 * (rng.random((N, N)) - 0.5)
    v = 0.2 * (rng.random((N, N)) - 0.5)
    p = 1.0 + 0.2 * rng.random((N, N))
    q0[0, 0] = rho
    q0[1, 0] = rho * u
    q0[2, 0] = rho * v
    q0[3, 0] = p / 0.4 + 0.5 * rho * (u * u + v * v)
    for c in range(4):
        for d in range(1, 10):
            q0[c, d] = (0.02 / d) * (rng.random((N, N)) - 0.5)
    del rho, u, v, p
    s = binding.Solver2D("euler", P, N, N, limiter=True, bc="periodic", x_right=N * h, y_right=N * h)
    try:
        s.set_launch(256, 0, variant)
        s.write(q0)
        s.step(cfl=0.25)
        q, info = s.read()
    finally:
        s.close()
    print(f"2D Euler {N}^2, variant {variant}: GPU step done", flush=True)
    assert info.flags & 3 == 0 and info.parity == 1 and q.shape == (4, 10, N, N)
    dt = info.t
    W = H = 40
    corners = [(0, 0), (N - W, N - H), (N // 2, 17), (5, N - H)]
    corners += [(int(rng.integers(0, N - W)), int(rng.integers(0, N - H))) for _ in range(4)]
    for a, b in corners:
        pb = oracle.Problem2D("euler", P, W, H, limiter=True, x_right=W * h, y_right=H * h)
        r = oracle.run2d(pb, np.ascontiguousarray(q0[:, :, b:b + H, a:a + W]), dt_fixed=dt, max_half_steps=1)
        got = q[:, :, b:b + H - 1, a:a + W - 1]
        assert np.array_equal(got, r.q[:, :, :H - 1, :W - 1]), f"window at ({a}, {b})"
