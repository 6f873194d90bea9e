"""GPU parity at the largest meshes the library accepts (32-bit cell and byte
offsets): 1D with N = 2^28 cells, 2D with (Nx+1) x (Ny+1) = 2^28 cells on
the transmissive mesh-point mesh.  Seeded random states (the limiter acts
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
