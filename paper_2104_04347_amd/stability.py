"""Linear stability of the WCC half-step for any degree P (Section 2.3).

For linear advection u_t + a u_x = 0 the unlimited half-step is linear in
the DOF vector q = [u, u_x, ..., u_Px] of the two parents (Eq.
1DSchemeMatrixForm):

    q_{i+1/2}^{n+1/2} = M1 q_i^n + M2 q_{i+1}^n,

with M1, M2 polynomials in nu = a dt / dx (dt the half-step).  A Fourier
mode exp(i theta x/dx) is multiplied per half-step by the amplification
matrix G(theta) = M1 exp(-i theta/2) + M2 exp(i theta/2) (Eq.
1DFourierAnalysis); the scheme is stable when the spectral radius of G stays
at most 1 for every theta.  Table 2 of the paper gives the resulting CFL
intervals for P = 1, 2, 3; this module extends the analysis to P = 4.

The matrices are read off the GPU half-step itself (FP64, limiter off,
periodic): one state holds the P+1 unit vectors in cells 4r + 1, far enough
apart that their responses do not overlap, and one half-step with a fixed
dt returns every column of M1 and M2.  Only the spectral analysis runs on
the host (numpy eigenvalues).

    python -m paper_2104_04347_amd.stability --P 4
"""
from __future__ import annotations

import argparse

import numpy as np


def matrices_from_gpu(P: int, nu: float):
    """(M1, M2) of the unlimited degree-P half-step at CFL nu, from the GPU path."""
    from . import binding
    N = 4 * (P + 1) + 4
    s = binding.Solver("advection", P, N, "periodic", limiter=False, precision="fp64",
                       x_left=0.0, x_right=1.0, a=1.0)
    try:
        q = np.zeros((1, P + 1, N))
        for r in range(P + 1):
            q[0, r, 4 * r + 1] = 1.0
        s.write(q)
        s.step(dt_fixed=nu * (1.0 / N))
        qn, _ = s.read()
    finally:
        s.close()
    M1 = np.zeros((P + 1, P + 1))
    M2 = np.zeros((P + 1, P + 1))
    for r in range(P + 1):
        i = 4 * r + 1
        M1[:, r] = qn[0, :, i]        # new cell i: left parent is old cell i
        M2[:, r] = qn[0, :, i - 1]    # new cell i-1: right parent is old cell i
    return M1, M2


def spectral_radius(M1: np.ndarray, M2: np.ndarray, n_theta: int = 1440) -> float:
    """max over theta in (0, 2 pi] of the spectral radius of G(theta)."""
    th = np.linspace(0.0, 2.0 * np.pi, n_theta + 1)[1:]
    G = (M1[None, :, :] * np.exp(-0.5j * th)[:, None, None] + M2[None, :, :] * np.exp(0.5j * th)[:, None, None])
    return float(np.max(np.abs(np.linalg.eigvals(G))))


def stability_limit(P: int, tol: float = 1e-9, matrices=matrices_from_gpu, lo: float = 0.0, hi: float = 1.0,
                    iters: int = 40, n_theta: int = 1440) -> float:
    """Largest nu in [lo, hi] with spectral radius <= 1 + tol, by bisection
    (the stable set is an interval [0, nu*] for these schemes)."""
    def stable(nu):
        return spectral_radius(*matrices(P, nu), n_theta=n_theta) <= 1.0 + tol
    if stable(hi):
        return hi
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if stable(mid):
            lo = mid
        else:
            hi = mid
    return lo


def main(argv=None) -> None:
    ap = argparse.ArgumentParser(description="CFL limit of the unlimited WCC half-step (linear advection)")
    ap.add_argument("--P", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--tol", type=float, nargs="+", default=[1e-9, 2e-4],
                    help="tolerances on the spectral radius (strict, and the one matching Table 2)")
    a = ap.parse_args(argv)
    for P in a.P:
        vals = ", ".join(f"tol {t:g}: {stability_limit(P, t):.4f}" for t in a.tol)
        print(f"P={P}: nu_max ({vals})", flush=True)


if __name__ == "__main__":
    main()
