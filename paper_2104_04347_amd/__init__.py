"""MI355X (gfx950) implementation of the explicit half-step of the 1D weighted
compact central (WCC) schemes of Shen & Parsani (arXiv:2104.04347).

* ``binding``  -- ctypes binding of the C ABI (include/wcc.h) of libwcc.so and
                  the torch-backed ``Solver`` / ``Batch`` wrappers;
* ``inputs``   -- seeded synthetic initial data shaped like the paper's
                  workloads (problem data only);
* ``autotune`` -- launch-shape search for the single and batched kernels;
* ``build``    -- compiles csrc/*.hip for gfx950 into _lib/libwcc.so.
"""
__all__ = ["binding", "inputs", "build", "autotune"]
