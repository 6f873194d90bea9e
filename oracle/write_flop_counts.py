"""Write the per-cell operation counts of the half-step (the oracle's counting
real type, one old cell + one new cell per new cell) to
paper_2104_04347_amd/flop_counts.json, which the benchmark reads to price the
kernels against the vector-ALU roof.  Calls only the oracle.

Counting convention: add/sub, mul, div and sqrt count 1 flop, fma counts 2.
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(HERE), "paper_2104_04347_amd", "flop_counts.json")


def sample_cell(eq, P, rng):
    if eq == "euler":
        rho, u, p = rng.uniform(0.3, 1.0), rng.uniform(-0.5, 0.5), rng.uniform(0.3, 1.0)
        q = np.zeros((3, P + 1))
        q[:, 0] = [rho, rho * u, p / 0.4 + 0.5 * rho * u * u]
        q[:, 1:] = rng.uniform(-0.05, 0.05, (3, P))
        return q
    q = np.zeros((1, P + 1))
    q[0, 0] = rng.uniform(0.2, 1.0)
    q[0, 1:] = rng.uniform(-0.05, 0.05, P)
    return q


def main():
    rng = np.random.default_rng(0)
    out = {"_doc": __doc__.strip(), "counts": {}}
    for eq in ("advection", "burgers", "euler"):
        for P in range(5):
            for lim in (False, True):
                if P == 0 and lim:
                    continue
                pb = oracle.Problem(eq, P, 64, limiter=lim)
                c = oracle.count_flops(pb, sample_cell(eq, P, rng), sample_cell(eq, P, rng), 0.1)
                out["counts"][f"{eq}/P{P}/{'lim' if lim else 'nolim'}"] = c
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print(OUT)


if __name__ == "__main__":
    main()
