"""Write the stored expected values under tests/golden/ from the CPU oracle.

Calls only the oracle and the seeded input generators.  Run from the
repository root:

    python tests/golden/make_golden.py

Outputs
  cfg2_coeffs_qr.npy  least-squares coefficients of the D=6, |n|_1<=12
                      exp-cos workload (seed 1), by dense Householder QR of
                      the stacked system folded in grid by grid.
  cfg2_meta.json      grids, sizes, kappa estimate and the QR diagonal range.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402


def main():
    p = W.config2()
    t0 = time.time()
    samples = O.sample_problem(p)
    plan = O.build_plan(p.support, p.grids)
    trans = [O.dct_grid(samples[l], p.grids[l]) for l in range(p.K)]
    b = O.rhs_from_transforms(plan, trans)
    c, rdiag = O.lstsq_qr(plan, b)
    t1 = time.time()
    full, kappa = O.rank_check(plan)
    np.save(os.path.join(HERE, "cfg2_coeffs_qr.npy"), c)
    meta = {
        "workload": p.name, "seed": p.seed, "D": p.D, "n_support": p.n,
        "K": p.K, "grids": p.grids.tolist(), "points": p.points, "M": plan.M,
        "kappa_A": kappa, "full_rank": full,
        "qr_abs_diag_min": float(np.abs(rdiag).min()),
        "qr_abs_diag_max": float(np.abs(rdiag).max()),
        "qr_seconds": t1 - t0,
        "method": "sequential Householder QR of [A | b] (numpy.linalg.qr, mode='r')",
    }
    with open(os.path.join(HERE, "cfg2_meta.json"), "w") as fh:
        json.dump(meta, fh, indent=1)
    print(json.dumps(meta))


if __name__ == "__main__":
    main()
