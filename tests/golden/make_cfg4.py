"""Reference data of the precision-sweep workload (D=12, |n|_1 <= 10,
646,646 coefficients, Gaussian bump), computed once with the oracle.

1. Grid count (Alg. 2).  Grids are drawn by the workload's rule
   (workloads.config4, N_i ~ U{2..6}); the count is the smallest one at which
   the stacked system has full column rank.  It starts where every dimension's folds
   separate its degrees 0..10 (a necessary condition) and is decided by exact
   recovery: LSQR from zero returns a random coefficient vector c from
   b = A c exactly (max-relative 1e-10) only when A has full column rank.
2. The least-squares minimiser for the Gaussian bump on those grids: oracle
   samples, direct-sum DCT-I per grid, LSQR on the explicit sparse A run to
   its attainable accuracy.  Dense QR is out of reach at this size; the same
   route is pinned against dense QR on the d = 4 twin of the workload
   (tests/test_oracle_pins.py).

Writes tests/golden/cfg4_coeffs_lsqr.npy and tests/golden/cfg4_meta.json.
Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_cfg4.py
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

OUT_C = os.path.join(HERE, "cfg4_coeffs_lsqr.npy")
OUT_META = os.path.join(HERE, "cfg4_meta.json")


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def full_rank(support, grids):
    plan = O.build_plan(support, grids)
    c = np.random.default_rng(0).standard_normal(len(support))
    x, its, acond = O.lstsq_lsqr(plan, O.sparse_A(plan) @ c, iter_lim=8000)
    err = O.max_rel_err(x, c)
    log(f"  K={len(grids)}: recovery max_rel {err:.1e} in {its} LSQR iterations "
        f"(condition estimate {acond:.1f})")
    return err <= 1e-10


def main():
    t0 = time.time()
    big = W.config4(min_grids=96)                # the draw stream, long enough
    S = big.support
    k_rule = W.config4(min_grids=1).K            # the 3x-oversampling stop alone
    k = k_rule
    while not O.fold_injective(S, big.grids[:k]):
        k += 1
    log(f"oversampling stop at K={k_rule}; per-dimension folds separate at K={k}")
    if k < 2:
        k = 2
    lo = k - 1
    if not full_rank(S, big.grids[:k]):
        lo, k = k, 2 * k
        while not full_rank(S, big.grids[:k]):
            lo, k = k, 2 * k
        while k - lo > 1:                         # smallest full-rank count
            mid = (lo + k) // 2
            if full_rank(S, big.grids[:mid]):
                k = mid
            else:
                lo = mid
    prob = W.config4(min_grids=k)
    assert prob.K == k and np.array_equal(prob.grids, big.grids[:k])
    log(f"K={k}, {prob.total_points} samples; sampling and DCT")
    plan = O.build_plan(prob.support, prob.grids)
    b = np.empty(plan.M)
    for l, g in enumerate(prob.grids):          # one grid at a time (up to ~4e8 points)
        t = O.dct_grid(O.sample_function(prob.family, prob.params, g), g)
        r0, r1 = plan.rows_of_grid(l)
        b[r0:r1] = t[plan.bin_id[r0:r1]]
        del t
        log(f"  grid {l}: {W.grid_points(g)} points")
    log(f"M={plan.M}; LSQR")
    c, its, acond = O.lstsq_lsqr(plan, b, tol=1e-16, iter_lim=20000)
    g = O.normal_residual(plan, b, c)
    gb = O.sparse_A(plan).T @ b
    np.save(OUT_C, c)
    meta = {"K": int(k), "total_points": int(prob.total_points), "rows": int(plan.M),
            "n_support": int(plan.n), "lsqr_iterations": its,
            "lsqr_condition_estimate": acond,
            "rel_normal_residual": float(np.linalg.norm(g) / np.linalg.norm(gb)),
            "max_abs_coeff": float(np.max(np.abs(c))), "seconds": time.time() - t0}
    with open(OUT_META, "w") as fh:
        json.dump(meta, fh, indent=1)
    log(json.dumps(meta))


if __name__ == "__main__":
    main()
