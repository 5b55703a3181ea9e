"""Grid-count selection (Alg. 2) for the serving pool, run with the oracle,
once; writes tests/golden/serving_extra_grids.json.

For every job, further grids are drawn by the job's own rule from its own
stream; the smallest number m of them for which the stacked system has full
column rank is found by bisection (rank only grows as grids are appended).
Full rank is decided as for the batched workload: LSQR from zero recovers a
random polynomial on the job's support exactly (max-relative 1e-10) when,
and only when, A has full column rank.

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_serving_pool.py
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "serving_extra_grids.json")
SEED = 4
MAX_EXTRA = 4096


def full_rank(support, grids):
    plan = O.build_plan(support, grids)
    c = np.random.default_rng(0).standard_normal(len(support))
    x, its, _ = O.lstsq_lsqr(plan, O.sparse_A(plan) @ c, iter_lim=6000)
    return O.max_rel_err(x, c) <= 1e-10


def select(i):
    p = W.serving_pool(SEED)[i]
    rng = np.random.default_rng([SEED, 1000 + i])
    more = [W.serving_extra_grid(p, rng) for _ in range(MAX_EXTRA)]

    def ok(m):
        g = p.grids if m == 0 else np.concatenate([p.grids, np.array(more[:m], dtype=np.int32)])
        return O.fold_injective(p.support, g) and full_rank(p.support, g)

    if ok(0):
        return i, 0
    lo, hi = 0, 1
    while not ok(hi):                  # exponential search for a sufficient count
        lo, hi = hi, 2 * hi
        if hi > MAX_EXTRA:
            raise RuntimeError(f"job {i}: no full rank within {MAX_EXTRA} extra grids")
    while hi - lo > 1:                 # smallest m with full rank
        mid = (lo + hi) // 2
        if ok(mid):
            hi = mid
        else:
            lo = mid
    return i, hi


def main():
    t0 = time.time()
    n = len(W.serving_pool(SEED))
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        res = dict(ex.map(select, range(n)))
    extra = {str(i): m for i, m in sorted(res.items()) if m > 0}
    with open(OUT, "w") as fh:
        json.dump({"seed": SEED, "extra_grids": extra, "seconds": time.time() - t0}, fh, indent=1)
    print(open(OUT).read())


if __name__ == "__main__":
    main()
