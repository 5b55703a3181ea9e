"""Grid-count selection (Alg. 2) for the serving pool, run with the oracle,
once; writes tests/golden/serving_extra_grids.json.

Jobs of the D=2, D=6 and batched kinds: further grids are drawn by the
job's own rule from its own stream, and the smallest number m of them for
which the stacked system has full column rank is found by exponential search
and bisection (rank only grows as grids are appended).  The D=20 jobs share
one L-grid (workloads.d20_grids), which is checked the same way.  Full rank is decided as for
the batched workload: LSQR from zero recovers a random coefficient vector on
the job's support exactly (max-relative 1e-10) when, and only when, A has
full column rank.  Results are written as they come (a rerun resumes).

Calls only the oracle and the seeded input generators.  Run from the
repository root:  python tests/golden/make_serving_pool.py
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "serving_extra_grids.json")
PARTIAL = OUT + ".partial"
SEED = 4
MAX_EXTRA = 4096


def full_rank(support, grids, iter_lim):
    if not O.fold_injective(support, grids):
        return False
    plan = O.build_plan(support, grids)
    c = np.random.default_rng(0).standard_normal(len(support))
    x, its, _ = O.lstsq_lsqr(plan, O.sparse_A(plan) @ c, iter_lim=iter_lim)
    return O.max_rel_err(x, c) <= 1e-10


def smallest(ok, lo):
    """Smallest m >= lo with ok(m), for ok monotone in m."""
    if ok(lo):
        return lo
    a, b = lo, max(2 * lo, lo + 1)
    while not ok(b):
        a, b = b, 2 * b
        if b > MAX_EXTRA + lo:
            raise RuntimeError("no full rank within the search limit")
    while b - a > 1:
        mid = (a + b) // 2
        if ok(mid):
            b = mid
        else:
            a = mid
    return b


def select_job(i):
    p = W.serving_pool(SEED)[i]
    rng = np.random.default_rng([SEED, 1000 + i])
    more = [W.serving_extra_grid(p, rng) for _ in range(MAX_EXTRA)]

    def ok(m):
        g = p.grids if m == 0 else np.concatenate([p.grids, np.array(more[:m], dtype=np.int32)])
        return full_rank(p.support, g, 6000)

    return f"job:{i}", smallest(ok, 0)


def select_d20():
    """The shared D=20 L-grid must be full rank as it stands; returns the
    LSQR iterations its recovery took."""
    S = W.total_degree_support(20, 2)
    g = W.d20_grids(SEED)
    plan = O.build_plan(S, g)
    c = np.random.default_rng(0).standard_normal(len(S))
    x, its, acond = O.lstsq_lsqr(plan, O.sparse_A(plan) @ c, iter_lim=40000)
    err = O.max_rel_err(x, c)
    if not (O.fold_injective(S, g) and err <= 1e-10):
        raise RuntimeError(f"shared D=20 L-grid not full rank (recovery {err:.1e})")
    return "d20", {"grids": int(len(g)), "lsqr_iterations": int(its),
                   "lsqr_condition_estimate": float(acond), "recovery_max_rel": err}


def main():
    t0 = time.time()
    done = {}
    if os.path.exists(PARTIAL):
        with open(PARTIAL) as fh:
            done = json.load(fh)
    kinds = W.SERVING_TYPES
    n = 16 * len(kinds)
    todo = [i for i in range(n) if kinds[i % len(kinds)] != "D20_d2" and f"job:{i}" not in done]
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        futs = [ex.submit(select_d20)] if "d20" not in done else []
        futs += [ex.submit(select_job, i) for i in todo]
        for f in as_completed(futs):
            key, m = f.result()
            done[key] = m
            with open(PARTIAL, "w") as fh:
                json.dump(done, fh)
            print(f"[{time.time() - t0:7.0f}s] {key}: {m}", flush=True)
    extra = {k.split(":")[1]: m for k, m in sorted(done.items()) if k.startswith("job:") and m > 0}
    with open(OUT, "w") as fh:
        json.dump({"seed": SEED, "extra_grids": extra, "d20": done["d20"],
                   "seconds": time.time() - t0}, fh, indent=1)
    os.remove(PARTIAL)
    print(open(OUT).read())


if __name__ == "__main__":
    main()
